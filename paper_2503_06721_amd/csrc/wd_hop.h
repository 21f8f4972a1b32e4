// Device and host helpers shared by the hopping-term kernels (hop.hip,
// hop_mr.hip): tile order, lattice lookup, link entry types and the tile
// bookkeeping of a launch.
#pragma once

#include "wd_common.h"
#include "wd_kernels.h"

namespace wd {

// ------------------------------------------------------------ tile mapping
// Blocks are dispatched round-robin over the 8 XCDs of the chip.  With
// remapping, XCD k receives a contiguous range of tiles, so the neighbours a
// tile reads (mostly in nearby tiles) stay in that XCD's L2.
__device__ __forceinline__ int tile_of_block(int b, int ntiles, int remap) {
  if (!remap) return b;
  const int q = ntiles >> 3, rmd = ntiles & 7;
  const int x = b & 7, j = b >> 3;
  return x * q + (x < rmd ? x : rmd) + j;
}

// Processing order of tiles.  With tb > 0 the tiles (each tiles_per_tx
// tiles cover one (t, x) row of Y*Z lexicographic sites) are visited in the
// order (t-block of tb slices, x, t within the block, tile within the row):
// t-neighbours are then tiles_per_tx tiles apart instead of a whole t-slice,
// so they are still in L2 when read.  tb = 0: lexicographic order.
// With tb < 0 the slices are taken in chunks of -tb with t fastest:
// (chunk, x, tile within the row, t within the chunk), so consecutive work
// items are t-neighbours and the tiles of a (t, x) row follow each other
// -tb items apart (for work items holding many right-hand sides, whose
// neighbourhoods would not stay in L2 across a whole row of tiles).
__device__ __forceinline__ int tile_order(int q, const HopArgs &a) {
  if (a.tblock == 0) return q;
  if (a.tblock < 0) {
    const int nb = a.tiles_per_tx, tc = -a.tblock, X = a.lat[0].g.X;
    const int per_c = X * nb * tc;
    const int ci = q / per_c;
    int r = q - ci * per_c;
    const int x = r / (nb * tc);
    r -= x * nb * tc;
    const int yb = r / tc;
    const int tin = r - yb * tc;
    return ((ci * tc + tin) * X + x) * nb + yb;
  }
  const int nb = a.tiles_per_tx, tb = a.tblock, X = a.lat[0].g.X;
  const int per_tb = X * tb * nb;
  const int tbi = q / per_tb;
  int r = q - tbi * per_tb;
  const int x = r / (tb * nb);
  r -= x * tb * nb;
  const int tin = r / nb;
  const int yb = r - tin * nb;
  return ((tbi * tb + tin) * X + x) * nb + yb;
}

// Lattice of a global tile index (the launch covers the tiles of every
// lattice of a batch back to back).
__device__ __forceinline__ int lattice_of_tile(const HopArgs &a, int tile) {
  int l = 0;
  while (l + 1 < a.nlat && tile >= a.lat[l + 1].tile0) ++l;
  return l;
}

template <typename T, bool REAL>
struct LinkT {
  using type = cplx<T>;
};
template <typename T>
struct LinkT<T, true> {
  using type = T;
};

template <typename T>
__device__ __forceinline__ cplx<T> link_mac(cplx<T> u, cplx<T> h, cplx<T> acc, bool conjugate) {
  return conjugate ? cfma_conj(u, h, acc) : cfma(u, h, acc);
}
template <typename T>
__device__ __forceinline__ cplx<T> link_mac(T u, cplx<T> h, cplx<T> acc, bool) {
  return rfma(u, h, acc);
}

// Tile bookkeeping of a launch with tiles of ts sites: per-lattice tile
// ranges, the partial-sum row length and counts, and the t-blocked order
// (single lattices only: tiles_per_tx is the number of tiles covering one
// (t, x) row of Y*Z sites; the order falls back to lexicographic if tiles
// straddle rows or tb does not divide T).
inline void set_tiles(HopArgs &a, int ts, int nrhs, Counts *counts, int *prow) {
  int tot = 0, mx = 0;
  for (int l = 0; l < a.nlat; ++l) {
    const int n = (a.lat[l].g.Vh + ts - 1) / ts;
    a.lat[l].tile0 = tot;
    a.lat[l].ntiles = n;
    tot += n;
    mx = n > mx ? n : mx;
    for (int r = 0; r < nrhs && l * nrhs + r < MAXSYS; ++r) counts->n[l * nrhs + r] = n;
  }
  a.ntiles = tot;
  a.prow = mx;
  *prow = mx;
  const Geom &g = a.lat[0].g;
  const int lex_per_tile = 2 * ts, rowl = g.Y * g.Z;
  const int tbabs = a.tblock < 0 ? -a.tblock : a.tblock;
  if (a.nlat == 1 && tbabs > 0 && rowl % lex_per_tile == 0 && g.T % tbabs == 0) {
    a.tiles_per_tx = rowl / lex_per_tile;
  } else {
    a.tblock = 0;
    a.tiles_per_tx = 0;
  }
}

}  // namespace wd
