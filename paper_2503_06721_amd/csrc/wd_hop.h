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
// With tb = -(10 bx + by) < 0 (for work items holding many right-hand
// sides, whose per-site inputs are too large for a whole row of tiles to
// stay in L2): the lattice is cut into sub-lattices of bx x-rows by by tiles
// of a (t, x) row, and each sub-lattice is swept along t, (sub-lattice, t,
// x within it, tile within it), so that a tile's t-neighbours are bx by
// items away and its x-neighbours inside the sub-lattice by items away.
// With the XCD remap each XCD sweeps a contiguous set of sub-lattices.
__device__ __forceinline__ int tile_order(int q, const HopArgs &a) {
  if (a.tblock == 0) return q;
  if (a.tblock < 0) {
    const int code = -a.tblock, bx = code / 10, by = code % 10;
    const int nb = a.tiles_per_tx, X = a.lat[0].g.X, T = a.lat[0].g.T;
    const int per_sub = T * bx * by;
    const int sub = q / per_sub;
    int r = q - sub * per_sub;
    const int t = r / (bx * by);
    r -= t * bx * by;
    const int xi = r / by, yi = r - xi * by;
    const int nyb = nb / by;
    const int xs = sub / nyb, ys = sub - xs * nyb;
    return (t * X + xs * bx + xi) * nb + ys * by + yi;
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
// ranges, the partial-sum row length and counts, and the t-blocked or
// sub-lattice order (single lattices only: tiles_per_tx is the number of
// tiles covering one (t, x) row of Y*Z sites; the order falls back to
// lexicographic if tiles straddle rows, tb > 0 does not divide T, or bx, by
// of tb < 0 are zero or do not divide X and the tiles of a row).
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
  const int nb = rowl / lex_per_tile;
  bool ok = a.nlat == 1 && a.tblock != 0 && rowl % lex_per_tile == 0;
  if (a.tblock > 0) {
    ok = ok && g.T % a.tblock == 0;
  } else if (a.tblock < 0) {
    const int bx = (-a.tblock) / 10, by = (-a.tblock) % 10;
    ok = ok && bx > 0 && by > 0 && g.X % bx == 0 && nb % by == 0;
  }
  if (ok) {
    a.tiles_per_tx = nb;
  } else {
    a.tblock = 0;
    a.tiles_per_tx = 0;
  }
}

}  // namespace wd
