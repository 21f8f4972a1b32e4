// Hopping term for several right-hand sides per block with the links staged
// in LDS once per block (HOP_MULTI).  The operator is that of hop.hip
// (Sec. 2.3, even-odd blocks of Sec. 5.3.3):
//   out(x) = alpha x_add(x) + beta * H in (x),
//   H in (x) = -1/2 sum_mu [ (1 - g_mu) U_R(x,mu) in(x+mu) + (1 + g_mu) U_R(x-mu,mu)^+ in(x-mu) ].
//
// Layout of the work.  A block covers a tile of TS sites and K right-hand
// sides, one wavefront per right-hand side.  For d_R >= 4 (even) the d_R
// colour rows of a site are split over two lanes, lanes 0..31 holding rows
// 0..d/2-1 and lanes 32..63 rows d/2..d-1 of the same 32 sites (TS = 32);
// otherwise one lane holds all rows (TS = 64).  Per hop:
//   * the block loads the tile's d_R^2 link entries once, coalesced, into
//     an LDS buffer (double buffered: the entries of the next hop are loaded
//     into registers while this hop computes and written after it);
//   * every lane loads the colours of its row group of its own right-hand
//     side's neighbour spinor and spin-projects them ((1 -+ g_mu) psi =
//     [h; -+ e_mu^+ h], two colour vectors instead of four); the two lanes
//     of a site swap halves (v_permlane32_swap), so each holds the full
//     projected two-spinor;
//   * every lane applies its rows of U (or of U^+ for the backward hop),
//     read from LDS, to both projected components and reconstructs the
//     lower spin half.
// A link entry is read from HBM once per block and from LDS by the K
// wavefronts; per output site and rhs the LDS reads are d_R^2 entries per hop
// (half of them per lane), against 2 d_R projected components per rhs and
// per colour row in the colour-per-wavefront form of hop.hip.
#include "wd_common.h"
#include "wd_hop.h"
#include "wd_kernels.h"

namespace wd {

template <int D>
struct MrShape {
  static constexpr int LPS = (D % 2 == 0 && D >= 4) ? 2 : 1;   // lanes per (site, rhs)
  static constexpr int RPL = D / LPS;                           // colour rows per lane
  static constexpr int TS = 64 / LPS;                           // sites per tile
};

// Two-lane split: lanes 0..31 hold a quantity for colour k, lanes 32..63 the
// same quantity for colour k + RPL of the same 32 sites.  One
// v_permlane32_swap of v with itself swaps the upper half of its first
// operand with the lower half of its second, so that its first result holds
// colour k in every lane and its second colour k + RPL: no select by lane.
__device__ __forceinline__ void split_halves(float v, float &lo, float &hi) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v), false, false);
  lo = __int_as_float(r[0]);
  hi = __int_as_float(r[1]);
}
__device__ __forceinline__ void split_halves(double v, double &lo, double &hi) {
  const long long b = __double_as_longlong(v);
  const int b0 = (int)(b & 0xffffffffLL), b1 = (int)(b >> 32);
  const auto r0 = __builtin_amdgcn_permlane32_swap(b0, b0, false, false);
  const auto r1 = __builtin_amdgcn_permlane32_swap(b1, b1, false, false);
  lo = __longlong_as_double((long long)(((unsigned long long)(unsigned)r1[0] << 32) | (unsigned)r0[0]));
  hi = __longlong_as_double((long long)(((unsigned long long)(unsigned)r1[1] << 32) | (unsigned)r0[1]));
}
template <typename T>
__device__ __forceinline__ void split_halves(cplx<T> v, cplx<T> &lo, cplx<T> &hi) {
  split_halves(v.re, lo.re, hi.re);
  split_halves(v.im, lo.im, hi.im);
}

// Element off of the array at base: base is the same for every lane of the
// wavefront and the 32-bit offset is per lane, which selects global loads
// and stores with a scalar base address and a single VGPR offset.
template <typename V>
__device__ __forceinline__ const V *at(const V *base, uint32_t off) {
  return reinterpret_cast<const V *>(reinterpret_cast<const char *>(base) + off * (uint32_t)sizeof(V));
}
template <typename V>
__device__ __forceinline__ V *at(V *base, uint32_t off) {
  return reinterpret_cast<V *>(reinterpret_cast<char *>(base) + off * (uint32_t)sizeof(V));
}

// Per-block staging of the link entries of one hop.  The block's 64 K lanes
// cover ROWS = K LPS entry rows of the TS-site tile per pass: wavefront w
// stages rows LPS (w + p K) + rg, p < PER, at its own sites (the lane's
// row group rg and site are those it computes with).  Rows past d_R^2 (when
// ROWS does not divide it) reload the last rows into scratch rows of the LDS
// tile, so that no branch surrounds the loads.
template <int D, int K>
struct MrTile {
  static constexpr int LPS = MrShape<D>::LPS;
  static constexpr int TS = MrShape<D>::TS;
  static constexpr int NE = D * D;
  static constexpr int ROWS = K * LPS;
  static constexpr int PER = (NE + ROWS - 1) / ROWS;
  static constexpr int NEP = PER * ROWS;
};

template <int D, bool REAL, typename T, int K, int MU, bool BWD, bool NTL>
__device__ __forceinline__ void mr_load_links(typename LinkT<T, REAL>::type (&lr)[(MrTile<D, K>::PER)],
                                              const typename LinkT<T, REAL>::type *links, const Geom &g, int parity,
                                              int w, int rg, int is, const int (&nbb)[4]) {
  using M = MrTile<D, K>;
  const int lpar = BWD ? 1 - parity : parity;
  // backward hop: U(x - mu, mu) sits at the neighbour's index
  const uint32_t off = (uint32_t)(link_row(rg, g.stride) + link_site(D * D, g.stride, BWD ? nbb[MU] : is));
  const auto *lk = links + (size_t)(lpar * 4 + MU) * D * D * g.stride;
#pragma unroll
  for (int p = 0; p < M::PER; ++p) {
    const int eu = M::LPS * (w + p * K);
    const int ec = eu < M::NE - M::LPS ? eu : M::NE - M::LPS;
    lr[p] = ld_stream<NTL>(at(lk + link_row(ec, g.stride), off));
  }
}

template <int D, typename L, int K>
__device__ __forceinline__ void mr_store_links(L (*buf)[(MrShape<D>::TS)], const L (&lr)[(MrTile<D, K>::PER)], int w,
                                               int rg, int sl) {
  using M = MrTile<D, K>;
#pragma unroll
  for (int p = 0; p < M::PER; ++p) buf[M::LPS * (w + p * K) + rg][sl] = lr[p];
}

// Direct global -> LDS loads of the same entries (16-byte link entries: FP64
// complex).  A wavefront's lanes fill LPS consecutive rows of TS entries,
// i.e. 64 consecutive LDS elements starting at row LPS (w + p K), so each
// load is one global_load_lds_dwordx4 with a wave-uniform LDS base; nothing
// passes through registers.  Completion is awaited with vmcnt(0) before the
// barrier that publishes the tile.
template <int D, typename L, int K, int MU, bool BWD>
__device__ __forceinline__ void mr_dma_links(L (*buf)[(MrShape<D>::TS)], const L *links, const Geom &g, int parity,
                                             int w, int rg, int is, const int (&nbb)[4]) {
  static_assert(sizeof(L) == 16, "direct LDS loads of 16-byte entries");
  using M = MrTile<D, K>;
  const int lpar = BWD ? 1 - parity : parity;
  const uint32_t off = (uint32_t)(link_row(rg, g.stride) + link_site(D * D, g.stride, BWD ? nbb[MU] : is));
  const L *lk = links + (size_t)(lpar * 4 + MU) * D * D * g.stride;
#pragma unroll
  for (int p = 0; p < M::PER; ++p) {
    const int eu = M::LPS * (w + p * K);
    const int ec = eu < M::NE - M::LPS ? eu : M::NE - M::LPS;
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(at(lk + link_row(ec, g.stride), off)),
                                     (__attribute__((address_space(3))) void *)(&buf[eu][0]), 16, 0, 0);
  }
}

// Raw neighbour components of this lane's colour rows: p[s][k] = in(nb) of
// spin s, colour c0 + k (loaded one hop ahead of their use).
template <int D, typename T>
__device__ __forceinline__ void mr_load_spinor(cplx<T> (&p)[4][MrShape<D>::RPL], const cplx<T> *in, int stride,
                                               uint32_t roff, int nb) {
  constexpr int RPL = MrShape<D>::RPL;
  const uint32_t off = roff + (uint32_t)nb;
#pragma unroll
  for (int k = 0; k < RPL; ++k)
#pragma unroll
    for (int s = 0; s < 4; ++s) p[s][k] = *at(in + (size_t)(s * D + k) * stride, off);
}

// Spin projection of loaded components into slots 0 .. RPL - 1 of h0/h1.
template <int D, typename T, int MU, int SIG>
__device__ __forceinline__ void mr_project_loaded(cplx<T> (&h0)[D], cplx<T> (&h1)[D],
                                                  const cplx<T> (&p)[4][MrShape<D>::RPL]) {
  constexpr int RPL = MrShape<D>::RPL;
#pragma unroll
  for (int k = 0; k < RPL; ++k) {
    h0[k] = p[0][k] + ipow<PROJ_PH(MU, SIG, 0)>(p[2 + ECOL(MU, 0)][k]);
    h1[k] = p[1][k] + ipow<PROJ_PH(MU, SIG, 1)>(p[2 + ECOL(MU, 1)][k]);
  }
}

// Complete h0/h1 (own colours in slots 0 .. RPL - 1) to the full projected
// two-spinor in colour order (with two lanes per site; see split_halves).
template <int D, typename T>
__device__ __forceinline__ void mr_gather(cplx<T> (&h0)[D], cplx<T> (&h1)[D]) {
  constexpr int RPL = MrShape<D>::RPL;
  if constexpr (MrShape<D>::LPS == 2) {
#pragma unroll
    for (int k = RPL - 1; k >= 0; --k) {
      split_halves(h0[k], h0[k], h0[RPL + k]);
      split_halves(h1[k], h1[k], h1[RPL + k]);
    }
  }
}

// Apply rows a0 .. a0 + RPL - 1 of U (forward) or U^+ (backward), read from
// the LDS tile at site s, to both projected components and accumulate the
// four spin components.
template <int D, bool REAL, typename T, int MU, int SIG, bool BWD>
__device__ __forceinline__ void mr_compute(cplx<T> (&acc)[4][MrShape<D>::RPL], const cplx<T> (&h0)[D],
                                           const cplx<T> (&h1)[D],
                                           const typename LinkT<T, REAL>::type (*buf)[MrShape<D>::TS], int a0,
                                           int s) {
  constexpr int RPL = MrShape<D>::RPL;
#pragma unroll
  for (int k = 0; k < RPL; ++k) {
    const int a = a0 + k;
    cplx<T> chi[2] = {mk<T>(0, 0), mk<T>(0, 0)};
#pragma unroll
    for (int b = 0; b < D; ++b) {
      // forward: U_ab;  backward: (U^+)_ab = conj(U_ba)
      const auto u = buf[BWD ? b * D + a : a * D + b][s];
      chi[0] = link_mac(u, h0[b], chi[0], BWD);
      chi[1] = link_mac(u, h1[b], chi[1], BWD);
    }
    acc[0][k] = acc[0][k] + chi[0];
    acc[1][k] = acc[1][k] + chi[1];
    acc[2][k] = acc[2][k] + ipow<RECON_PH(MU, SIG, 0)>(chi[RECON_SRC(MU, 0)]);
    acc[3][k] = acc[3][k] + ipow<RECON_PH(MU, SIG, 1)>(chi[RECON_SRC(MU, 1)]);
  }
}

// Hop H = 2 mu + (backward) of the pipeline.  On entry the raw neighbour
// components of hop H are in registers (p) and its link tile is on its way
// to LDS buffer H & 1 (direct loads, or registers lr for other entry sizes).
//   wait for the tile, barrier (every wave has finished hop H - 1, the last
//   reader of buffer (H + 1) & 1);
//   start hop H + 1: its link tile towards buffer (H + 1) & 1, its raw
//   neighbour components into registers;
//   project and gather hop H, compute it from buffer H & 1;
//   (register staging) store hop H + 1's entries.
template <int D, bool REAL, typename T, int K, bool DAG, bool NTL, int H>
__device__ __forceinline__ void mr_step(cplx<T> (&acc)[4][(MrShape<D>::RPL)],
                                        typename LinkT<T, REAL>::type (*lbuf)[(MrTile<D, K>::NEP)][(MrShape<D>::TS)],
                                        typename LinkT<T, REAL>::type (&lr)[(MrTile<D, K>::PER)],
                                        cplx<T> (&p)[4][(MrShape<D>::RPL)],
                                        const typename LinkT<T, REAL>::type *links, const cplx<T> *in, const Geom &g,
                                        int parity, const int (&nbf)[4], const int (&nbb)[4], int w, int rg, int is,
                                        int sl, uint32_t roff) {
  using L = typename LinkT<T, REAL>::type;
  constexpr bool DMA = sizeof(L) == 16;
  constexpr int RPL = MrShape<D>::RPL;
  constexpr int MU = H / 2;
  constexpr bool BWD = (H & 1) != 0;
  constexpr int SF = DAG ? -1 : 1;   // forward hop: 1 - g_mu (dagger: 1 + g_mu)
  constexpr int SIG = BWD ? -SF : SF;
  constexpr int MU1 = (H + 1) / 2;
  constexpr bool BWD1 = ((H + 1) & 1) != 0;
  if constexpr (DMA) __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this hop's tile has landed
  __syncthreads();
  cplx<T> h0[D], h1[D];
  mr_project_loaded<D, T, MU, SIG>(h0, h1, p);
  if constexpr (H < 7) {
    if constexpr (DMA)
      mr_dma_links<D, L, K, MU1, BWD1>(lbuf[(H + 1) & 1], links, g, parity, w, rg, is, nbb);
    else
      mr_load_links<D, REAL, T, K, MU1, BWD1, NTL>(lr, links, g, parity, w, rg, is, nbb);
    mr_load_spinor<D, T>(p, in, g.stride, roff, BWD1 ? nbb[MU1] : nbf[MU1]);
  }
  mr_gather<D, T>(h0, h1);
  mr_compute<D, REAL, T, MU, SIG, BWD>(acc, h0, h1, lbuf[H & 1], rg * RPL, sl);
  if constexpr (H < 7 && !DMA) mr_store_links<D, L, K>(lbuf[(H + 1) & 1], lr, w, rg, sl);
}

template <int D, bool REAL, typename T, int K, bool DAG, bool NTL, int H = 0>
__device__ __forceinline__ void mr_steps(cplx<T> (&acc)[4][(MrShape<D>::RPL)],
                                         typename LinkT<T, REAL>::type (*lbuf)[(MrTile<D, K>::NEP)][(MrShape<D>::TS)],
                                         typename LinkT<T, REAL>::type (&lr)[(MrTile<D, K>::PER)],
                                         cplx<T> (&p)[4][(MrShape<D>::RPL)],
                                         const typename LinkT<T, REAL>::type *links, const cplx<T> *in,
                                         const Geom &g, int parity, const int (&nbf)[4], const int (&nbb)[4], int w,
                                         int rg, int is, int sl, uint32_t roff) {
  if constexpr (H < 8) {
    mr_step<D, REAL, T, K, DAG, NTL, H>(acc, lbuf, lr, p, links, in, g, parity, nbf, nbb, w, rg, is, sl, roff);
    mr_steps<D, REAL, T, K, DAG, NTL, H + 1>(acc, lbuf, lr, p, links, in, g, parity, nbf, nbb, w, rg, is, sl, roff);
  }
}

// Work item = (tile, group of K right-hand sides), group fastest (the
// groups of a tile run back to back on one XCD and re-read the links from its
// L2).  NTL: links read with streaming loads (one group: no block re-reads).
template <int D, bool REAL, typename T, bool DAG, int K, bool NTL, int W>
__global__ __launch_bounds__(64 * K) __attribute__((amdgpu_waves_per_eu(W))) void k_hop_mr(HopArgs a) {
  using L = typename LinkT<T, REAL>::type;
  constexpr int LPS = MrShape<D>::LPS, RPL = MrShape<D>::RPL, TS = MrShape<D>::TS;
  __shared__ L lbuf[2][MrTile<D, K>::NEP][TS];
  const int ngroups = a.ngroups;
  const int wi = tile_of_block(blockIdx.x, a.ntiles * ngroups, a.xcd_remap);
  const int q = wi / ngroups, grp = wi - q * ngroups;
  const int tile = tile_order(q, a);
  const int l = lattice_of_tile(a, tile);
  const Geom g = a.lat[l].g;
  const int tl = tile - a.lat[l].tile0;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wavefront = right-hand side
  const int rg = LPS == 2 ? lane >> 5 : 0;           // row group of this lane
  const int sl = LPS == 2 ? lane & 31 : lane;        // site within the tile
  const int i = tl * TS + sl;
  const bool valid = i < g.Vh;
  const int is = valid ? i : g.Vh - 1;   // lanes past the end recompute the last site, store into the padding
  const int r = grp * K + w;             // right-hand side of this wavefront
  const size_t fbase = (size_t)a.lat[l].soff + (size_t)r * 4 * D * g.stride;
  const cplx<T> *in = static_cast<const cplx<T> *>(a.in) + fbase;
  const L *links = static_cast<const L *>(a.links) + a.lat[l].loff;
  const uint32_t roff = (uint32_t)(rg * RPL * g.stride);
  int t, x, y, z;
  cb_coords(g, is, a.parity, t, x, y, z);
  int nbf[4], nbb[4];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    nbf[mu] = nb_index(g, t, x, y, z, mu, 1);
    nbb[mu] = nb_index(g, t, x, y, z, mu, 0);
  }
  cplx<T> acc[4][RPL];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int k = 0; k < RPL; ++k) acc[s][k] = mk<T>(0, 0);
  L lr[(MrTile<D, K>::PER)];
  cplx<T> p[4][RPL];
  if constexpr (sizeof(L) == 16) {
    mr_dma_links<D, L, K, 0, false>(lbuf[0], links, g, a.parity, w, rg, is, nbb);
  } else {
    mr_load_links<D, REAL, T, K, 0, false, NTL>(lr, links, g, a.parity, w, rg, is, nbb);
    mr_store_links<D, L, K>(lbuf[0], lr, w, rg, sl);
  }
  mr_load_spinor<D, T>(p, in, g.stride, roff, nbf[0]);
  mr_steps<D, REAL, T, K, DAG, NTL>(acc, lbuf, lr, p, links, in, g, a.parity, nbf, nbb, w, rg, is, sl, roff);
  const T cb = (T)(-0.5 * a.beta), ca = (T)a.alpha;
  cplx<T> *out = static_cast<cplx<T> *>(a.out) + fbase;
  const uint32_t ooff = roff + (uint32_t)i;   // i < stride: lanes past the end write the padding
  double nrm = 0.0;
  // two straight-line epilogues (see hop.hip); output and x_add streamed
  if (a.xadd) {
    const cplx<T> *xa = static_cast<const cplx<T> *>(a.xadd) + fbase;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const size_t row = (size_t)(s * D + k) * g.stride;
        cplx<T> v = cb * acc[s][k];
        const cplx<T> xv = ld_nt(at(xa + row, ooff));
        v.re = fma(ca, xv.re, v.re);
        v.im = fma(ca, xv.im, v.im);
        st_nt(at(out + row, ooff), v);
        nrm += (double)v.re * v.re + (double)v.im * v.im;
      }
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const size_t row = (size_t)(s * D + k) * g.stride;
        const cplx<T> v = cb * acc[s][k];
        st_nt(at(out + row, ooff), v);
        nrm += (double)v.re * v.re + (double)v.im * v.im;
      }
  }
  if (a.partial) {
    // one wavefront = one right-hand side over the whole tile
    const double v = wave_sum(valid ? nrm : 0.0);
    if (lane == 0) a.partial[(size_t)(l * ngroups * K + r) * a.prow + tl] = v;
  }
}

// Waves per SIMD asked of the register allocator, per (d_R, precision).
constexpr int mr_waves(int D, bool dbl) { return dbl ? (D <= 4 ? 3 : 2) : (D <= 4 ? 6 : 4); }

template <int D, bool REAL, typename T, bool DAG, int K>
static hipError_t launch_mr_k(HopArgs a, int nrhs, hipStream_t st, Counts *counts, int *prow) {
  set_tiles(a, MrShape<D>::TS, nrhs, counts, prow);
  a.ngroups = nrhs / K;
  dim3 grid(a.ntiles * a.ngroups);
  constexpr int W = mr_waves(D, sizeof(T) == 8);
  if (a.ngroups == 1) hipLaunchKernelGGL((k_hop_mr<D, REAL, T, DAG, K, true, W>), grid, dim3(64 * K), 0, st, a);
  else hipLaunchKernelGGL((k_hop_mr<D, REAL, T, DAG, K, false, W>), grid, dim3(64 * K), 0, st, a);
  return hipGetLastError();
}

template <int D, bool REAL, typename T, bool DAG>
static hipError_t launch_mr_t(const HopArgs &a, int nrhs, int nr, hipStream_t st, Counts *c, int *prow) {
  switch (nr) {
    case 1: return launch_mr_k<D, REAL, T, DAG, 1>(a, nrhs, st, c, prow);
    case 2: return launch_mr_k<D, REAL, T, DAG, 2>(a, nrhs, st, c, prow);
    case 3: return launch_mr_k<D, REAL, T, DAG, 3>(a, nrhs, st, c, prow);
    case 4: return launch_mr_k<D, REAL, T, DAG, 4>(a, nrhs, st, c, prow);
    case 6: return launch_mr_k<D, REAL, T, DAG, 6>(a, nrhs, st, c, prow);
    case 12: return launch_mr_k<D, REAL, T, DAG, 12>(a, nrhs, st, c, prow);
  }
  return hipErrorInvalidValue;
}

template <int D, bool REAL>
static hipError_t launch_mr_d(const HopArgs &a, int prec, int dagger, int nrhs, int nr, hipStream_t st, Counts *c,
                              int *prow) {
  if (prec == 0)
    return dagger ? launch_mr_t<D, REAL, double, true>(a, nrhs, nr, st, c, prow)
                  : launch_mr_t<D, REAL, double, false>(a, nrhs, nr, st, c, prow);
  return dagger ? launch_mr_t<D, REAL, float, true>(a, nrhs, nr, st, c, prow)
                : launch_mr_t<D, REAL, float, false>(a, nrhs, nr, st, c, prow);
}

bool hop_mr_ok(int d, int real) { return real ? d == 3 : (d == 3 || d == 6); }

hipError_t launch_hop_mr(const HopArgs &a, int d, int real, int prec, int dagger, int nrhs, int nr, hipStream_t st,
                         Counts *counts, int *prow) {
  if (nr < 1 || nrhs % nr) return hipErrorInvalidValue;
  if (real) {
    if (d == 3) return launch_mr_d<3, true>(a, prec, dagger, nrhs, nr, st, counts, prow);
  } else {
    if (d == 3) return launch_mr_d<3, false>(a, prec, dagger, nrhs, nr, st, counts, prow);
    if (d == 6) return launch_mr_d<6, false>(a, prec, dagger, nrhs, nr, st, counts, prow);
  }
  return hipErrorInvalidValue;
}

}  // namespace wd
