// Hopping term of the Wilson-Dirac operator on packed half spinors
// (Sec. 2.3; even-odd blocks of Sec. 5.3.3):
//   out(x) = alpha x_add(x) + beta * H in (x),
//   H in (x) = -1/2 sum_mu [ (1 - g_mu) U_R(x,mu) in(x+mu) + (1 + g_mu) U_R(x-mu,mu)^+ in(x-mu) ],
// for the sites x of one parity.  The dagger form swaps the two projectors.
//
// Two kernels compute the same thing:
//  * k_hop_sp: one lane per output site; the whole spinor accumulator, the
//    projected neighbour two-spinor and one link row live in registers.
//    Good for small d_R.
//  * k_hop_cs: one wavefront per colour row a of a tile of 64 consecutive
//    sites (block = 64 * d_R lanes).  Lane (site, a) loads colour component a
//    of the neighbour spinor, spin-projects it to two complex numbers and
//    publishes them in LDS; after one barrier every lane reads the full
//    projected two-spinor of its site and applies row a of U (or column a of
//    U^+), which it loads itself -- each link entry is read exactly once, by
//    one lane, coalesced across the 64 sites of the wavefront.  Register use
//    no longer grows with d_R^2, which is what limits the site-parallel form
//    for large representations.
#include "wd_common.h"
#include "wd_hop.h"
#include "wd_kernels.h"
#include "wd_rep.h"

namespace wd {

// ------------------------------------------------------- site-parallel form
template <int D, bool REAL, typename T, int MU, int SIG, bool BWD, bool NTL>
__device__ __forceinline__ void sp_dir(cplx<T> (&acc)[4][D], const cplx<T> *__restrict__ in, int stride, int nb,
                                       const typename LinkT<T, REAL>::type *__restrict__ lk, int lsite) {
  cplx<T> h[2][D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    cplx<T> p[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) p[s] = in[(size_t)(s * D + c) * stride + nb];
    h[0][c] = p[0] + ipow<PROJ_PH(MU, SIG, 0)>(p[2 + ECOL(MU, 0)]);
    h[1][c] = p[1] + ipow<PROJ_PH(MU, SIG, 1)>(p[2 + ECOL(MU, 1)]);
    // FP64, large d_R: at most half of the spinor loads in flight
    if constexpr (D >= 6 && sizeof(T) == 8)
      if (2 * c + 2 == D) __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    cplx<T> chi[2] = {mk<T>(0, 0), mk<T>(0, 0)};
#pragma unroll
    for (int b = 0; b < D; ++b) {
      // forward: U_ab;  backward: (U^+)_ab = conj(U_ba)
      const auto u = ld_stream<NTL>(lk + link_row(BWD ? b * D + a : a * D + b, stride) + link_site(D * D, stride, lsite));
      chi[0] = link_mac(u, h[0][b], chi[0], BWD);
      chi[1] = link_mac(u, h[1][b], chi[1], BWD);
    }
    acc[0][a] = acc[0][a] + chi[0];
    acc[1][a] = acc[1][a] + chi[1];
    acc[2][a] = acc[2][a] + ipow<RECON_PH(MU, SIG, 0)>(chi[RECON_SRC(MU, 0)]);
    acc[3][a] = acc[3][a] + ipow<RECON_PH(MU, SIG, 1)>(chi[RECON_SRC(MU, 1)]);
    // large d_R: keep each row's link loads next to their use, so that the
    // d_R^2 entries of a link are not all live at once
    if constexpr (D >= 6) __builtin_amdgcn_sched_barrier(0);
  }
  __builtin_amdgcn_sched_barrier(0);
}

template <int D, bool REAL, typename T, bool DAG, int MU, bool NTL>
__device__ __forceinline__ void sp_mu(cplx<T> (&acc)[4][D], const Geom &g, int parity,
                                      const typename LinkT<T, REAL>::type *links, const cplx<T> *in, int i, int t,
                                      int x, int y, int z) {
  const size_t lstride = (size_t)D * D * g.stride;
  constexpr int SF = DAG ? -1 : 1;   // forward hop: 1 - g_mu (dagger: 1 + g_mu)
  const int nbf = nb_index(g, t, x, y, z, MU, 1);
  sp_dir<D, REAL, T, MU, SF, false, NTL>(acc, in, g.stride, nbf, links + (size_t)(parity * 4 + MU) * lstride, i);
  const int nbb = nb_index(g, t, x, y, z, MU, 0);
  sp_dir<D, REAL, T, MU, -SF, true, NTL>(acc, in, g.stride, nbb, links + (size_t)((1 - parity) * 4 + MU) * lstride,
                                    nbb);
}

// Lanes of a site-parallel block: RL = 1: 256 sites of one right-hand side.
// RL = 4: 64 sites x 4 right-hand sides; in each wavefront 16 consecutive
// sites x 4 rhs (rhs = lane / 16), so the 4 lanes of a site load the same
// link entries (one memory request serves them) and each rhs reads 16
// consecutive spinor elements.  Work item = (tile, group of RL rhs), group
// fastest.  NTL: links read with streaming loads (set when the launch has a
// single group, so no other block re-reads them).
template <int D, bool REAL, typename T, bool DAG, bool NTL, int RL, int W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W))) void k_hop_sp(HopArgs a) {
  using L = typename LinkT<T, REAL>::type;
  constexpr int TS = 256 / RL;   // sites per tile
  const int ngroups = a.ngroups;
  const int w = tile_of_block(blockIdx.x, a.ntiles * ngroups, a.xcd_remap);
  const int q = w / ngroups, grp = w - q * ngroups;
  const int tile = tile_order(q, a);
  const int l = lattice_of_tile(a, tile);
  const Geom g = a.lat[l].g;
  const int tl = tile - a.lat[l].tile0;   // tile within its lattice
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int sl = RL == 1 ? (int)threadIdx.x : wv * 16 + (lane & 15);
  const int rk = RL == 1 ? 0 : lane >> 4;   // rhs of this lane within the group
  const int i = tl * TS + sl;
  const int r = grp * RL + rk;
  const int sys0 = l * ngroups * RL + grp * RL;
  const size_t rstride = (size_t)4 * D * g.stride;
  const size_t fbase = (size_t)a.lat[l].soff + r * rstride;
  const L *links = static_cast<const L *>(a.links) + a.lat[l].loff;
  // Lanes past the last site recompute the last site and store into the row
  // padding (stride is a multiple of 256), so that no branch separates the
  // arithmetic from its stores.
  const bool valid = i < g.Vh;
  const int is = valid ? i : g.Vh - 1;
  const cplx<T> *in = static_cast<const cplx<T> *>(a.in) + fbase;
  int t, x, y, z;
  cb_coords(g, is, a.parity, t, x, y, z);
  cplx<T> acc[4][D];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < D; ++c) acc[s][c] = mk<T>(0, 0);
  sp_mu<D, REAL, T, DAG, 0, NTL>(acc, g, a.parity, links, in, is, t, x, y, z);
  sp_mu<D, REAL, T, DAG, 1, NTL>(acc, g, a.parity, links, in, is, t, x, y, z);
  sp_mu<D, REAL, T, DAG, 2, NTL>(acc, g, a.parity, links, in, is, t, x, y, z);
  sp_mu<D, REAL, T, DAG, 3, NTL>(acc, g, a.parity, links, in, is, t, x, y, z);
  cplx<T> *out = static_cast<cplx<T> *>(a.out) + fbase;
  const T cb = (T)(-0.5 * a.beta), ca = (T)a.alpha;
  double nrm = 0.0;
  // Two straight-line epilogues: every accumulator is used on both paths.
  // The output and x_add are streamed (each element is touched once).
  if (a.xadd) {
    const cplx<T> *xa = static_cast<const cplx<T> *>(a.xadd) + fbase;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const size_t o = (size_t)(s * D + c) * g.stride + i;
        cplx<T> v = cb * acc[s][c];
        const cplx<T> xv = ld_nt(xa + o);
        v.re = fma(ca, xv.re, v.re);
        v.im = fma(ca, xv.im, v.im);
        st_nt(out + o, v);
        nrm += (double)v.re * v.re + (double)v.im * v.im;
      }
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const size_t o = (size_t)(s * D + c) * g.stride + i;
        const cplx<T> v = cb * acc[s][c];
        st_nt(out + o, v);
        nrm += (double)v.re * v.re + (double)v.im * v.im;
      }
  }
  if (a.partial) {
    __shared__ double sh[4][RL];
    double v = valid ? nrm : 0.0;
    if constexpr (RL == 1) {
      v = block_sum(v, &sh[0][0]);
      if (threadIdx.x == 0) a.partial[(size_t)sys0 * a.prow + tl] = v;
    } else {
      // sum over the 16 sites of each rhs in the wave, then over the waves
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      __syncthreads();
      if ((lane & 15) == 0) sh[wv][rk] = v;
      __syncthreads();
      if (threadIdx.x < RL) {
        const double s4 = ((sh[0][threadIdx.x] + sh[1][threadIdx.x]) + sh[2][threadIdx.x]) + sh[3][threadIdx.x];
        a.partial[(size_t)(sys0 + threadIdx.x) * a.prow + tl] = s4;
      }
    }
  }
}

// ------------------------------------------------------ colour-split form
// Stage: this lane's link entries (row `row` of U for a forward hop, column
// `row` of U for a backward hop, whose U^+ row is the conjugated column) and
// colour component `row` of the neighbour spinor, spin-projected into LDS.
//
// Compact form (FLY = 2 SYM, 3 2AS): the entries are rebuilt from the
// fundamental link, (U_R)_AB = n_A n_B (U_ac U_bd +- U_ad U_bc) with
// (a, b) = pair(A), (c, d) = pair(B), n = 1/sqrt2 on the diagonal pairs of
// SYM and 1 otherwise -- the closed forms of wd_rep.h.  Row `row` of U_R needs
// the fundamental rows a, b; column `row` (backward hop) the columns a, b.
// The boundary phase is stored as i U (the maps are quadratic).
template <int D, bool SYM>
constexpr int two_index_n() {
  return SYM ? (D == 3 ? 2 : D == 6 ? 3 : 4) : (D == 3 ? 3 : D == 6 ? 4 : 5);
}

// First and second index of two-index basis element A, at compile time.
constexpr int pair_first(int N, bool SYM, int A) {
  int a = 0, rem = A;
  while (rem >= (SYM ? N - a : N - 1 - a)) {
    rem -= SYM ? N - a : N - 1 - a;
    ++a;
  }
  return a;
}
constexpr int pair_second(int N, bool SYM, int A) {
  int a = 0, rem = A;
  while (rem >= (SYM ? N - a : N - 1 - a)) {
    rem -= SYM ? N - a : N - 1 - a;
    ++a;
  }
  return a + rem + (SYM ? 0 : 1);
}

// u[B] = nA nB (x[c] y[d] +- x[d] y[c]), (c, d) = pair(B), unrolled over B so
// that every register index is a constant.
template <int D, int N, bool SYM, typename T, int B = 0>
__device__ __forceinline__ void rebuild_row(cplx<T> (&u)[D], const cplx<T> (&xr)[N], const cplx<T> (&yr)[N], T na) {
  if constexpr (B < D) {
    constexpr int c = pair_first(N, SYM, B), d = pair_second(N, SYM, B);
    const T nn = (SYM && c == d) ? na * (T)0.70710678118654752440 : na;
    const cplx<T> p = cmul(xr[c], yr[d]), q = cmul(xr[d], yr[c]);
    u[B] = SYM ? mk<T>(nn * (p.re + q.re), nn * (p.im + q.im)) : mk<T>(nn * (p.re - q.re), nn * (p.im - q.im));
    rebuild_row<D, N, SYM, T, B + 1>(u, xr, yr, na);
  }
}

// Fundamental entries per link of the compact form FLY (1 for stored links),
// and the LDS rows that hold them: a multiple of D, so that every wave loads
// the same number of entries (the last rows repeat entry NE - 1 unused).
template <int D, int FLY>
constexpr int fly_entries() {
  return FLY ? two_index_n<D, FLY == 2>() * two_index_n<D, FLY == 2>() : 1;
}
template <int D, int FLY>
constexpr int fly_rows() {
  return FLY ? (fly_entries<D, FLY>() + D - 1) / D * D : 1;
}

// Stage one hop.  Stored links: this lane's row (forward) or column
// (backward) of U_R into registers u.  Compact form: the block's waves share
// the N^2 fundamental entries of each site's link, wave `row` loading entries
// row, row + D, ... into fl (each entry is read from memory once per site, not
// once per wave that needs it); u is rebuilt from fl after the barrier
// (cs_rebuild).  Then the spin projection of colour `row` of the neighbour
// spinor into hs.
template <int D, bool REAL, typename T, int MU, int SIG, bool BWD, int NR, bool NTL, int FLY>
__device__ __forceinline__ void cs_stage(typename LinkT<T, REAL>::type (&u)[D], cplx<T> (*hs)[2][D][64],
                                         cplx<T> (*fl)[64], const Geom &g, int parity,
                                         const typename LinkT<T, REAL>::type *links, const cplx<T> *flinks,
                                         const cplx<T> *in0, size_t rstride, int nb, int lsite, int row, int lane) {
  using L = typename LinkT<T, REAL>::type;
  const int stride = g.stride;
  const int lpar = BWD ? 1 - parity : parity;
  if constexpr (FLY != 0) {
    constexpr int NE = fly_entries<D, FLY>();
    const cplx<T> *fk = flinks + (size_t)(lpar * 4 + MU) * NE * stride + link_site(NE, stride, lsite);
#pragma unroll
    for (int j = 0; j < fly_rows<D, FLY>() / D; ++j) {
      const int e = row + j * D;
      fl[e][lane] = ld_stream<NTL>(fk + link_row(e < NE ? e : NE - 1, stride));
    }
  } else {
    const L *lk = links + (size_t)(lpar * 4 + MU) * D * D * stride;
#pragma unroll
    for (int b = 0; b < D; ++b)
      u[b] = ld_stream<NTL>(lk + link_row(BWD ? b * D + row : row * D + b, stride) + link_site(D * D, stride, lsite));
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const cplx<T> *in = in0 + k * rstride;
    cplx<T> p[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) p[s] = in[(size_t)(s * D + row) * stride + nb];
    hs[k][0][row][lane] = p[0] + ipow<PROJ_PH(MU, SIG, 0)>(p[2 + ECOL(MU, 0)]);
    hs[k][1][row][lane] = p[1] + ipow<PROJ_PH(MU, SIG, 1)>(p[2 + ECOL(MU, 1)]);
  }
}

// Compact form, after the barrier: rebuild this lane's row (forward) or
// column (backward) of U_R from the fundamental rows (columns) a1, a2 staged
// in fl.
// (No-op for stored links.)
template <int D, typename T, bool BWD, int FLY, typename U>
__device__ __forceinline__ void cs_rebuild(U (&u)[D], cplx<T> (*fl)[64], int row, int lane) {
  if constexpr (FLY != 0) {
    constexpr bool SYM = FLY == 2;
    constexpr int N = two_index_n<D, SYM>();
    int a1, a2;
    pair_of<N, SYM>(row, a1, a2);
    cplx<T> xr[N], yr[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      xr[c] = fl[BWD ? c * N + a1 : a1 * N + c][lane];
      yr[c] = fl[BWD ? c * N + a2 : a2 * N + c][lane];
    }
    rebuild_row<D, N, SYM, T>(u, xr, yr, (SYM && a1 == a2) ? (T)0.70710678118654752440 : (T)1);
  }
}

// Compute: after the barrier, the full projected two-spinor of this lane's
// site is in LDS; apply the link row and reconstruct the lower spin half.
template <int D, bool REAL, typename T, int MU, int SIG, bool BWD, int NR>
__device__ __forceinline__ void cs_compute(cplx<T> (&acc)[NR][4], const typename LinkT<T, REAL>::type (&u)[D],
                                           cplx<T> (*hs)[2][D][64], int lane) {
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    cplx<T> chi[2] = {mk<T>(0, 0), mk<T>(0, 0)};
#pragma unroll
    for (int b = 0; b < D; ++b) {
      chi[0] = link_mac(u[b], hs[k][0][b][lane], chi[0], BWD);
      chi[1] = link_mac(u[b], hs[k][1][b][lane], chi[1], BWD);
    }
    acc[k][0] = acc[k][0] + chi[0];
    acc[k][1] = acc[k][1] + chi[1];
    acc[k][2] = acc[k][2] + ipow<RECON_PH(MU, SIG, 0)>(chi[RECON_SRC(MU, 0)]);
    acc[k][3] = acc[k][3] + ipow<RECON_PH(MU, SIG, 1)>(chi[RECON_SRC(MU, 1)]);
  }
  // keep each phase's arithmetic next to its barrier
  __builtin_amdgcn_sched_barrier(0);
}

// One direction mu.  STG = 1: forward and backward hops are two barrier
// phases (LDS buffers 0 and 1).  STG = 2: both are staged before a single
// barrier (LDS buffers 2*(MU&1) and 2*(MU&1)+1), which halves the barriers and
// doubles the loads in flight per phase at the cost of twice the LDS.
// (STG = 4, two directions per phase, is cs_mu2 below.)
template <int D, bool REAL, typename T, int MU, int SF, int NR, int STG, bool NTL, int NB, int FLY>
__device__ __forceinline__ void cs_mu(cplx<T> (&acc)[NR][4], cplx<T> (*hs)[NR][2][D][64],
                                      cplx<T> (*fls)[(fly_rows<D, FLY>())][64], const Geom &g, int parity,
                                      const typename LinkT<T, REAL>::type *links, const cplx<T> *flinks,
                                      const cplx<T> *in0, size_t rstride, int t, int x, int y, int z, int is, int row,
                                      int lane) {
  using L = typename LinkT<T, REAL>::type;
  const int nbf = nb_index(g, t, x, y, z, MU, 1);
  const int nbb = nb_index(g, t, x, y, z, MU, 0);
  L uf[D], ub[D];
  if constexpr (STG == 2) {
    constexpr int B0 = 2 * (MU & 1);
    cs_stage<D, REAL, T, MU, SF, false, NR, NTL, FLY>(uf, hs[B0], fls[B0], g, parity, links, flinks, in0, rstride,
                                                      nbf, is, row, lane);
    cs_stage<D, REAL, T, MU, -SF, true, NR, NTL, FLY>(ub, hs[B0 + 1], fls[B0 + 1], g, parity, links, flinks, in0,
                                                      rstride, nbb, nbb, row, lane);
    __syncthreads();
    cs_rebuild<D, T, false, FLY>(uf, fls[B0], row, lane);
    cs_compute<D, REAL, T, MU, SF, false, NR>(acc, uf, hs[B0], lane);
    cs_rebuild<D, T, true, FLY>(ub, fls[B0 + 1], row, lane);
    cs_compute<D, REAL, T, MU, -SF, true, NR>(acc, ub, hs[B0 + 1], lane);
  } else {
    cs_stage<D, REAL, T, MU, SF, false, NR, NTL, FLY>(uf, hs[0], fls[0], g, parity, links, flinks, in0, rstride, nbf,
                                                      is, row, lane);
    __syncthreads();
    cs_rebuild<D, T, false, FLY>(uf, fls[0], row, lane);
    cs_compute<D, REAL, T, MU, SF, false, NR>(acc, uf, hs[0], lane);
    cs_stage<D, REAL, T, MU, -SF, true, NR, NTL, FLY>(ub, hs[1], fls[1], g, parity, links, flinks, in0,
                                                      rstride, nbb, nbb, row, lane);
    __syncthreads();
    cs_rebuild<D, T, true, FLY>(ub, fls[1], row, lane);
    cs_compute<D, REAL, T, MU, -SF, true, NR>(acc, ub, hs[1], lane);
  }
}

// Compact form, software-pipelined (FP64, one rhs per block, STG = 1): the
// global loads of hop h + 1 (this wave's fundamental link entries and spinor
// components) are issued right after hop h's barrier and land while hop h
// rebuilds its link row and computes; one barrier per hop over the two LDS
// buffer sets (a buffer is rewritten two hops after it was read, with a
// barrier between).  Measured per hop: SU(3) SYM 48x24^3 212 -> 191 us,
// SU(4) 2AS 96x48^3 4769 -> 4014 us; in FP32 it gains nothing (1811 -> 1859
// us for SU(4) 2AS) and is not used.
template <int D, typename T, int NR, int FLY>
struct CsRaw {
  cplx<T> f[fly_rows<D, FLY>() / D];   // fundamental entries row, row + D, ...
  cplx<T> p[NR][4];                     // colour `row` of the neighbour spinor, per spin
};

template <int D, typename T, int MU, bool BWD, int NR, bool NTL, int FLY>
__device__ __forceinline__ void cs_load(CsRaw<D, T, NR, FLY> &rw, const Geom &g, int parity, const cplx<T> *flinks,
                                        const cplx<T> *in0, size_t rstride, int nb, int lsite, int row) {
  constexpr int NE = fly_entries<D, FLY>();
  const int stride = g.stride;
  const int lpar = BWD ? 1 - parity : parity;
  const cplx<T> *fk = flinks + (size_t)(lpar * 4 + MU) * NE * stride + link_site(NE, stride, lsite);
#pragma unroll
  for (int j = 0; j < fly_rows<D, FLY>() / D; ++j) {
    const int e = row + j * D;
    rw.f[j] = ld_stream<NTL>(fk + link_row(e < NE ? e : NE - 1, stride));
  }
#pragma unroll
  for (int k = 0; k < NR; ++k)
#pragma unroll
    for (int s = 0; s < 4; ++s) rw.p[k][s] = in0[k * rstride + (size_t)(s * D + row) * stride + nb];
}

template <int D, typename T, int MU, int SIG, int NR, int FLY>
__device__ __forceinline__ void cs_publish(const CsRaw<D, T, NR, FLY> &rw, cplx<T> (*hs)[2][D][64], cplx<T> (*fl)[64],
                                           int row, int lane) {
#pragma unroll
  for (int j = 0; j < fly_rows<D, FLY>() / D; ++j) fl[row + j * D][lane] = rw.f[j];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    hs[k][0][row][lane] = rw.p[k][0] + ipow<PROJ_PH(MU, SIG, 0)>(rw.p[k][2 + ECOL(MU, 0)]);
    hs[k][1][row][lane] = rw.p[k][1] + ipow<PROJ_PH(MU, SIG, 1)>(rw.p[k][2 + ECOL(MU, 1)]);
  }
}

template <int D, typename T, int SF, int NR, bool NTL, int FLY, int H = 0>
__device__ __forceinline__ void cs_pipe(cplx<T> (&acc)[NR][4], cplx<T> (*hs)[NR][2][D][64],
                                        cplx<T> (*fls)[(fly_rows<D, FLY>())][64], CsRaw<D, T, NR, FLY> &rw,
                                        const Geom &g, int parity, const cplx<T> *flinks, const cplx<T> *in0,
                                        size_t rstride, const int (&nbf)[4], const int (&nbb)[4], int is, int row,
                                        int lane) {
  if constexpr (H < 8) {
    constexpr int MU = H / 2;
    constexpr bool BWD = (H & 1) != 0;
    constexpr int SIG = BWD ? -SF : SF;
    cs_publish<D, T, MU, SIG, NR, FLY>(rw, hs[H & 1], fls[H & 1], row, lane);
    __syncthreads();
    if constexpr (H < 7) {
      constexpr int MU1 = (H + 1) / 2;
      constexpr bool BWD1 = ((H + 1) & 1) != 0;
      cs_load<D, T, MU1, BWD1, NR, NTL, FLY>(rw, g, parity, flinks, in0, rstride, BWD1 ? nbb[MU1] : nbf[MU1],
                                             BWD1 ? nbb[MU1] : is, row);
    }
    cplx<T> u[D];
    cs_rebuild<D, T, BWD, FLY>(u, fls[H & 1], row, lane);
    cs_compute<D, false, T, MU, SIG, BWD, NR>(acc, u, hs[H & 1], lane);
    cs_pipe<D, T, SF, NR, NTL, FLY, H + 1>(acc, hs, fls, rw, g, parity, flinks, in0, rstride, nbf, nbb, is, row,
                                           lane);
  }
}

// Directions MU0 and MU0 + 1 together (STG = 4): the four hops are staged
// into LDS buffers 2*MU0 .. 2*MU0 + 3 before one barrier, so a launch has two
// barrier phases and four hops' loads in flight in each.
template <int D, bool REAL, typename T, int MU0, int SF, int NR, bool NTL, int FLY>
__device__ __forceinline__ void cs_mu2(cplx<T> (&acc)[NR][4], cplx<T> (*hs)[NR][2][D][64], const Geom &g, int parity,
                                       const typename LinkT<T, REAL>::type *links, const cplx<T> *flinks,
                                       const cplx<T> *in0, size_t rstride, int t, int x, int y, int z, int is, int row,
                                       int lane) {
  using L = typename LinkT<T, REAL>::type;
  constexpr int MU1 = MU0 + 1, B0 = 2 * MU0;
  const int f0 = nb_index(g, t, x, y, z, MU0, 1), b0 = nb_index(g, t, x, y, z, MU0, 0);
  const int f1 = nb_index(g, t, x, y, z, MU1, 1), b1 = nb_index(g, t, x, y, z, MU1, 0);
  static_assert(FLY == 0, "four hops per phase: stored links only");
  L u0f[D], u0b[D], u1f[D], u1b[D];
  cs_stage<D, REAL, T, MU0, SF, false, NR, NTL, 0>(u0f, hs[B0], nullptr, g, parity, links, flinks, in0, rstride, f0,
                                                   is, row, lane);
  cs_stage<D, REAL, T, MU0, -SF, true, NR, NTL, 0>(u0b, hs[B0 + 1], nullptr, g, parity, links, flinks, in0, rstride,
                                                   b0, b0, row, lane);
  cs_stage<D, REAL, T, MU1, SF, false, NR, NTL, 0>(u1f, hs[B0 + 2], nullptr, g, parity, links, flinks, in0, rstride,
                                                   f1, is, row, lane);
  cs_stage<D, REAL, T, MU1, -SF, true, NR, NTL, 0>(u1b, hs[B0 + 3], nullptr, g, parity, links, flinks, in0, rstride,
                                                   b1, b1, row, lane);
  __syncthreads();
  cs_compute<D, REAL, T, MU0, SF, false, NR>(acc, u0f, hs[B0], lane);
  cs_compute<D, REAL, T, MU0, -SF, true, NR>(acc, u0b, hs[B0 + 1], lane);
  cs_compute<D, REAL, T, MU1, SF, false, NR>(acc, u1f, hs[B0 + 2], lane);
  cs_compute<D, REAL, T, MU1, -SF, true, NR>(acc, u1b, hs[B0 + 3], lane);
}

// NTL: links read with streaming loads (set when the launch has a single
// group of right-hand sides, so that no other block re-reads them).
template <int D, bool REAL, typename T, bool DAG, int NR, int STG, bool NTL, int W, int FLY>
__global__ __launch_bounds__(64 * D) __attribute__((amdgpu_waves_per_eu(W))) void k_hop_cs(HopArgs a) {
  constexpr int NB = 2 * STG;   // LDS buffers
  constexpr int NE = fly_rows<D, FLY>();
  __shared__ cplx<T> hs[NB][NR][2][D][64];
  __shared__ double sh[D];
  cplx<T>(*fls)[NE][64] = nullptr;   // compact form: staged fundamental entries
  if constexpr (FLY != 0) {
    __shared__ cplx<T> fbuf[NB][NE][64];
    fls = fbuf;
  }
  // Work item = (tile, group of NR right-hand sides), group fastest, so the
  // groups of one tile are consecutive and (after the XCD remap) run on the
  // same XCD at nearly the same time: each link entry comes from HBM once
  // and from that XCD's L2 for the other groups.
  using L = typename LinkT<T, REAL>::type;
  const int ngroups = a.ngroups;
  const int w = tile_of_block(blockIdx.x, a.ntiles * ngroups, a.xcd_remap);
  const int q = w / ngroups, grp = w - q * ngroups;
  const int tile = tile_order(q, a);
  const int l = lattice_of_tile(a, tile);
  const Geom g = a.lat[l].g;
  const int tl = tile - a.lat[l].tile0;   // tile within its lattice
  const int lane = threadIdx.x & 63;
  const int row = FLY ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : (int)(threadIdx.x >> 6);
  const int i = tl * 64 + lane;
  const bool valid = i < g.Vh;
  const int is = valid ? i : g.Vh - 1;   // lanes past the end: see k_hop_sp
  const int r0 = grp * NR;
  const int sys0 = l * ngroups * NR + r0;
  const size_t rstride = (size_t)4 * D * g.stride;
  const size_t fbase = (size_t)a.lat[l].soff + r0 * rstride;
  const cplx<T> *in0 = static_cast<const cplx<T> *>(a.in) + fbase;
  const L *links = static_cast<const L *>(a.links) + a.lat[l].loff;
  const cplx<T> *flinks = FLY ? static_cast<const cplx<T> *>(a.flinks) + a.lat[l].floff : nullptr;
  int t, x, y, z;
  cb_coords(g, is, a.parity, t, x, y, z);
  cplx<T> acc[NR][4];
#pragma unroll
  for (int k = 0; k < NR; ++k)
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[k][s] = mk<T>(0, 0);
  constexpr int SF = DAG ? -1 : 1;   // forward hop: 1 - g_mu (dagger: 1 + g_mu)
  if constexpr (FLY != 0 && STG == 1 && NR == 1 && sizeof(T) == 8) {
    int nbf[4], nbb[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      nbf[mu] = nb_index(g, t, x, y, z, mu, 1);
      nbb[mu] = nb_index(g, t, x, y, z, mu, 0);
    }
    CsRaw<D, T, NR, FLY> rw;
    cs_load<D, T, 0, false, NR, NTL, FLY>(rw, g, a.parity, flinks, in0, rstride, nbf[0], is, row);
    cs_pipe<D, T, SF, NR, NTL, FLY>(acc, hs, fls, rw, g, a.parity, flinks, in0, rstride, nbf, nbb, is, row, lane);
  } else if constexpr (STG == 4) {
    cs_mu2<D, REAL, T, 0, SF, NR, NTL, FLY>(acc, hs, g, a.parity, links, flinks, in0, rstride, t, x, y, z, is, row,
                                            lane);
    cs_mu2<D, REAL, T, 2, SF, NR, NTL, FLY>(acc, hs, g, a.parity, links, flinks, in0, rstride, t, x, y, z, is, row,
                                            lane);
  } else {
    cs_mu<D, REAL, T, 0, SF, NR, STG, NTL, NB, FLY>(acc, hs, fls, g, a.parity, links, flinks, in0, rstride, t, x, y, z,
                                                    is, row, lane);
    cs_mu<D, REAL, T, 1, SF, NR, STG, NTL, NB, FLY>(acc, hs, fls, g, a.parity, links, flinks, in0, rstride, t, x, y, z,
                                                    is, row, lane);
    cs_mu<D, REAL, T, 2, SF, NR, STG, NTL, NB, FLY>(acc, hs, fls, g, a.parity, links, flinks, in0, rstride, t, x, y, z,
                                                    is, row, lane);
    cs_mu<D, REAL, T, 3, SF, NR, STG, NTL, NB, FLY>(acc, hs, fls, g, a.parity, links, flinks, in0, rstride, t, x, y, z,
                                                    is, row, lane);
  }
  const T cb = (T)(-0.5 * a.beta), ca = (T)a.alpha;
  // Two straight-line epilogues (with and without x_add): every accumulator
  // is used on both paths, so no arithmetic is sunk behind a branch.  The
  // output and x_add are streamed (each element is touched once).
  double nrm[NR];
  if (a.xadd) {
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      nrm[k] = 0.0;
      cplx<T> *out = static_cast<cplx<T> *>(a.out) + fbase + k * rstride;
      const cplx<T> *xa = static_cast<const cplx<T> *>(a.xadd) + fbase + k * rstride;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const size_t o = (size_t)(s * D + row) * g.stride + i;   // i < stride always
        cplx<T> v = cb * acc[k][s];
        const cplx<T> xv = ld_nt(xa + o);
        v.re = fma(ca, xv.re, v.re);
        v.im = fma(ca, xv.im, v.im);
        st_nt(out + o, v);
        nrm[k] += (double)v.re * v.re + (double)v.im * v.im;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      nrm[k] = 0.0;
      cplx<T> *out = static_cast<cplx<T> *>(a.out) + fbase + k * rstride;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const size_t o = (size_t)(s * D + row) * g.stride + i;
        const cplx<T> v = cb * acc[k][s];
        st_nt(out + o, v);
        nrm[k] += (double)v.re * v.re + (double)v.im * v.im;
      }
    }
  }
  if (a.partial) {
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const double s = block_sum(valid ? nrm[k] : 0.0, sh);
      if (threadIdx.x == 0) a.partial[(size_t)(sys0 + k) * a.prow + tl] = s;
    }
  }
}

// -------------------------------------------------------------- dispatch
// Waves per SIMD the register allocator is asked to allow (VGPR budget
// 512 / W per lane), chosen per (d_R, precision, right-hand sides per block)
// as the largest value that compiles without spills for the colour-split
// kernel.  (d_R = 15 is capped at 128 VGPRs by its 960-lane block and
// spills a little.)
constexpr int cs_waves(int D, bool dbl, int NR) {
  const int w = dbl ? (D <= 3 ? 4 : D <= 8 ? 3 : 2) : (D <= 4 ? 6 : D <= 6 ? 5 : D <= 10 ? 4 : 3);
  const int cut = NR >= 6 ? 3 : NR >= 3 ? 2 : NR == 2 ? 1 : 0;
  return w - cut > 1 ? w - cut : 1;
}
constexpr int sp_waves(int D, bool dbl) { return dbl ? 2 : (D <= 2 ? 4 : D <= 4 ? 2 : 3); }
// LDS of one colour-split block, hs[NB][NR][2][D][64], must fit the 160 KB
// a gfx950 workgroup may allocate (less the reduction scratch).  Blocks above
// 80 KB run one per CU; the autotuner weighs that against the link sharing.
constexpr int LDS_BUDGET = 160 * 1024 - 256;
template <int D, typename T, int NR, int STG, int FLY = 0>
constexpr bool cs_fits() {
  return 2 * STG * (NR * 2 * D + (FLY ? fly_rows<D, FLY>() : 0)) * 64 * (int)sizeof(cplx<T>) <= LDS_BUDGET;
}
// Six right-hand sides per block: colour form (unpaired) with d_R <= 4 only;
// beyond that the accumulators no longer fit in registers.
template <int D, typename T>
constexpr bool cs6_ok() {
  return D <= 4 && cs_fits<D, T, 6, 1>();
}

// The compact forms rebuild the entries after the barrier from LDS, so they
// hold no link registers across it: the same occupancy as the stored form.
constexpr int cs_waves_form(int D, bool dbl, int NR, bool, int) { return cs_waves(D, dbl, NR); }

// Four hops per phase (stage 4): one right-hand side per block, stored links,
// d_R <= 6 (at d_R = 6 in FP64 the block's 96 KB of LDS leave one block per
// CU; still the fastest stored form on SU(3) SYM 48x24^3, 324 against 331 us).
template <int D, typename T, int NR, int FLY>
constexpr bool cs4_ok() {
  return NR == 1 && FLY == 0 && D <= 6 && cs_fits<D, T, 1, 4>();
}

// stage: hops staged per barrier phase, 1, 2 (paired directions) or 4.
template <int D, bool REAL, typename T, bool DAG, int NR, bool NTL, int FLY>
static hipError_t launch_cs2(const HopArgs &a, int stage, hipStream_t st) {
  constexpr int WU = cs_waves_form(D, sizeof(T) == 8, NR, false, FLY);
  constexpr int WP = cs_waves_form(D, sizeof(T) == 8, NR, true, FLY);
  dim3 grid(a.ntiles * a.ngroups);
  if constexpr (cs4_ok<D, T, NR, FLY>()) {
    // (d_R = 6 in FP32: one wave per SIMD fewer, so that it compiles without spills)
    constexpr int WQ = (D == 6 && sizeof(T) == 4) ? WP - 1 : WP;
    if (stage == 4) {
      hipLaunchKernelGGL((k_hop_cs<D, REAL, T, DAG, NR, 4, NTL, WQ, FLY>), grid, dim3(64 * D), 0, st, a);
      return hipGetLastError();
    }
  }
  if constexpr (NR <= 4 && cs_fits<D, T, NR, 2, FLY>()) {
    if (stage == 2) {
      hipLaunchKernelGGL((k_hop_cs<D, REAL, T, DAG, NR, 2, NTL, WP, FLY>), grid, dim3(64 * D), 0, st, a);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_hop_cs<D, REAL, T, DAG, NR, 1, NTL, WU, FLY>), grid, dim3(64 * D), 0, st, a);
  return hipGetLastError();
}

// Links are streamed when one block group covers all right-hand sides (with
// several groups the groups of a tile re-read the links from L2).  Only the
// one-rhs-per-block kernels carry the streaming form.
template <int D, bool REAL, typename T, bool DAG, int NR, int FLY = 0>
static hipError_t launch_cs(HopArgs a, int nrhs, int stage, hipStream_t st, Counts *counts, int *prow) {
  set_tiles(a, 64, nrhs, counts, prow);
  a.ngroups = nrhs / NR;
  if constexpr (NR == 1) {
    if (a.ngroups == 1) return launch_cs2<D, REAL, T, DAG, 1, true, FLY>(a, stage, st);
  }
  return launch_cs2<D, REAL, T, DAG, NR, false, FLY>(a, stage, st);
}

// Compact forms: 1 or 2 right-hand sides per block (more spill registers).
template <int D, typename T, bool DAG, int FLY>
static hipError_t launch_compact(const HopArgs &a0, int nrhs, int pair, int nr, hipStream_t st, Counts *counts,
                                 int *prow) {
  if (nr >= 2 && nrhs % 2 == 0) {
    if constexpr (cs_fits<D, T, 2, 1, FLY>())
      return launch_cs<D, false, T, DAG, 2, FLY>(a0, nrhs, pair ? 2 : 1, st, counts, prow);
  }
  return launch_cs<D, false, T, DAG, 1, FLY>(a0, nrhs, pair ? 2 : 1, st, counts, prow);
}

template <int D, int FLY>
static hipError_t compact_d(const HopArgs &a, int prec, int dagger, int nrhs, int pair, int nr, hipStream_t st,
                            Counts *c, int *prow) {
  if (prec == 0)
    return dagger ? launch_compact<D, double, true, FLY>(a, nrhs, pair, nr, st, c, prow)
                  : launch_compact<D, double, false, FLY>(a, nrhs, pair, nr, st, c, prow);
  return dagger ? launch_compact<D, float, true, FLY>(a, nrhs, pair, nr, st, c, prow)
                : launch_compact<D, float, false, FLY>(a, nrhs, pair, nr, st, c, prow);
}

template <int D, bool REAL, typename T, bool DAG>
static hipError_t launch_typed(const HopArgs &a0, int nrhs, int variant, int nr, hipStream_t st, Counts *counts,
                               int *prow) {
  const int stage = variant == HOP_COLOUR_QUAD ? 4 : variant == HOP_COLOUR_PAIR ? 2 : 1;
  if (variant == HOP_SITE) {
    if constexpr (D <= 6) {
      HopArgs a = a0;
      const int rl = (nr == 4 && nrhs % 4 == 0) ? 4 : 1;
      set_tiles(a, 256 / rl, nrhs, counts, prow);
      a.ngroups = nrhs / rl;
      dim3 grid(a.ntiles * a.ngroups);
      constexpr int SW = sp_waves(D, sizeof(T) == 8);
      if (rl == 4) {
        if (a.ngroups == 1) hipLaunchKernelGGL((k_hop_sp<D, REAL, T, DAG, true, 4, SW>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_hop_sp<D, REAL, T, DAG, false, 4, SW>), grid, dim3(256), 0, st, a);
      } else {
        if (a.ngroups == 1) hipLaunchKernelGGL((k_hop_sp<D, REAL, T, DAG, true, 1, SW>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_hop_sp<D, REAL, T, DAG, false, 1, SW>), grid, dim3(256), 0, st, a);
      }
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (nr == 6 && nrhs % 6 == 0 && stage == 1) {
    if constexpr (cs6_ok<D, T>()) return launch_cs<D, REAL, T, DAG, 6>(a0, nrhs, stage, st, counts, prow);
  }
  if (nr == 4 && nrhs % 4 == 0) {
    if constexpr (cs_fits<D, T, 4, 1>()) return launch_cs<D, REAL, T, DAG, 4>(a0, nrhs, stage, st, counts, prow);
  }
  if (nr == 3 && nrhs % 3 == 0) {
    if constexpr (cs_fits<D, T, 3, 1>()) return launch_cs<D, REAL, T, DAG, 3>(a0, nrhs, stage, st, counts, prow);
  }
  if (nr == 2 && nrhs % 2 == 0) {
    if constexpr (cs_fits<D, T, 2, 1>()) return launch_cs<D, REAL, T, DAG, 2>(a0, nrhs, stage, st, counts, prow);
  }
  return launch_cs<D, REAL, T, DAG, 1>(a0, nrhs, stage, st, counts, prow);
}

template <int D, bool REAL>
static hipError_t launch_d(const HopArgs &a, int prec, int dagger, int nrhs, int variant, int nr, hipStream_t st,
                           Counts *c, int *prow) {
  if (prec == 0)
    return dagger ? launch_typed<D, REAL, double, true>(a, nrhs, variant, nr, st, c, prow)
                  : launch_typed<D, REAL, double, false>(a, nrhs, variant, nr, st, c, prow);
  return dagger ? launch_typed<D, REAL, float, true>(a, nrhs, variant, nr, st, c, prow)
                : launch_typed<D, REAL, float, false>(a, nrhs, variant, nr, st, c, prow);
}

hipError_t launch_hop(const HopArgs &a, int N, int rep, int d, int real, int prec, int dagger, int nrhs, int variant,
                      int nr, hipStream_t st, Counts *counts, int *prow) {
  if (variant == HOP_MULTI) return launch_hop_mr(a, d, real, prec, dagger, nrhs, nr, st, counts, prow);
  if (variant == HOP_COMPACT || variant == HOP_COMPACT_PAIR) {
    const int pair = variant == HOP_COMPACT_PAIR;
    if (rep == 2 && N == 2) return compact_d<3, 2>(a, prec, dagger, nrhs, pair, nr, st, counts, prow);
    if (rep == 2 && N == 3) return compact_d<6, 2>(a, prec, dagger, nrhs, pair, nr, st, counts, prow);
    if (rep == 2 && N == 4) return compact_d<10, 2>(a, prec, dagger, nrhs, pair, nr, st, counts, prow);
    if (rep == 3 && N == 4) return compact_d<6, 3>(a, prec, dagger, nrhs, pair, nr, st, counts, prow);
    return hipErrorInvalidValue;
  }
  if (real) {
    switch (d) {
      case 3: return launch_d<3, true>(a, prec, dagger, nrhs, variant, nr, st, counts, prow);
      case 8: return launch_d<8, true>(a, prec, dagger, nrhs, variant, nr, st, counts, prow);
      case 15: return launch_d<15, true>(a, prec, dagger, nrhs, variant, nr, st, counts, prow);
    }
  } else {
    switch (d) {
      case 2: return launch_d<2, false>(a, prec, dagger, nrhs, variant, nr, st, counts, prow);
      case 3: return launch_d<3, false>(a, prec, dagger, nrhs, variant, nr, st, counts, prow);
      case 4: return launch_d<4, false>(a, prec, dagger, nrhs, variant, nr, st, counts, prow);
      case 6: return launch_d<6, false>(a, prec, dagger, nrhs, variant, nr, st, counts, prow);
      case 10: return launch_d<10, false>(a, prec, dagger, nrhs, variant, nr, st, counts, prow);
    }
  }
  return hipErrorInvalidValue;
}

bool hop_nr_supported(int N, int d, int prec, int variant, int nr) {
  if (variant == HOP_MULTI) return nr == 1 || nr == 2 || nr == 3 || nr == 4 || nr == 6 || nr == 12;
  // as cs_fits, cs6_ok and launch_compact
  const int cb = prec == 0 ? 16 : 8;
  const int nbuf = variant == HOP_COLOUR_QUAD ? 8 : (variant == HOP_COLOUR_PAIR || variant == HOP_COMPACT_PAIR) ? 4 : 2;
  const bool compact = variant == HOP_COMPACT || variant == HOP_COMPACT_PAIR;
  if (variant == HOP_COLOUR_QUAD && (nr != 1 || d > 6)) return false;
  if (nr < 1 || nr > 6 || nr == 5) return false;
  if (nr == 6 && (variant != HOP_COLOUR || d > 4)) return false;
  if (compact && nr > 2) return false;
  return nbuf * (nr * 2 * d + (compact ? (N * N + d - 1) / d * d : 0)) * 64 * cb <= LDS_BUDGET;
}

bool compact_links_ok(int N, int rep) { return (rep == 2 && N >= 2 && N <= 4) || (rep == 3 && N == 4); }

bool hop_variant_ok(int N, int rep, int d, int variant) {
  if (variant == HOP_MULTI) return hop_mr_ok(d, rep == 1);
  if (variant == HOP_SITE) return d <= 6;
  if (variant == HOP_COMPACT || variant == HOP_COMPACT_PAIR) return compact_links_ok(N, rep);
  if (variant == HOP_COLOUR_QUAD) return d <= 6;
  return variant == HOP_COLOUR || variant == HOP_COLOUR_PAIR;
}

}  // namespace wd
