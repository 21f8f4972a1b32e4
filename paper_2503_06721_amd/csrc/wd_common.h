// Internal device/host helpers shared by the libwdirac HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace wd {

// ------------------------------------------------------------------ complex
template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T r, T i) {
  cplx<T> c;
  c.re = r;
  c.im = i;
  return c;
}
template <typename T>
__device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
__device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
__device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) { return mk(s * a.re, s * a.im); }
// a * b
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// acc + a * b
template <typename T>
__device__ __forceinline__ cplx<T> cfma(cplx<T> a, cplx<T> b, cplx<T> acc) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}
// acc + conj(a) * b
template <typename T>
__device__ __forceinline__ cplx<T> cfma_conj(cplx<T> a, cplx<T> b, cplx<T> acc) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
  return acc;
}
// acc + r * b for a real link entry r
template <typename T>
__device__ __forceinline__ cplx<T> rfma(T r, cplx<T> b, cplx<T> acc) {
  acc.re = fma(r, b.re, acc.re);
  acc.im = fma(r, b.im, acc.im);
  return acc;
}
// Non-temporal (streaming) loads and stores: the data is not kept in L2
// for reuse, so it does not displace data that is.
template <typename T>
__device__ __forceinline__ cplx<T> ld_nt(const cplx<T> *p) {
  using V = T __attribute__((ext_vector_type(2)));
  const V v = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
  return mk<T>(v.x, v.y);
}
__device__ __forceinline__ double ld_nt(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ld_nt(const float *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void st_nt(cplx<T> *p, cplx<T> c) {
  using V = T __attribute__((ext_vector_type(2)));
  V v;
  v.x = c.re;
  v.y = c.im;
  __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
}
// *p, streamed if NT
template <bool NT, typename L>
__device__ __forceinline__ L ld_stream(const L *p) {
  if constexpr (NT) return ld_nt(p);
  else return *p;
}

// i^K * a for a compile-time K in {0,1,2,3}
template <int K, typename T>
__device__ __forceinline__ cplx<T> ipow(cplx<T> a) {
  constexpr int k = ((K % 4) + 4) % 4;
  if constexpr (k == 0) return a;
  else if constexpr (k == 1) return mk(-a.im, a.re);
  else if constexpr (k == 2) return mk(-a.re, -a.im);
  else return mk(a.im, -a.re);
}

// ------------------------------------------------------------ spin algebra
// The paper's chiral basis (Sec. 2.2): gamma_mu = [[0, e_mu], [e_mu^+, 0]] with
// e_0 = -1 and e_k = -i sigma_k.  Every e_mu has exactly one non-zero per row:
// row s holds i^EPH[mu][s] in column ECOL[mu][s].
//   e_0 = [[-1, 0], [0, -1]]     e_1 = [[0, -i], [-i, 0]]
//   e_2 = [[0, -1], [1, 0]]      e_3 = [[-i, 0], [0, i]]
__host__ __device__ constexpr int ECOL(int mu, int s) { return (mu == 1 || mu == 2) ? 1 - s : s; }
__host__ __device__ constexpr int EPH(int mu, int s) {
  return mu == 0 ? 2 : mu == 1 ? 3 : mu == 2 ? (s == 0 ? 2 : 0) : (s == 0 ? 3 : 1);
}
// Spin projection.  For sigma = +1 (the projector 1 - gamma_mu) or -1 (1 + gamma_mu):
//   (1 - sigma gamma_mu) psi = [ h ; -sigma e_mu^+ h ],   h = psi_up - sigma e_mu psi_dn,
// because e_mu^+ e_mu = 1.  So only the two-spinor h is multiplied by the link.
//   h_s        = psi_s + i^PROJ_PH(mu,sig,s) psi_{2 + ECOL(mu,s)}
//   lower_r    = i^RECON_PH(mu,sig,r) chi_{RECON_SRC(mu,r)}      (chi = U h)
// with -sigma = i^(sigma > 0 ? 2 : 0) and conj(i^k) = i^(4-k).
__host__ __device__ constexpr int SIGPH(int sig) { return sig > 0 ? 2 : 0; }
__host__ __device__ constexpr int PROJ_PH(int mu, int sig, int s) { return (EPH(mu, s) + SIGPH(sig)) & 3; }
__host__ __device__ constexpr int RECON_SRC(int mu, int r) { return ECOL(mu, r); }
__host__ __device__ constexpr int RECON_PH(int mu, int sig, int r) {
  return (4 - EPH(mu, ECOL(mu, r)) + SIGPH(sig)) & 3;
}

// ---------------------------------------------------------------- geometry
struct Geom {
  int T, X, Y, Z;   // extents, all even
  int Vh;           // sites per parity
  int stride;       // padded site count of one packed component row
  int bc[4];
};

// Coordinates of the site with index i among the sites of parity p.  With Z
// even, that site has lexicographic index 2i or 2i+1 and both share t, x, y.
__device__ __forceinline__ void cb_coords(const Geom &g, int i, int p, int &t, int &x, int &y, int &z) {
  int lex0 = 2 * i;
  int z0 = lex0 % g.Z;
  int r = lex0 / g.Z;
  y = r % g.Y;
  r /= g.Y;
  x = r % g.X;
  t = r / g.X;
  z = z0 + ((t + x + y + p) & 1);
}
__device__ __forceinline__ int cb_index(const Geom &g, int t, int x, int y, int z) {
  return (((t * g.X + x) * g.Y + y) * g.Z + z) >> 1;
}
// Index (among the opposite parity) of the neighbour x + dir*mu.
__device__ __forceinline__ int nb_index(const Geom &g, int t, int x, int y, int z, int mu, int fwd) {
  if (mu == 0) t = fwd ? (t + 1 == g.T ? 0 : t + 1) : (t == 0 ? g.T - 1 : t - 1);
  else if (mu == 1) x = fwd ? (x + 1 == g.X ? 0 : x + 1) : (x == 0 ? g.X - 1 : x - 1);
  else if (mu == 2) y = fwd ? (y + 1 == g.Y ? 0 : y + 1) : (y == 0 ? g.Y - 1 : y - 1);
  else z = fwd ? (z + 1 == g.Z ? 0 : z + 1) : (z == 0 ? g.Z - 1 : z - 1);
  return cb_index(g, t, x, y, z);
}

// ------------------------------------------------------------ link layout
// Packed links of one lattice: (parity, direction) blocks of E x stride
// elements (E = d_R^2 represented entries, or N^2 for the compact copy).
// Inside a block the sites go in tiles of kLinkTile: the E entry rows of a
// tile (kLinkTile consecutive sites each) follow one another, so that the
// link entries a wavefront reads for its 64 sites form one contiguous run
// instead of E runs a whole stride apart.  (kLinkTile = 0: plain
// structure of arrays, element (e, i) at e * stride + i.)
constexpr int kLinkTile = 64;
// Offset of site i's element of entry row 0 inside a block; entry e adds
// link_row(e).
__host__ __device__ __forceinline__ size_t link_site(int E, int stride, int i) {
  if constexpr (kLinkTile == 0) {
    (void)E;
    (void)stride;
    return (size_t)i;
  } else {
    return (size_t)(i / kLinkTile) * ((size_t)E * kLinkTile) + (size_t)(i % kLinkTile);
  }
}
__host__ __device__ __forceinline__ size_t link_row(int e, int stride) {
  if constexpr (kLinkTile == 0) return (size_t)e * stride;
  else {
    (void)stride;
    return (size_t)e * kLinkTile;
  }
}
// Element (e, i) of (parity, direction) block pmu.
__host__ __device__ __forceinline__ size_t link_at(int pmu, int E, int stride, int e, int i) {
  return (size_t)pmu * E * stride + link_site(E, stride, i) + link_row(e, stride);
}

// ------------------------------------------------------------- reductions
// Sum over a 64-lane wavefront (result valid in every lane).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
// Block sum, result valid in thread 0.  `sh` holds blockDim/64 doubles.
__device__ __forceinline__ double block_sum(double v, double *sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < nw; ++k) s += sh[k];
  return s;
}

}  // namespace wd
