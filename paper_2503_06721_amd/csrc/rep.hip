// Represented links U -> U_R (Sec. 2.3), the fermion boundary phase folded
// into the links that cross the boundary (Sec. 6.3.1), and the packing of
// fields between the caller's canonical layout and the structure-of-arrays
// layout of the kernels.
// The bases of the representations are fixed in wd_rep.h.
#include "wd_common.h"
#include "wd_kernels.h"
#include "wd_rep.h"

namespace wd {

template <typename T>
__device__ __forceinline__ void store_entry(void *base, size_t off, cplx<double> v, double sign, bool real) {
  if (real) static_cast<T *>(base)[off] = (T)(sign * v.re);
  else static_cast<cplx<T> *>(base)[off] = mk<T>((T)(sign * v.re), (T)(sign * v.im));
}

template <int N, int REP, typename T>
__global__ __launch_bounds__(256) void k_rep_links(const cplx<double> *__restrict__ U, void *__restrict__ UR,
                                                    void *__restrict__ F, Geom g) {
  constexpr int D = rep_dim(N, REP);
  const int V = 2 * g.Vh;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= 4 * V) return;
  const int lex = gid >> 2, mu = gid & 3;
  int r = lex;
  const int z = r % g.Z; r /= g.Z;
  const int y = r % g.Y; r /= g.Y;
  const int x = r % g.X;
  const int t = r / g.X;
  const int par = (t + x + y + z) & 1;
  const int cb = lex >> 1;
  const int c[4] = {t, x, y, z};
  const int L[4] = {g.T, g.X, g.Y, g.Z};
  const double sign = (c[mu] == L[mu] - 1) ? (double)g.bc[mu] : 1.0;
  cplx<double> u[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) u[i][j] = U[(size_t)gid * N * N + i * N + j];
  for (int A = 0; A < D; ++A)
    for (int B = 0; B < D; ++B)
      store_entry<T>(UR, link_at(par * 4 + mu, D * D, g.stride, A * D + B, cb), rep_entry<N, REP>(u, A, B), sign,
                     REP == 1);
  if (F) {
    // compact fundamental copy: i U where the phase is -1
    cplx<T> *f = static_cast<cplx<T> *>(F);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        const cplx<double> v = u[i][j];
        f[link_at(par * 4 + mu, N * N, g.stride, i * N + j, cb)] =
            sign < 0.0 ? mk<T>((T)(-v.im), (T)v.re) : mk<T>((T)v.re, (T)v.im);
      }
  }
}

template <int N, int REP>
static hipError_t rep_launch(const void *U, void *UR, void *F, const Geom &g, int prec, hipStream_t st) {
  const int n = 8 * g.Vh;
  dim3 grid((n + 255) / 256);
  if (prec == 0)
    hipLaunchKernelGGL((k_rep_links<N, REP, double>), grid, dim3(256), 0, st, (const cplx<double> *)U, UR, F, g);
  else
    hipLaunchKernelGGL((k_rep_links<N, REP, float>), grid, dim3(256), 0, st, (const cplx<double> *)U, UR, F, g);
  return hipGetLastError();
}

template <int N>
static hipError_t rep_launch_n(const void *U, void *UR, void *F, const Geom &g, int rep, int prec,
                               hipStream_t st) {
  switch (rep) {
    case 0: return rep_launch<N, 0>(U, UR, F, g, prec, st);
    case 1: return rep_launch<N, 1>(U, UR, F, g, prec, st);
    case 2: return rep_launch<N, 2>(U, UR, F, g, prec, st);
    case 3:
      if constexpr (N > 2) return rep_launch<N, 3>(U, UR, F, g, prec, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_rep_links(const void *U, void *UR, void *F, const Geom &g, int N, int rep, int prec,
                            hipStream_t st) {
  switch (N) {
    case 2: return rep_launch_n<2>(U, UR, F, g, rep, prec, st);
    case 3: return rep_launch_n<3>(U, UR, F, g, rep, prec, st);
    case 4: return rep_launch_n<4>(U, UR, F, g, rep, prec, st);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------ link unpack
template <typename T>
__global__ __launch_bounds__(256) void k_unpack_links(double *__restrict__ out, const void *__restrict__ UR,
                                                       Geom g, int d, int real) {
  const int V = 2 * g.Vh;
  const size_t n = (size_t)4 * V * d * d;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n) return;
  const int e = gid % (d * d);
  const size_t link = gid / (d * d);
  const int lex = (int)(link >> 2), mu = (int)(link & 3);
  int r = lex;
  const int z = r % g.Z; r /= g.Z;
  const int y = r % g.Y; r /= g.Y;
  const int x = r % g.X;
  const int t = r / g.X;
  const int par = (t + x + y + z) & 1;
  const size_t src = link_at(par * 4 + mu, d * d, g.stride, e, lex >> 1);
  if (real) {
    out[gid] = (double)static_cast<const T *>(UR)[src];
  } else {
    const cplx<T> v = static_cast<const cplx<T> *>(UR)[src];
    out[2 * gid] = (double)v.re;
    out[2 * gid + 1] = (double)v.im;
  }
}

hipError_t launch_unpack_links(void *canon, const void *UR, const Geom &g, int d, int real, int prec,
                               hipStream_t st) {
  const size_t n = (size_t)8 * g.Vh * d * d;
  dim3 grid((unsigned)((n + 255) / 256));
  if (prec == 0)
    hipLaunchKernelGGL(k_unpack_links<double>, grid, dim3(256), 0, st, (double *)canon, UR, g, d, real);
  else
    hipLaunchKernelGGL(k_unpack_links<float>, grid, dim3(256), 0, st, (double *)canon, UR, g, d, real);
  return hipGetLastError();
}

// ---------------------------------------------------------- spinor packing
// Thread per (rhs, site of the parity, component); the packed side is the
// coalesced one.
template <typename T>
__global__ __launch_bounds__(256) void k_pack_spinor(cplx<T> *__restrict__ packed, cplx<T> *__restrict__ canon,
                                                      Geom g, int d, int parity, int nrhs, int unpack) {
  const int ncomp = 4 * d;
  const size_t n = (size_t)nrhs * ncomp * g.Vh;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n) return;
  const int i = (int)(gid % g.Vh);
  const size_t rc = gid / g.Vh;
  const int comp = (int)(rc % ncomp);
  const int r = (int)(rc / ncomp);
  int t, x, y, z;
  cb_coords(g, i, parity, t, x, y, z);
  const size_t lex = (((size_t)t * g.X + x) * g.Y + y) * g.Z + z;
  const size_t co = ((size_t)r * 2 * g.Vh + lex) * ncomp + comp;
  const size_t po = ((size_t)r * ncomp + comp) * g.stride + i;
  if (unpack) canon[co] = packed[po];
  else packed[po] = canon[co];
}

hipError_t launch_pack_spinor(void *packed, const void *canon, const Geom &g, int d, int parity, int nrhs,
                              int prec, int unpack, hipStream_t st) {
  const size_t n = (size_t)nrhs * 4 * d * g.Vh;
  dim3 grid((unsigned)((n + 255) / 256));
  if (prec == 0)
    hipLaunchKernelGGL(k_pack_spinor<double>, grid, dim3(256), 0, st, (cplx<double> *)packed,
                       (cplx<double> *)canon, g, d, parity, nrhs, unpack);
  else
    hipLaunchKernelGGL(k_pack_spinor<float>, grid, dim3(256), 0, st, (cplx<float> *)packed,
                       (cplx<float> *)canon, g, d, parity, nrhs, unpack);
  return hipGetLastError();
}

}  // namespace wd
