// Fermion force of S_f = phi^+ (D-hat^+ D-hat)^{-1} phi per link (force of
// Sec. 2.5 written for the even-odd operator of Sec. 5.3.3):
//   dS/dw^a_mu(x) = Im tr[T^a_R U_R(x,mu) Sigma_mu(x)],
//   Sigma_mu(x) = tr_spin[(1 - g_mu) X(x+mu) Y(x)^+ + (1 + g_mu) Y(x+mu) X(x)^+],
// for the variation U -> exp(i w^a T^a_F) U, returned as the Hermitian
// traceless P_mu(x) = sum_a (dS/dw^a) T^a_F.
//
// Evaluation used here:
//  * 1 - s g_mu is Hermitian with (1 - s g_mu)^2 = 2 (1 - s g_mu), so
//    tr_spin[(1 - s g_mu) A B^+] = sum_{k=0,1} h_k(A) h_k(B)^+ with h the
//    spin-projected two-spinor of the hopping kernel; Sigma is a sum of four
//    colour outer products and U_R Sigma = sum_j (U_R h_j) k_j^+.
//  * for every representation tr(T^a_R M) = tr(T^a Z) for an N x N matrix
//    Z(M), the pull-back of wd_rep.h, and
//    sum_a Im tr(T^a Z) T^a = 1/2 (A - tr(A)/N) with A = (Z - Z^+)/(2i)
//    (completeness of the generators, tr T^a T^b = delta/2).
// The boundary phase is already folded into U_R, so neighbours are periodic.
#include "wd_common.h"
#include "wd_kernels.h"
#include "wd_rep.h"

namespace wd {

template <int D, int MU, int SIG>
__device__ __forceinline__ void project(const cplx<double> *__restrict__ f, int stride, int site,
                                        cplx<double> (&h)[2][D]) {
#pragma unroll
  for (int c = 0; c < D; ++c) {
    cplx<double> p[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) p[s] = f[(size_t)(s * D + c) * stride + site];
    h[0][c] = p[0] + ipow<PROJ_PH(MU, SIG, 0)>(p[2 + ECOL(MU, 0)]);
    h[1][c] = p[1] + ipow<PROJ_PH(MU, SIG, 1)>(p[2 + ECOL(MU, 1)]);
  }
}

template <int N, int REP, int MU>
__device__ void force_link(double *__restrict__ P, const cplx<double> *Xe, const cplx<double> *Xo,
                           const cplx<double> *Ye, const cplx<double> *Yo, const void *UR,
                           const cplx<double> *__restrict__ U, const Geom &g, int lex,
                           int par, int cb, int t, int x, int y, int z, double scale, int accumulate) {
  constexpr int D = rep_dim(N, REP);
  constexpr bool REAL = REP == 1;
  const int nb = nb_index(g, t, x, y, z, MU, 1);
  const cplx<double> *Xh = par ? Xo : Xe, *Yh = par ? Yo : Ye;   // own parity
  const cplx<double> *Xn = par ? Xe : Xo, *Yn = par ? Ye : Yo;   // neighbour parity
  // v_j = U_R h_j and w_j for the four outer products of U_R Sigma
  cplx<double> hv[4][D], w[4][D];
  {
    cplx<double> h[2][D], k[2][D];
    project<D, MU, 1>(Xn, g.stride, nb, h);    // (1 - g) X(x+mu)
    project<D, MU, 1>(Yh, g.stride, cb, k);    //         Y(x)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      hv[0][c] = h[0][c]; hv[1][c] = h[1][c];
      w[0][c] = k[0][c]; w[1][c] = k[1][c];
    }
    project<D, MU, -1>(Yn, g.stride, nb, h);   // (1 + g) Y(x+mu)
    project<D, MU, -1>(Xh, g.stride, cb, k);   //         X(x)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      hv[2][c] = h[0][c]; hv[3][c] = h[1][c];
      w[2][c] = k[0][c]; w[3][c] = k[1][c];
    }
  }
  cplx<double> v[4][D];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int a = 0; a < D; ++a) v[j][a] = mk(0.0, 0.0);
  const size_t lbase = (size_t)(par * 4 + MU) * D * D * g.stride + link_site(D * D, g.stride, cb);
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      const size_t o = lbase + link_row(a * D + b, g.stride);
      if constexpr (REAL) {
        const double u = static_cast<const double *>(UR)[o];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j][a] = rfma(u, hv[j][b], v[j][a]);
      } else {
        const cplx<double> u = static_cast<const cplx<double> *>(UR)[o];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j][a] = cfma(u, hv[j][b], v[j][a]);
      }
    }
  // M_BA = sum_j v_j[B] conj(w_j[A])
  auto Mel = [&](int B, int A) {
    cplx<double> m = mk(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < 4; ++j) m = cfma_conj(w[j][A], v[j][B], m);
    return m;
  };
  cplx<double> Z[N][N];
  rep_pullback<N, REP>(Mel, Z);
  // A = (Z - Z^+)/(2i);  P = (A - tr(A)/N) / 2
  cplx<double> Am[N][N];
  double trA = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      // (Z_ij - conj(Z_ji)) / (2i)
      const cplx<double> dlt = mk(Z[i][j].re - Z[j][i].re, Z[i][j].im + Z[j][i].im);
      Am[i][j] = mk(0.5 * dlt.im, -0.5 * dlt.re);
    }
#pragma unroll
  for (int i = 0; i < N; ++i) trA += Am[i][i].re;
  cplx<double> F[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j)
      F[i][j] = mk(scale * (0.5 * Am[i][j].re - (i == j ? 0.5 * trA / N : 0.0)), scale * 0.5 * Am[i][j].im);
  if (U) {
    // G = 2i P U, the gradient for dS = Re tr(G^+ dU) along dU = i w T U
    const cplx<double> *u = U + ((size_t)lex * 4 + MU) * N * N;
    cplx<double> G[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) {
        cplx<double> g = mk(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < N; ++k) g = cfma(F[i][k], u[k * N + j], g);
        G[i][j] = mk(-2.0 * g.im, 2.0 * g.re);
      }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) F[i][j] = G[i][j];
  }
  double *out = P + ((size_t)lex * 4 + MU) * N * N * 2;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double re = F[i][j].re, im = F[i][j].im;
      if (accumulate) {
        re += out[2 * (i * N + j)];
        im += out[2 * (i * N + j) + 1];
      }
      out[2 * (i * N + j)] = re;
      out[2 * (i * N + j) + 1] = im;
    }
}

template <int N, int REP>
__global__ __launch_bounds__(256) void k_force(double *P, const cplx<double> *Xe, const cplx<double> *Xo,
                                               const cplx<double> *Ye, const cplx<double> *Yo, const void *UR,
                                               const cplx<double> *U, Geom g, double scale, int accumulate) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= 8 * g.Vh) return;
  const int lex = gid >> 2, mu = gid & 3;
  int r = lex;
  const int z = r % g.Z; r /= g.Z;
  const int y = r % g.Y; r /= g.Y;
  const int x = r % g.X;
  const int t = r / g.X;
  const int par = (t + x + y + z) & 1, cb = lex >> 1;
  switch (mu) {
    case 0: force_link<N, REP, 0>(P, Xe, Xo, Ye, Yo, UR, U, g, lex, par, cb, t, x, y, z, scale, accumulate); break;
    case 1: force_link<N, REP, 1>(P, Xe, Xo, Ye, Yo, UR, U, g, lex, par, cb, t, x, y, z, scale, accumulate); break;
    case 2: force_link<N, REP, 2>(P, Xe, Xo, Ye, Yo, UR, U, g, lex, par, cb, t, x, y, z, scale, accumulate); break;
    default: force_link<N, REP, 3>(P, Xe, Xo, Ye, Yo, UR, U, g, lex, par, cb, t, x, y, z, scale, accumulate); break;
  }
}

template <int N, int REP>
static hipError_t force_launch(void *P, const void *Xe, const void *Xo, const void *Ye, const void *Yo, const void *UR,
                               const void *U, const Geom &g, double scale, int accumulate, hipStream_t st) {
  const int n = 8 * g.Vh;
  hipLaunchKernelGGL((k_force<N, REP>), dim3((n + 255) / 256), dim3(256), 0, st, (double *)P,
                     (const cplx<double> *)Xe, (const cplx<double> *)Xo, (const cplx<double> *)Ye,
                     (const cplx<double> *)Yo, UR, (const cplx<double> *)U, g, scale, accumulate);
  return hipGetLastError();
}

template <int N>
static hipError_t force_n(void *P, const void *Xe, const void *Xo, const void *Ye, const void *Yo, const void *UR,
                          const void *U, const Geom &g, int rep, double scale, int accumulate, hipStream_t st) {
  switch (rep) {
    case 0: return force_launch<N, 0>(P, Xe, Xo, Ye, Yo, UR, U, g, scale, accumulate, st);
    case 1: return force_launch<N, 1>(P, Xe, Xo, Ye, Yo, UR, U, g, scale, accumulate, st);
    case 2: return force_launch<N, 2>(P, Xe, Xo, Ye, Yo, UR, U, g, scale, accumulate, st);
    case 3:
      if constexpr (N > 2) return force_launch<N, 3>(P, Xe, Xo, Ye, Yo, UR, U, g, scale, accumulate, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_force_links(void *P, const void *X_e, const void *X_o, const void *Y_e, const void *Y_o,
                              const void *UR, const void *U, const Geom &g, int N, int rep, double scale,
                              int accumulate, hipStream_t st) {
  switch (N) {
    case 2: return force_n<2>(P, X_e, X_o, Y_e, Y_o, UR, U, g, rep, scale, accumulate, st);
    case 3: return force_n<3>(P, X_e, X_o, Y_e, Y_o, UR, U, g, rep, scale, accumulate, st);
    case 4: return force_n<4>(P, X_e, X_o, Y_e, Y_o, UR, U, g, rep, scale, accumulate, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace wd
