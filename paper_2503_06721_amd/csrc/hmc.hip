// Gauge-field pieces of the HMC molecular dynamics (Sec. 5.2, 5.3), on the
// caller's canonical fundamental links U [T][X][Y][Z][4][N][N] and momenta pi
// of the same layout (Hermitian traceless matrices pi = pi^a T^a):
//  * Wilson plaquette action S_g = beta sum_x sum_{mu<nu} (1 - Re tr P / N),
//  * its force F = sum_a (dS_g/dw^a) T^a for U -> exp(i w^a T^a) U,
//    dS_g/dw^a_mu(x) = (beta/N) Im tr(T^a U_mu(x) A_mu(x)), A the staple sum,
//    which with B = (M - M^+)/(2i), M = U A, is (beta/N) (B - tr B / N)/2,
//  * the link update U <- exp(i eps pi) U and the kinetic term sum tr(pi^2).
#include "wd_common.h"
#include "wd_kernels.h"

namespace wd {

template <int N>
struct Mat {
  cplx<double> a[N][N];
};

template <int N>
__device__ __forceinline__ Mat<N> ld_mat(const cplx<double> *p, bool dag) {
  Mat<N> m;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const cplx<double> v = p[dag ? j * N + i : i * N + j];
      m.a[i][j] = dag ? mk(v.re, -v.im) : v;
    }
  return m;
}

template <int N>
__device__ __forceinline__ Mat<N> mul(const Mat<N> &x, const Mat<N> &y) {
  Mat<N> r;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      cplx<double> s = mk(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < N; ++k) s = cfma(x.a[i][k], y.a[k][j], s);
      r.a[i][j] = s;
    }
  return r;
}

__device__ __forceinline__ size_t lex_shift(const Geom &g, size_t lex, int mu, int step) {
  size_t r = lex;
  int c[4];
  c[3] = (int)(r % g.Z); r /= g.Z;
  c[2] = (int)(r % g.Y); r /= g.Y;
  c[1] = (int)(r % g.X);
  c[0] = (int)(r / g.X);
  const int L[4] = {g.T, g.X, g.Y, g.Z};
  c[mu] = (c[mu] + step + L[mu]) % L[mu];
  return (((size_t)c[0] * g.X + c[1]) * g.Y + c[2]) * g.Z + c[3];
}

template <int N>
__device__ __forceinline__ const cplx<double> *link(const cplx<double> *U, size_t lex, int mu) {
  return U + (lex * 4 + mu) * N * N;
}

// Thread per link (lex, mu): F = scale * (beta/N) (B - tr B/N)/2 (+ F).
template <int N>
__global__ __launch_bounds__(256) void k_gauge_force(const cplx<double> *__restrict__ U, cplx<double> *F, Geom g,
                                                     double beta, double scale, int accumulate) {
  const size_t V = 2 * (size_t)g.Vh;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= 4 * V) return;
  const size_t x = gid >> 2;
  const int mu = (int)(gid & 3);
  Mat<N> A;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) A.a[i][j] = mk(0.0, 0.0);
  const size_t xp = lex_shift(g, x, mu, 1);
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    // upper: U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
    const size_t xn = lex_shift(g, x, nu, 1);
    Mat<N> s = mul<N>(mul<N>(ld_mat<N>(link<N>(U, xp, nu), false), ld_mat<N>(link<N>(U, xn, mu), true)),
                      ld_mat<N>(link<N>(U, x, nu), true));
    // lower: U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)
    const size_t xm = lex_shift(g, x, nu, -1);
    const size_t xpm = lex_shift(g, xp, nu, -1);
    Mat<N> l = mul<N>(mul<N>(ld_mat<N>(link<N>(U, xpm, nu), true), ld_mat<N>(link<N>(U, xm, mu), true)),
                      ld_mat<N>(link<N>(U, xm, nu), false));
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) A.a[i][j] = A.a[i][j] + s.a[i][j] + l.a[i][j];
  }
  const Mat<N> M = mul<N>(ld_mat<N>(link<N>(U, x, mu), false), A);
  // B = (M - M^+)/(2i): B_ij = (M_ij - conj(M_ji)) / (2i)
  Mat<N> B;
  double trB = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const double re = M.a[i][j].re - M.a[j][i].re, im = M.a[i][j].im + M.a[j][i].im;
      B.a[i][j] = mk(0.5 * im, -0.5 * re);
      if (i == j) trB += 0.5 * im;
    }
  const double c = scale * beta / N * 0.5;
  cplx<double> *out = F + gid * N * N;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      cplx<double> v = B.a[i][j];
      if (i == j) v.re -= trB / N;
      v = c * v;
      if (accumulate) v = v + out[i * N + j];
      out[i * N + j] = v;
    }
}

// Per-site sum of Re tr P_mu,nu / N over the six planes; block partial sums.
template <int N>
__global__ __launch_bounds__(256) void k_plaquette_partial(const cplx<double> *__restrict__ U, double *partial,
                                                           Geom g) {
  __shared__ double sh[4];
  const size_t V = 2 * (size_t)g.Vh;
  const size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (x < V) {
    for (int mu = 0; mu < 4; ++mu) {
      const size_t xm = lex_shift(g, x, mu, 1);
      for (int nu = mu + 1; nu < 4; ++nu) {
        const size_t xn = lex_shift(g, x, nu, 1);
        const Mat<N> P = mul<N>(mul<N>(ld_mat<N>(link<N>(U, x, mu), false), ld_mat<N>(link<N>(U, xm, nu), false)),
                                mul<N>(ld_mat<N>(link<N>(U, xn, mu), true), ld_mat<N>(link<N>(U, x, nu), true)));
        double tr = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) tr += P.a[i][i].re;
        s += tr / N;
      }
    }
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Thread per link: U <- exp(i eps pi) U, the exponential by scaling and
// squaring of its Taylor series (degree 16 after scaling below 1/4).
template <int N>
__global__ __launch_bounds__(256) void k_link_update(cplx<double> *U, const cplx<double> *__restrict__ pi, Geom g,
                                                     double eps) {
  const size_t V = 2 * (size_t)g.Vh;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= 4 * V) return;
  Mat<N> X;   // i eps pi
  double nrm = 0.0;
  const cplx<double> *p = pi + gid * N * N;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double rs = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const cplx<double> v = p[i * N + j];
      X.a[i][j] = mk(-eps * v.im, eps * v.re);
      rs += sqrt(v.re * v.re + v.im * v.im);
    }
    nrm = rs > nrm ? rs : nrm;
  }
  nrm *= fabs(eps);
  int sq = 0;
  while (nrm > 0.25 && sq < 40) {
    nrm *= 0.5;
    ++sq;
  }
  const double sc = ldexp(1.0, -sq);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) X.a[i][j] = sc * X.a[i][j];
  Mat<N> E;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) E.a[i][j] = mk(i == j ? 1.0 : 0.0, 0.0);
  for (int k = 16; k >= 1; --k) {   // Horner: E = I + X E / k
    Mat<N> T = mul<N>(X, E);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) E.a[i][j] = (1.0 / k) * T.a[i][j] + mk(i == j ? 1.0 : 0.0, 0.0);
  }
  for (int q = 0; q < sq; ++q) E = mul<N>(E, E);
  cplx<double> *u = U + gid * N * N;
  const Mat<N> Un = mul<N>(E, ld_mat<N>(u, false));
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) u[i * N + j] = Un.a[i][j];
}

// Block partial sums of sum_links tr(pi^2) = sum |pi_ij|^2 (pi Hermitian).
__global__ __launch_bounds__(256) void k_kinetic_partial(const cplx<double> *__restrict__ pi, double *partial,
                                                         size_t nlinks, int n2) {
  __shared__ double sh[4];
  const size_t l = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (l < nlinks)
    for (int e = 0; e < n2; ++e) {
      const cplx<double> v = pi[l * n2 + e];
      s += v.re * v.re + v.im * v.im;
    }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// pi = sum_a w^a T^a (generators of wd_rep.h's basis: off-diagonal pairs
// (symmetric, antisymmetric) in lexicographic order, then the diagonals).
template <int N>
__global__ __launch_bounds__(256) void k_algebra(cplx<double> *pi, const double *__restrict__ w, size_t nlinks) {
  const size_t l = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nlinks) return;
  constexpr int NA = N * N - 1;
  const double *wl = w + l * NA;
  cplx<double> m[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) m[i][j] = mk(0.0, 0.0);
  int a = 0;
  for (int j = 0; j < N; ++j)
    for (int k = j + 1; k < N; ++k) {
      // (E_jk + E_kj)/2 and (-i E_jk + i E_kj)/2
      const double s = 0.5 * wl[a], t = 0.5 * wl[a + 1];
      m[j][k] = mk(s, -t);
      m[k][j] = mk(s, t);
      a += 2;
    }
  for (int kk = 1; kk < N; ++kk) {
    const double c = wl[a++] / sqrt(2.0 * kk * (kk + 1));
    for (int i = 0; i < kk; ++i) m[i][i].re += c;
    m[kk][kk].re -= kk * c;
  }
  cplx<double> *o = pi + l * N * N;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) o[i * N + j] = m[i][j];
}

// ------------------------------------------------------------------ launch
template <int N>
static hipError_t gf_launch(const void *U, void *F, const Geom &g, double beta, double scale, int accumulate,
                            hipStream_t st) {
  const size_t n = 8 * (size_t)g.Vh;
  hipLaunchKernelGGL(k_gauge_force<N>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     (const cplx<double> *)U, (cplx<double> *)F, g, beta, scale, accumulate);
  return hipGetLastError();
}

hipError_t launch_gauge_force(const void *U, void *F, const Geom &g, int N, double beta, double scale,
                              int accumulate, hipStream_t st) {
  switch (N) {
    case 2: return gf_launch<2>(U, F, g, beta, scale, accumulate, st);
    case 3: return gf_launch<3>(U, F, g, beta, scale, accumulate, st);
    case 4: return gf_launch<4>(U, F, g, beta, scale, accumulate, st);
  }
  return hipErrorInvalidValue;
}

int plaquette_blocks(const Geom &g) { return (int)((2 * (size_t)g.Vh + 255) / 256); }

hipError_t launch_plaquette_partial(const void *U, double *partial, const Geom &g, int N, hipStream_t st) {
  const dim3 grid(plaquette_blocks(g));
  switch (N) {
    case 2: hipLaunchKernelGGL(k_plaquette_partial<2>, grid, dim3(256), 0, st, (const cplx<double> *)U, partial, g);
      return hipGetLastError();
    case 3: hipLaunchKernelGGL(k_plaquette_partial<3>, grid, dim3(256), 0, st, (const cplx<double> *)U, partial, g);
      return hipGetLastError();
    case 4: hipLaunchKernelGGL(k_plaquette_partial<4>, grid, dim3(256), 0, st, (const cplx<double> *)U, partial, g);
      return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

hipError_t launch_link_update(void *U, const void *pi, const Geom &g, int N, double eps, hipStream_t st) {
  const size_t n = 8 * (size_t)g.Vh;
  const dim3 grid((unsigned)((n + 255) / 256));
  switch (N) {
    case 2: hipLaunchKernelGGL(k_link_update<2>, grid, dim3(256), 0, st, (cplx<double> *)U, (const cplx<double> *)pi,
                               g, eps);
      return hipGetLastError();
    case 3: hipLaunchKernelGGL(k_link_update<3>, grid, dim3(256), 0, st, (cplx<double> *)U, (const cplx<double> *)pi,
                               g, eps);
      return hipGetLastError();
    case 4: hipLaunchKernelGGL(k_link_update<4>, grid, dim3(256), 0, st, (cplx<double> *)U, (const cplx<double> *)pi,
                               g, eps);
      return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

int kinetic_blocks(const Geom &g) { return (int)((8 * (size_t)g.Vh + 255) / 256); }

hipError_t launch_kinetic_partial(const void *pi, double *partial, const Geom &g, int N, hipStream_t st) {
  const size_t nl = 8 * (size_t)g.Vh;
  hipLaunchKernelGGL(k_kinetic_partial, dim3(kinetic_blocks(g)), dim3(256), 0, st, (const cplx<double> *)pi, partial,
                     nl, N * N);
  return hipGetLastError();
}

hipError_t launch_algebra(void *pi, const double *w, const Geom &g, int N, hipStream_t st) {
  const size_t nl = 8 * (size_t)g.Vh;
  const dim3 grid((unsigned)((nl + 255) / 256));
  switch (N) {
    case 2: hipLaunchKernelGGL(k_algebra<2>, grid, dim3(256), 0, st, (cplx<double> *)pi, w, nl);
      return hipGetLastError();
    case 3: hipLaunchKernelGGL(k_algebra<3>, grid, dim3(256), 0, st, (cplx<double> *)pi, w, nl);
      return hipGetLastError();
    case 4: hipLaunchKernelGGL(k_algebra<4>, grid, dim3(256), 0, st, (cplx<double> *)pi, w, nl);
      return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

}  // namespace wd
