// Clover improvement (Sec. 6.1.2; exponential form Sec. 6.1.3): the site-diagonal blocks
//   D_ee + D_oo = (4 + m) + c_sw (i/4) sum_{mu,nu} sigma_mu,nu F_mu,nu
// (or, exponential form, (4 + m) exp(c_sw/(4+m) (i/4) sum sigma F)), with
// F_mu,nu = (Q_mu,nu - Q_mu,nu^+)/8 and Q the sum of the four clover leaves of
// the (mu, nu) plane at x, all starting at x and turning from mu to nu.
//
// The leaves are products of fundamental links (N x N); each leaf is mapped to
// the fermion representation entry by entry (wd_rep.h), which is far cheaper
// than multiplying d_R x d_R represented links.  Since R(L)^+ = R(L^+),
//   F_R = sum_leaves (R(L) - R(L)^+) / 8.
// sigma_mu,nu = (i/2)[gamma_mu, gamma_nu] commutes with gamma_5 =
// diag(1,1,-1,-1), so each site holds two 2d x 2d chirality blocks (spins
// {0,1} and {2,3}).  Stored per parity: the even sites keep the blocks
// (D_ee), the odd sites their inverses (D_oo^{-1}), which is what the
// even-odd operator D-hat = D_ee - D_eo D_oo^{-1} D_oe applies.  All these
// blocks are Hermitian, so only the upper triangle (row-major, diagonal
// included: 2d(2d+1)/2 complex entries) is stored.
#include "wd_common.h"
#include "wd_kernels.h"
#include "wd_rep.h"

namespace wd {

// Plane p = 0..5 <-> (mu, nu) = (0,1) (0,2) (0,3) (1,2) (1,3) (2,3).
__device__ __forceinline__ void plane_dirs(int p, int &mu, int &nu) {
  mu = p < 3 ? 0 : p < 5 ? 1 : 2;
  nu = p < 3 ? p + 1 : p < 5 ? p - 1 : 3;
}

// Position of entry (i, j), i <= j, of the packed upper triangle of an
// NB x NB Hermitian block; entry (j, i) is its conjugate.
__host__ __device__ constexpr int tri_index(int NB, int i, int j) { return i * NB - i * (i - 1) / 2 + (j - i); }

// Entry (i, j) of a packed Hermitian block (any i, j).
template <typename T>
__device__ __forceinline__ cplx<T> herm_entry(const cplx<T> *P, size_t es, int NB, int i, int j) {
  if (i <= j) return P[(size_t)tri_index(NB, i, j) * es];
  const cplx<T> v = P[(size_t)tri_index(NB, j, i) * es];
  return mk<T>(v.re, -v.im);
}

// Workgroups are dispatched to the 8 XCDs round-robin; block b is given the
// logical index that makes each XCD's blocks one contiguous range, so that
// consecutive logical blocks (the planes or directions of one site chunk)
// run on the same XCD and share its L2 (the leaf and gather kernels; the F
// kernel is faster without it).
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned n) {
  const unsigned q = n >> 3, rmd = n & 7, x = b & 7, j = b >> 3;
  return x * q + (x < rmd ? x : rmd) + j;
}

// Sites c + a e_lo + b e_hi (|a|, |b| <= 1) around one site in the plane
// (lo, hi), lexicographic: only the two coordinates that move are wrapped,
// by compare and select (no integer division).
struct PlaneNb {
  long long base, slo, shi;
  int clo, chi, Llo, Lhi;
  __device__ __forceinline__ static long long pick(int i, long long v0, long long v1, long long v2, long long v3) {
    return i == 0 ? v0 : i == 1 ? v1 : i == 2 ? v2 : v3;
  }
  __device__ __forceinline__ PlaneNb(const Geom &g, const int (&c)[4], size_t lex, int lo, int hi) {
    const long long sz = g.Z, sy = (long long)g.Y * g.Z, sx = sy * g.X;
    base = (long long)lex;
    slo = pick(lo, sx, sy, sz, 1);
    shi = pick(hi, sx, sy, sz, 1);
    clo = (int)pick(lo, c[0], c[1], c[2], c[3]);
    chi = (int)pick(hi, c[0], c[1], c[2], c[3]);
    Llo = (int)pick(lo, g.T, g.X, g.Y, g.Z);
    Lhi = (int)pick(hi, g.T, g.X, g.Y, g.Z);
  }
  __device__ __forceinline__ size_t at(int a, int b) const {
    const int qa = clo + a, qb = chi + b;
    const int da = qa < 0 ? a + Llo : qa >= Llo ? a - Llo : a;
    const int db = qb < 0 ? b + Lhi : qb >= Lhi ? b - Lhi : b;
    return (size_t)(base + da * slo + db * shi);
  }
};

// The clover kernels read the fundamental links from a structure-of-arrays
// copy Us[mu][N*N][V] (lexicographic site minor; k_links_soa), so that the
// lanes of a wavefront, on consecutive sites, read consecutive addresses.
template <int N>
__device__ __forceinline__ void load_link(cplx<double> (&u)[N][N], const cplx<double> *Us, size_t V, size_t lex,
                                          int mu, bool dag) {
  const cplx<double> *p = Us + (size_t)mu * N * N * V + lex;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const cplx<double> v = p[(size_t)(dag ? j * N + i : i * N + j) * V];
      u[i][j] = dag ? mk(v.re, -v.im) : v;
    }
}

// Us[mu][e][lex] = U[lex][mu][e] (canonical [T][X][Y][Z][4][N][N] complex).
// A block transposes 64 sites through LDS: the 64 x 4 N^2 entries are read in
// canonical order (consecutive threads, consecutive addresses) and written
// per (mu, e) as a run of 64 consecutive sites.
template <int N>
__global__ __launch_bounds__(256) void k_links_soa(const cplx<double> *__restrict__ U, cplx<double> *__restrict__ Us,
                                                   size_t V) {
  constexpr int E = 4 * N * N;   // complex entries per site
  constexpr int S = E + 1;       // LDS row, padded against bank conflicts
  __shared__ cplx<double> t[64 * S];
  const size_t s0 = (size_t)blockIdx.x * 64;
  const int ns = V - s0 < 64 ? (int)(V - s0) : 64;
  const cplx<double> *src = U + s0 * E;
  for (int k = threadIdx.x; k < ns * E; k += 256) t[(k / E) * S + k % E] = src[k];
  __syncthreads();
  for (int k = threadIdx.x; k < 64 * E; k += 256) {
    const int j = k >> 6, site = k & 63;   // j = mu N^2 + e
    if (site < ns) Us[(size_t)j * V + s0 + site] = t[site * S + j];
  }
}

template <int N>
static hipError_t links_soa_launch(const void *U, double *Us, const Geom &g, hipStream_t st) {
  const size_t V = 2 * (size_t)g.Vh;
  hipLaunchKernelGGL((k_links_soa<N>), dim3((unsigned)((V + 63) / 64)), dim3(256), 0, st,
                     (const cplx<double> *)U, (cplx<double> *)Us, V);
  return hipGetLastError();
}

// acc = acc * u
template <int N>
__device__ __forceinline__ void mul_right(cplx<double> (&acc)[N][N], const cplx<double> (&u)[N][N]) {
  cplx<double> r[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      cplx<double> s = mk(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < N; ++k) s = cfma(acc[i][k], u[k][j], s);
      r[i][j] = s;
    }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) acc[i][j] = r[i][j];
}

// Leaf k of plane (mu, nu) at x as four (site offset (a_mu, b_nu), direction,
// dagger) factors.
struct LeafStep {
  signed char a, b, dir, dag;   // dir 0 = mu, 1 = nu
};
// Used in loops unrolled over (leaf, step), so that every lookup folds into a
// constant.
__device__ constexpr LeafStep kLeafC[4][4] = {
    // U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
    {{0, 0, 0, 0}, {1, 0, 1, 0}, {0, 1, 0, 1}, {0, 0, 1, 1}},
    // U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu)
    {{0, 0, 1, 0}, {-1, 1, 0, 1}, {-1, 0, 1, 1}, {-1, 0, 0, 0}},
    // U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
    {{-1, 0, 0, 1}, {-1, -1, 1, 1}, {-1, -1, 0, 0}, {0, -1, 1, 0}},
    // U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^+
    {{0, -1, 1, 1}, {0, -1, 0, 0}, {1, -1, 1, 0}, {0, 0, 0, 1}},
};

// F scratch: F[p][A][B] of every site, [6][D][D][V] complex FP64.  Thread per
// (plane, site), consecutive threads on consecutive sites.
template <int N, int REP>
__global__ __launch_bounds__(256) void k_clover_F(const cplx<double> *__restrict__ U, cplx<double> *__restrict__ F,
                                                  Geom g) {
  constexpr int D = rep_dim(N, REP);
  const size_t V = 2 * (size_t)g.Vh;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  // 64-site chunks, the six planes of a chunk in consecutive wavefronts (the
  // planes that share a link direction read it close together in time)
  const size_t chunk = gid / 384;
  const int r6 = (int)(gid - chunk * 384);
  const int p = r6 >> 6;
  const size_t lex = chunk * 64 + (r6 & 63);
  if (lex >= V) return;
  int mu, nu;
  plane_dirs(p, mu, nu);
  size_t r = lex;
  int c[4];
  c[3] = (int)(r % g.Z); r /= g.Z;
  c[2] = (int)(r % g.Y); r /= g.Y;
  c[1] = (int)(r % g.X);
  c[0] = (int)(r / g.X);
  const PlaneNb pn(g, c, lex, mu, nu);
  cplx<double> *Fp = F + (size_t)p * D * D * V + lex;
  if constexpr (REP == 0) {
    // fundamental representation (R = 1): the four leaves summed in
    // registers, F = (Q - Q^+)/8 written once (the other representations
    // accumulate (R(L) - R(L)^+)/8 leaf by leaf in F below: their d_R^2
    // accumulators do not fit in registers beside the leaf products)
    constexpr bool FUND = true;
    constexpr int DA = FUND ? N : D;
    cplx<double> acc[DA][DA];
#pragma unroll
    for (int A = 0; A < DA; ++A)
#pragma unroll
      for (int B = 0; B < DA; ++B) acc[A][B] = mk(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      cplx<double> L[N][N];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const LeafStep st = kLeafC[k][f];
        cplx<double> u[N][N];
        load_link<N>(u, U, V, pn.at(st.a, st.b), st.dir ? nu : mu, st.dag != 0);
        if (f == 0) {
#pragma unroll
          for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = 0; j < N; ++j) L[i][j] = u[i][j];
        } else {
          mul_right<N>(L, u);
        }
      }
#pragma unroll
      for (int A = 0; A < DA; ++A)
#pragma unroll
        for (int B = 0; B < DA; ++B) {
          if constexpr (FUND) {
            acc[A][B] = acc[A][B] + L[A][B];
          } else {
            const cplx<double> rab = rep_entry<N, REP>(L, A, B), rba = rep_entry<N, REP>(L, B, A);
            acc[A][B] = acc[A][B] + mk(rab.re - rba.re, rab.im + rba.im);
          }
        }
      // one leaf's links live at a time
      __builtin_amdgcn_sched_barrier(0);
    }
    // F = (Q - Q^+)/8 (fundamental), or the sum of (R(L) - R(L)^+)/8
#pragma unroll
    for (int A = 0; A < DA; ++A)
#pragma unroll
      for (int B = 0; B < DA; ++B) {
        const cplx<double> v = FUND ? mk(0.125 * (acc[A][B].re - acc[B][A].re), 0.125 * (acc[A][B].im + acc[B][A].im))
                                    : 0.125 * acc[A][B];
        Fp[(size_t)(A * D + B) * V] = v;
      }
    return;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    cplx<double> L[N][N];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const LeafStep s = kLeafC[k][f];
      cplx<double> u[N][N];
      load_link<N>(u, U, V, pn.at(s.a, s.b), s.dir ? nu : mu, s.dag != 0);
      if (f == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
          for (int j = 0; j < N; ++j) L[i][j] = u[i][j];
      } else {
        mul_right<N>(L, u);
      }
    }
    // F += (R(L) - R(L)^+) / 8
    for (int A = 0; A < D; ++A)
      for (int B = 0; B < D; ++B) {
        const cplx<double> rab = rep_entry<N, REP>(L, A, B), rba = rep_entry<N, REP>(L, B, A);
        cplx<double> v = mk(0.125 * (rab.re - rba.re), 0.125 * (rab.im + rba.im));
        const size_t o = (size_t)(A * D + B) * V;
        if (k > 0) v = v + Fp[o];
        Fp[o] = v;
      }
  }
}

// sigma blocks: S.v[p][c][s][t] = 2 x (chirality block c of sigma_mu,nu)_st for
// plane p (the factor 2 counts the (nu, mu) term of the sum).
struct SigmaBlocks {
  cplx<double> v[6][2][2][2];
};

// Gauss-Jordan inverse with partial pivoting of the n x n matrix a (destroyed).
template <int NB>
__device__ void invert(cplx<double> (&a)[NB][NB], cplx<double> (&inv)[NB][NB]) {
  for (int i = 0; i < NB; ++i)
    for (int j = 0; j < NB; ++j) inv[i][j] = mk(i == j ? 1.0 : 0.0, 0.0);
  for (int col = 0; col < NB; ++col) {
    int piv = col;
    double best = a[col][col].re * a[col][col].re + a[col][col].im * a[col][col].im;
    for (int r = col + 1; r < NB; ++r) {
      const double m2 = a[r][col].re * a[r][col].re + a[r][col].im * a[r][col].im;
      if (m2 > best) {
        best = m2;
        piv = r;
      }
    }
    if (piv != col)
      for (int j = 0; j < NB; ++j) {
        const cplx<double> t1 = a[col][j], t2 = inv[col][j];
        a[col][j] = a[piv][j];
        inv[col][j] = inv[piv][j];
        a[piv][j] = t1;
        inv[piv][j] = t2;
      }
    const cplx<double> d = a[col][col];
    const double dn = 1.0 / (d.re * d.re + d.im * d.im);
    const cplx<double> di = mk(d.re * dn, -d.im * dn);
    for (int j = 0; j < NB; ++j) {
      a[col][j] = cmul(a[col][j], di);
      inv[col][j] = cmul(inv[col][j], di);
    }
    for (int r = 0; r < NB; ++r) {
      if (r == col) continue;
      const cplx<double> f = a[r][col];
      for (int j = 0; j < NB; ++j) {
        a[r][j] = a[r][j] - cmul(f, a[col][j]);
        inv[r][j] = inv[r][j] - cmul(f, inv[col][j]);
      }
    }
  }
}

// e = exp(a) by scaling and squaring of the Taylor series (a destroyed).
template <int NB>
__device__ void expm(cplx<double> (&a)[NB][NB], cplx<double> (&e)[NB][NB]) {
  double nrm = 0.0;   // max column sum
  for (int j = 0; j < NB; ++j) {
    double s = 0.0;
    for (int i = 0; i < NB; ++i) s += sqrt(a[i][j].re * a[i][j].re + a[i][j].im * a[i][j].im);
    nrm = s > nrm ? s : nrm;
  }
  int sq = 0;
  while (nrm > 0.25 && sq < 60) {
    nrm *= 0.5;
    ++sq;
  }
  const double sc = ldexp(1.0, -sq);
  for (int i = 0; i < NB; ++i)
    for (int j = 0; j < NB; ++j) a[i][j] = sc * a[i][j];
  // Horner: e = I + a (I + a/2 (I + a/3 (... (I + a/K))))
  // (||a|| <= 1/4: the first dropped term is below 0.25^13 / 13! ~ 2e-18)
  constexpr int K = 12;
  cplx<double> t[NB][NB];
  for (int i = 0; i < NB; ++i)
    for (int j = 0; j < NB; ++j) e[i][j] = mk(i == j ? 1.0 : 0.0, 0.0);
  for (int k = K; k >= 1; --k) {
    for (int i = 0; i < NB; ++i)
      for (int j = 0; j < NB; ++j) {
        cplx<double> s = mk(0.0, 0.0);
        for (int l = 0; l < NB; ++l) s = cfma(a[i][l], e[l][j], s);
        t[i][j] = (1.0 / k) * s;
      }
    for (int i = 0; i < NB; ++i)
      for (int j = 0; j < NB; ++j) e[i][j] = t[i][j] + mk(i == j ? 1.0 : 0.0, 0.0);
  }
  for (int q = 0; q < sq; ++q) {
    for (int i = 0; i < NB; ++i)
      for (int j = 0; j < NB; ++j) {
        cplx<double> s = mk(0.0, 0.0);
        for (int l = 0; l < NB; ++l) s = cfma(e[i][l], e[l][j], s);
        t[i][j] = s;
      }
    for (int i = 0; i < NB; ++i)
      for (int j = 0; j < NB; ++j) e[i][j] = t[i][j];
  }
}

// Thread per (site, chirality block c): assemble the block from F, add the
// mass term (or exponentiate), invert on odd sites, store in precision T.
// Clover field layout: [parity][c][row][col][stride] complex.
template <int D, typename T>
__global__ __launch_bounds__(64) void k_clover_finish(const cplx<double> *__restrict__ F, void *__restrict__ clov,
                                                      Geom g, SigmaBlocks S, double m0, double csw, int expo) {
  constexpr int NB = 2 * D;
  const size_t V = 2 * (size_t)g.Vh;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= 2 * V) return;
  const int c = (int)(gid / V);
  const size_t lex = gid - (size_t)c * V;
  size_t r = lex;
  const int z = (int)(r % g.Z); r /= g.Z;
  const int y = (int)(r % g.Y); r /= g.Y;
  const int x = (int)(r % g.X);
  const int t = (int)(r / g.X);
  const int par = (t + x + y + z) & 1;
  const size_t cb = lex >> 1;
  cplx<double> M[NB][NB];
  // (i/4) c_sw sum_p S[p][c][s][t] F_p[a][b]
  for (int s = 0; s < 2; ++s)
    for (int a = 0; a < D; ++a)
      for (int tt = 0; tt < 2; ++tt)
        for (int b = 0; b < D; ++b) {
          cplx<double> acc = mk(0.0, 0.0);
          for (int p = 0; p < 6; ++p) acc = cfma(S.v[p][c][s][tt], F[((size_t)p * D * D + a * D + b) * V + lex], acc);
          M[s * D + a][tt * D + b] = mk(-0.25 * csw * acc.im, 0.25 * csw * acc.re);   // (i/4) c_sw acc
        }
  cplx<double> out[NB][NB];
  const double m4 = 4.0 + m0;
  if (!expo) {
    for (int i = 0; i < NB; ++i) M[i][i].re += m4;
    if (par == 0) {
      for (int i = 0; i < NB; ++i)
        for (int j = 0; j < NB; ++j) out[i][j] = M[i][j];
    } else {
      invert<NB>(M, out);
    }
  } else {
    // even: (4+m) exp(M/(4+m)); odd: exp(-M/(4+m))/(4+m)
    const double f = (par == 0 ? 1.0 : -1.0) / m4;
    for (int i = 0; i < NB; ++i)
      for (int j = 0; j < NB; ++j) M[i][j] = f * M[i][j];
    expm<NB>(M, out);
    const double sc = par == 0 ? m4 : 1.0 / m4;
    for (int i = 0; i < NB; ++i)
      for (int j = 0; j < NB; ++j) out[i][j] = sc * out[i][j];
  }
  constexpr int NT = NB * (NB + 1) / 2;
  cplx<T> *dst = static_cast<cplx<T> *>(clov) + ((size_t)(par * 2 + c) * NT) * g.stride + cb;
  for (int i = 0; i < NB; ++i)
    for (int j = i; j < NB; ++j) {
      // the computed block is Hermitian up to rounding: store the mean of (i,j) and conj(j,i)
      const double re = 0.5 * (out[i][j].re + out[j][i].re), im = 0.5 * (out[i][j].im - out[j][i].im);
      dst[(size_t)tri_index(NB, i, j) * g.stride] = mk<T>((T)re, (T)(i == j ? 0.0 : im));
    }
}

// In-place Gauss-Jordan inverse with partial pivoting of the NB x NB matrix
// a, every index a compile-time constant so that the matrix stays in
// registers: the row interchange of a step is a set of selects over the rows
// below the diagonal, and the interchanges are undone at the end as column
// interchanges in reverse order (A^-1 = (P A)^-1 P).
template <int NB>
__device__ __forceinline__ void invert_in_place(cplx<double> (&a)[NB][NB]) {
  int piv[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    int p = k;
    double best = a[k][k].re * a[k][k].re + a[k][k].im * a[k][k].im;
#pragma unroll
    for (int r = k + 1; r < NB; ++r) {
      const double m2 = a[r][k].re * a[r][k].re + a[r][k].im * a[r][k].im;
      p = m2 > best ? r : p;
      best = m2 > best ? m2 : best;
    }
    piv[k] = p;
#pragma unroll
    for (int r = k + 1; r < NB; ++r) {
      const bool sw = p == r;
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const cplx<double> tk = a[k][j], tr = a[r][j];
        a[k][j] = sw ? tr : tk;
        a[r][j] = sw ? tk : tr;
      }
    }
    const cplx<double> d = a[k][k];
    const double dn = 1.0 / (d.re * d.re + d.im * d.im);
    const cplx<double> di = mk(d.re * dn, -d.im * dn);
    a[k][k] = mk(1.0, 0.0);
#pragma unroll
    for (int j = 0; j < NB; ++j) a[k][j] = cmul(a[k][j], di);
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      if (r == k) continue;
      const cplx<double> f = a[r][k];
      a[r][k] = mk(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < NB; ++j) a[r][j] = a[r][j] - cmul(f, a[k][j]);
    }
  }
#pragma unroll
  for (int k = NB - 1; k >= 0; --k) {
#pragma unroll
    for (int r = k + 1; r < NB; ++r) {
      const bool sw = piv[k] == r;
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const cplx<double> tk = a[i][k], tr = a[i][r];
        a[i][k] = sw ? tr : tk;
        a[i][r] = sw ? tk : tr;
      }
    }
  }
}

// Regular clover (no exponential), d_R <= 4: as k_clover_finish with the
// block in registers throughout.  Thread per (site, chirality block), the
// block index fastest, so that the two threads of a site read the same F
// entries together (F comes from HBM once).
template <int D, typename T>
__global__ __launch_bounds__(64) void k_clover_finish_reg(const cplx<double> *__restrict__ F, void *__restrict__ clov,
                                                          Geom g, SigmaBlocks S, double m0, double csw) {
  constexpr int NB = 2 * D;
  const size_t V = 2 * (size_t)g.Vh;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= 2 * V) return;
  const int c = (int)(gid & 1);
  const size_t lex = gid >> 1;
  size_t r = lex;
  const int z = (int)(r % g.Z); r /= g.Z;
  const int y = (int)(r % g.Y); r /= g.Y;
  const int x = (int)(r % g.X);
  const int t = (int)(r / g.X);
  const int par = (t + x + y + z) & 1;
  const size_t cb = lex >> 1;
  cplx<double> M[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) M[i][j] = mk(0.0, 0.0);
  // (i/4) c_sw sum_p S[p][c][s][t] F_p[a][b], plane by plane
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    cplx<double> fp[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) fp[a][b] = F[((size_t)p * D * D + a * D + b) * V + lex];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
      for (int tt = 0; tt < 2; ++tt) {
        const cplx<double> sv = S.v[p][c][s2][tt];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int b = 0; b < D; ++b) M[s2 * D + a][tt * D + b] = cfma(sv, fp[a][b], M[s2 * D + a][tt * D + b]);
      }
    // one plane's F entries live at a time
    __builtin_amdgcn_sched_barrier(0);
  }
  const double m4 = 4.0 + m0;
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const cplx<double> v = M[i][j];
      M[i][j] = mk(-0.25 * csw * v.im + (i == j ? m4 : 0.0), 0.25 * csw * v.re);   // (i/4) c_sw acc (+ 4 + m)
    }
  if (par == 1) invert_in_place<NB>(M);
  constexpr int NT = NB * (NB + 1) / 2;
  cplx<T> *dst = static_cast<cplx<T> *>(clov) + ((size_t)(par * 2 + c) * NT) * g.stride + cb;
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = i; j < NB; ++j) {
      // Hermitian up to rounding: store the mean of (i,j) and conj(j,i)
      const double re = 0.5 * (M[i][j].re + M[j][i].re), im = 0.5 * (M[i][j].im - M[j][i].im);
      dst[(size_t)tri_index(NB, i, j) * g.stride] = mk<T>((T)re, (T)(i == j ? 0.0 : im));
    }
}

// out = M_c in on the sites of `parity` (thread per (site, rhs, block); the
// thread reads its block's spin components before writing them, so out may
// alias in).
template <int D, typename T>
__global__ __launch_bounds__(256) void k_clover_apply(cplx<T> *out, const cplx<T> *in, const cplx<T> *__restrict__ clov,
                                                      Geom g, int parity, int nrhs) {
  constexpr int NB = 2 * D;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int rc = blockIdx.y;   // rhs * 2 + block
  const int rr = rc >> 1, c = rc & 1;
  if (i >= g.Vh || rr >= nrhs) return;
  const size_t rbase = (size_t)rr * 4 * D * g.stride + i;
  cplx<T> v[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) v[k] = in[rbase + (size_t)(2 * c * D + k) * g.stride];
  constexpr int NT = NB * (NB + 1) / 2;
  const cplx<T> *M = clov + ((size_t)(parity * 2 + c) * NT) * g.stride + i;
  cplx<T> w[NB];
#pragma unroll
  for (int a = 0; a < NB; ++a) w[a] = mk<T>(0, 0);
  // each stored entry (a, b), a <= b, serves (a, b) and, conjugated, (b, a)
#pragma unroll
  for (int a = 0; a < NB; ++a) {
    const cplx<T> d = M[(size_t)tri_index(NB, a, a) * g.stride];
    w[a] = cfma(d, v[a], w[a]);
#pragma unroll
    for (int b = a + 1; b < NB; ++b) {
      const cplx<T> m = M[(size_t)tri_index(NB, a, b) * g.stride];
      w[a] = cfma(m, v[b], w[a]);
      w[b] = cfma_conj(m, v[a], w[b]);
    }
  }
#pragma unroll
  for (int k = 0; k < NB; ++k) out[rbase + (size_t)(2 * c * D + k) * g.stride] = w[k];
}

// ------------------------------------------------------------------ launch
template <int N, int REP>
static hipError_t F_launch(const void *U, double *F, const Geom &g, hipStream_t st) {
  const size_t n = 384 * ((2 * (size_t)g.Vh + 63) / 64);   // six planes per 64-site chunk
  hipLaunchKernelGGL((k_clover_F<N, REP>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     (const cplx<double> *)U, (cplx<double> *)F, g);
  return hipGetLastError();
}

template <int D>
static hipError_t finish_launch(const double *F, void *clov, const Geom &g, const SigmaBlocks &S, double m0,
                                double csw, int expo, int prec, hipStream_t st) {
  const size_t n = 2 * 2 * (size_t)g.Vh;
  const dim3 grid((unsigned)((n + 63) / 64));
  if constexpr (D <= 4) {
    if (!expo) {
      if (prec == 0)
        hipLaunchKernelGGL((k_clover_finish_reg<D, double>), grid, dim3(64), 0, st, (const cplx<double> *)F, clov, g,
                           S, m0, csw);
      else
        hipLaunchKernelGGL((k_clover_finish_reg<D, float>), grid, dim3(64), 0, st, (const cplx<double> *)F, clov, g,
                           S, m0, csw);
      return hipGetLastError();
    }
  }
  if (prec == 0)
    hipLaunchKernelGGL((k_clover_finish<D, double>), grid, dim3(64), 0, st, (const cplx<double> *)F, clov, g, S, m0,
                       csw, expo);
  else
    hipLaunchKernelGGL((k_clover_finish<D, float>), grid, dim3(64), 0, st, (const cplx<double> *)F, clov, g, S, m0,
                       csw, expo);
  return hipGetLastError();
}

static SigmaBlocks sigma_blocks() {
  // gamma_mu = [[0, e_mu], [e_mu^+, 0]], e_0 = -1, e_k = -i sigma_k (Sec. 2.2);
  // sigma_mu,nu = i gamma_mu gamma_nu (mu != nu) = diag(i e_mu e_nu^+, i e_mu^+ e_nu).
  cplx<double> e[4][2][2];
  const cplx<double> z = mk(0.0, 0.0);
  e[0][0][0] = mk(-1.0, 0.0); e[0][0][1] = z; e[0][1][0] = z; e[0][1][1] = mk(-1.0, 0.0);
  // -i sigma_1, -i sigma_2, -i sigma_3
  e[1][0][0] = z; e[1][0][1] = mk(0.0, -1.0); e[1][1][0] = mk(0.0, -1.0); e[1][1][1] = z;
  e[2][0][0] = z; e[2][0][1] = mk(-1.0, 0.0); e[2][1][0] = mk(1.0, 0.0); e[2][1][1] = z;
  e[3][0][0] = mk(0.0, -1.0); e[3][0][1] = z; e[3][1][0] = z; e[3][1][1] = mk(0.0, 1.0);
  auto hmul = [](cplx<double> a, cplx<double> b) { return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); };
  auto conj = [](cplx<double> a) { return mk(a.re, -a.im); };
  SigmaBlocks S{};
  const int pm[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  for (int p = 0; p < 6; ++p) {
    const int mu = pm[p][0], nu = pm[p][1];
    for (int s = 0; s < 2; ++s)
      for (int t = 0; t < 2; ++t) {
        cplx<double> up = z, lo = z;
        for (int k = 0; k < 2; ++k) {
          const cplx<double> a = hmul(e[mu][s][k], conj(e[nu][t][k]));      // (e_mu e_nu^+)_st
          const cplx<double> b = hmul(conj(e[mu][k][s]), e[nu][k][t]);      // (e_mu^+ e_nu)_st
          up = mk(up.re + a.re, up.im + a.im);
          lo = mk(lo.re + b.re, lo.im + b.im);
        }
        // 2 i (...)
        S.v[p][0][s][t] = mk(-2.0 * up.im, 2.0 * up.re);
        S.v[p][1][s][t] = mk(-2.0 * lo.im, 2.0 * lo.re);
      }
  }
  return S;
}

template <int N>
static hipError_t F_launch_n(const void *U, double *F, const Geom &g, int rep, hipStream_t st) {
  switch (rep) {
    case 0: return F_launch<N, 0>(U, F, g, st);
    case 1: return F_launch<N, 1>(U, F, g, st);
    case 2: return F_launch<N, 2>(U, F, g, st);
    case 3:
      if constexpr (N > 2) return F_launch<N, 3>(U, F, g, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_clover_field(void *clov, const void *U, double *F, double *Us, const Geom &g, int N, int rep, int d,
                               double m0, double csw, int expo, int prec, hipStream_t st) {
  hipError_t e = hipErrorInvalidValue;
  switch (N) {
    case 2: e = links_soa_launch<2>(U, Us, g, st); if (e == hipSuccess) e = F_launch_n<2>(Us, F, g, rep, st); break;
    case 3: e = links_soa_launch<3>(U, Us, g, st); if (e == hipSuccess) e = F_launch_n<3>(Us, F, g, rep, st); break;
    case 4: e = links_soa_launch<4>(U, Us, g, st); if (e == hipSuccess) e = F_launch_n<4>(Us, F, g, rep, st); break;
  }
  if (e != hipSuccess) return e;
  const SigmaBlocks S = sigma_blocks();
  switch (d) {
    case 2: return finish_launch<2>(F, clov, g, S, m0, csw, expo, prec, st);
    case 3: return finish_launch<3>(F, clov, g, S, m0, csw, expo, prec, st);
    case 4: return finish_launch<4>(F, clov, g, S, m0, csw, expo, prec, st);
    case 6: return finish_launch<6>(F, clov, g, S, m0, csw, expo, prec, st);
  }
  return hipErrorInvalidValue;
}

template <int D>
static hipError_t apply_launch(void *out, const void *in, const void *clov, const Geom &g, int parity, int nrhs,
                               int prec, hipStream_t st) {
  const dim3 grid((g.Vh + 255) / 256, 2 * nrhs);
  if (prec == 0)
    hipLaunchKernelGGL((k_clover_apply<D, double>), grid, dim3(256), 0, st, (cplx<double> *)out,
                       (const cplx<double> *)in, (const cplx<double> *)clov, g, parity, nrhs);
  else
    hipLaunchKernelGGL((k_clover_apply<D, float>), grid, dim3(256), 0, st, (cplx<float> *)out,
                       (const cplx<float> *)in, (const cplx<float> *)clov, g, parity, nrhs);
  return hipGetLastError();
}

hipError_t launch_clover_apply(void *out, const void *in, const void *clov, const Geom &g, int d, int parity,
                               int nrhs, int prec, hipStream_t st) {
  switch (d) {
    case 2: return apply_launch<2>(out, in, clov, g, parity, nrhs, prec, st);
    case 3: return apply_launch<3>(out, in, clov, g, parity, nrhs, prec, st);
    case 4: return apply_launch<4>(out, in, clov, g, parity, nrhs, prec, st);
    case 6: return apply_launch<6>(out, in, clov, g, parity, nrhs, prec, st);
  }
  return hipErrorInvalidValue;
}

bool clover_supported(int d) { return d == 2 || d == 3 || d == 4 || d == 6; }

// ------------------------------------------------------------ clover force
// Link derivative of a functional whose variation is
//   -2 Re sum_x tr[dM(x) Omega(x)]      (M: the site-diagonal blocks),
// the form of both clover contributions to the HMC force: the pseudofermion
// action with Omega = X Y^+ (X = (x, D_oo^{-1} D_oe x), Y = (D-hat x,
// D_oo^{-1} D_eo^+ D-hat x)) and S_det = -2 sum_{x odd} log|det D_oo| with
// Omega = D_oo^{-1} on the odd sites.
//
// With C = (i c_sw/2) sum_p sigma_p (x) F_p (p = mu < nu) and dM = dC
// (exponential form: tr[dM Omega] = tr[dC Omega'], Omega' = L(A, Omega), the
// Frechet derivative of exp at A = C/(4+m), which is its own adjoint for the
// trace pairing), the variation is (c_sw/8) sum_x sum_p Im tr[dQ_p K_p] with
//   K_p = Lam_p + Lam_p^+,  (Lam_p)_ba = sum_st (sigma_p)_st Omega'_(t b),(s a).
// A leaf l of Q_p varied from the left, R(l) -> exp(i th^b T^b_R) R(l),
// changes Im tr[R(l) K_p] by th^b Re tr[T^b_R R(l) K_p]; its matrix
// g = sum_b Re tr[T^b_R R(l) K_p] T^b is formed in the fundamental by the
// representation pull-back.  A link U inside the leaf, l = B U rest, moves it
// by the generator B T B^+ (l = B' U^+ rest: by -(B'U^+) T (B'U^+)^+), so the
// link's force receives +-B^+ g B with B the fundamental path from the
// leaf's corner up to (forward) or through (dagger) the link.
//
// Pipeline (one lattice): insertion K per (site, chirality) -> leaf matrices
// g per (plane, site) -> gather over the 24 (leaf, corner) pairs holding each
// link.  Scratch: K [2][6][d][d][V], g [6][4][N][N][V] complex FP64.

// Thread per (site, chirality block c): Omega_c = X_c Y_c^+ (Xe non-null)
// + cdet D_oo^{-1} (odd sites), then this block's share of Lam_p for the six
// planes into K[c][p][b][a][V] (regular clover; the exponential form is
// k_clover_insert_rows).
template <int D>
__global__ __launch_bounds__(64) void k_clover_insert(const cplx<double> *Xe, const cplx<double> *Xo,
                                                      const cplx<double> *Ye, const cplx<double> *Yo,
                                                      const cplx<double> *__restrict__ clov,
                                                      const cplx<double> *__restrict__ F, cplx<double> *__restrict__ K,
                                                      Geom g, SigmaBlocks S, double m0, double csw, double cdet) {
  constexpr int NB = 2 * D;
  const size_t V = 2 * (size_t)g.Vh;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= 2 * V) return;
  const int c = (int)(gid / V);
  const size_t lex = gid - (size_t)c * V;
  size_t r = lex;
  const int z = (int)(r % g.Z); r /= g.Z;
  const int y = (int)(r % g.Y); r /= g.Y;
  const int x = (int)(r % g.X);
  const int t = (int)(r / g.X);
  const int par = (t + x + y + z) & 1;
  const size_t cb = lex >> 1;
  cplx<double> Om[NB][NB];
  for (int i = 0; i < NB; ++i)
    for (int j = 0; j < NB; ++j) Om[i][j] = mk(0.0, 0.0);
  if (Xe) {
    const cplx<double> *X = par ? Xo : Xe, *Y = par ? Yo : Ye;
    cplx<double> xv[NB], yv[NB];
    for (int sl = 0; sl < 2; ++sl)
      for (int a = 0; a < D; ++a) {
        const size_t o = (size_t)((2 * c + sl) * D + a) * g.stride + cb;
        xv[sl * D + a] = X[o];
        yv[sl * D + a] = Y[o];
      }
    for (int i = 0; i < NB; ++i)
      for (int j = 0; j < NB; ++j)
        Om[i][j] = mk(xv[i].re * yv[j].re + xv[i].im * yv[j].im, xv[i].im * yv[j].re - xv[i].re * yv[j].im);
  }
  if (cdet != 0.0 && par == 1) {
    const cplx<double> *Mi = clov + (size_t)(2 + c) * (NB * (NB + 1) / 2) * g.stride + cb;
    for (int i = 0; i < NB; ++i)
      for (int j = 0; j < NB; ++j) Om[i][j] = Om[i][j] + cdet * herm_entry(Mi, g.stride, NB, i, j);
  }
  // S.v holds 2 sigma
  for (int p = 0; p < 6; ++p)
    for (int b = 0; b < D; ++b)
      for (int a = 0; a < D; ++a) {
        cplx<double> acc = mk(0.0, 0.0);
        for (int s = 0; s < 2; ++s)
          for (int tt = 0; tt < 2; ++tt) acc = cfma(S.v[p][c][s][tt], Om[tt * D + b][s * D + a], acc);
        K[(((size_t)(c * 6 + p) * D + b) * D + a) * V + lex] = 0.5 * acc;
      }
}

// Exponential form: as k_clover_insert with Omega_c <- L(A_c, Omega_c) before
// the K entries, L the Frechet derivative of exp at A = C / (4 + m) along
// Omega: scaling by 2^-s (s from the largest column sum of |A|, down to 1/4),
// Horner for exp(A') and its derivative along Omega / 2^s (Taylor degree 12,
// as in expm), then s squarings (e, l) <- (e e, l e + e l).
// NB = 2 d_R lanes per (site, chirality block): lane i holds row i of A,
// Omega and of the iterates and reads the other rows from LDS at each matrix
// product (one lane holding whole NB x NB matrices spills them to scratch).  64-lane blocks (one wavefront) hold MPB = 64 / NB matrices;
// the lanes past MPB * NB and past the last matrix follow the barriers and
// store nothing (the former write no LDS either).  Every barrier is reached
// the same number of times by all lanes: the squarings run to the block's
// largest count, a matrix that needs fewer keeping its iterates.
template <int D>
__global__ __launch_bounds__(64) void k_clover_insert_rows(const cplx<double> *Xe, const cplx<double> *Xo,
                                                           const cplx<double> *Ye, const cplx<double> *Yo,
                                                           const cplx<double> *__restrict__ clov,
                                                           const cplx<double> *__restrict__ F,
                                                           cplx<double> *__restrict__ K, Geom g, SigmaBlocks S,
                                                           double m0, double csw, double cdet) {
  constexpr int NB = 2 * D, MPB = 64 / NB;
  __shared__ cplx<double> se[MPB][NB][NB], sl[MPB][NB][NB];
  const size_t V = 2 * (size_t)g.Vh;
  const int mloc0 = (int)threadIdx.x / NB;
  const bool lane_used = mloc0 < MPB;
  const int mloc = lane_used ? mloc0 : MPB - 1;
  const int i = lane_used ? (int)threadIdx.x - mloc * NB : 0;   // row of this lane
  const size_t m0g = (size_t)blockIdx.x * MPB + mloc;
  const bool valid = lane_used && m0g < 2 * V;
  const size_t mg = m0g < 2 * V ? m0g : 2 * V - 1;
  const int c = (int)(mg / V);
  const size_t lex = mg - (size_t)c * V;
  size_t r = lex;
  const int z = (int)(r % g.Z); r /= g.Z;
  const int y = (int)(r % g.Y); r /= g.Y;
  const int x = (int)(r % g.X);
  const int t = (int)(r / g.X);
  const int par = (t + x + y + z) & 1;
  const size_t cb = lex >> 1;
  const int si = i / D, ai = i - si * D;   // row i = (spin si, colour ai) of the block
  cplx<double> om[NB], a[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) om[j] = mk(0.0, 0.0);
  if (Xe) {
    const cplx<double> *X = par ? Xo : Xe, *Y = par ? Yo : Ye;
    const cplx<double> xi = X[(size_t)((2 * c + si) * D + ai) * g.stride + cb];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int sj = j / D, aj = j - sj * D;
      const cplx<double> yj = Y[(size_t)((2 * c + sj) * D + aj) * g.stride + cb];
      om[j] = mk(xi.re * yj.re + xi.im * yj.im, xi.im * yj.re - xi.re * yj.im);
    }
  }
  if (cdet != 0.0 && par == 1) {
    const cplx<double> *Mi = clov + (size_t)(2 + c) * (NB * (NB + 1) / 2) * g.stride + cb;
#pragma unroll
    for (int j = 0; j < NB; ++j) om[j] = om[j] + cdet * herm_entry(Mi, g.stride, NB, i, j);
  }
  // row i of A = (i/4) c_sw sum_p S[p][c][s][t] F_p[a][b] / (4 + m)
  const double f = 0.25 * csw / (4.0 + m0);
#pragma unroll
  for (int tt = 0; tt < 2; ++tt)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      cplx<double> acc = mk(0.0, 0.0);
#pragma unroll
      for (int p = 0; p < 6; ++p)
        acc = cfma(S.v[p][c][si][tt], F[((size_t)p * D * D + ai * D + b) * V + lex], acc);
      a[tt * D + b] = mk(-f * acc.im, f * acc.re);
    }
  // scaling: the maximum column sum of |A|, from LDS
  if (lane_used)
#pragma unroll
    for (int j = 0; j < NB; ++j) se[mloc][i][j] = mk(sqrt(a[j].re * a[j].re + a[j].im * a[j].im), 0.0);
  __syncthreads();
  double nrm = 0.0;
  for (int j = 0; j < NB; ++j) {
    double sum = 0.0;
    for (int q = 0; q < NB; ++q) sum += se[mloc][q][j].re;
    nrm = sum > nrm ? sum : nrm;
  }
  __syncthreads();
  int sq = 0;
  while (nrm > 0.25 && sq < 60) {
    nrm *= 0.5;
    ++sq;
  }
  int sqmax = sq;   // largest over the wavefront (the block)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int o = __shfl_xor(sqmax, off, 64);
    sqmax = o > sqmax ? o : sqmax;
  }
  const double sc = ldexp(1.0, -sq);
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    a[j] = sc * a[j];
    om[j] = sc * om[j];
  }
  constexpr int KT = 12;   // as in expm
  cplx<double> e[NB], l[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    e[j] = mk(i == j ? 1.0 : 0.0, 0.0);
    l[j] = mk(0.0, 0.0);
  }
  // e_k = 1 + a e_{k+1} / k,  l_k = (om e_{k+1} + a l_{k+1}) / k
  for (int k = KT; k >= 1; --k) {
    if (lane_used)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        se[mloc][i][j] = e[j];
        sl[mloc][i][j] = l[j];
      }
    __syncthreads();
    const double rk = 1.0 / k;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      cplx<double> ae = mk(0.0, 0.0), al = mk(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const cplx<double> eq = se[mloc][q][j];
        ae = cfma(a[q], eq, ae);
        al = cfma(om[q], eq, al);
        al = cfma(a[q], sl[mloc][q][j], al);
      }
      e[j] = rk * ae + mk(i == j ? 1.0 : 0.0, 0.0);
      l[j] = rk * al;
    }
    __syncthreads();
  }
  for (int s2 = 0; s2 < sqmax; ++s2) {
    if (lane_used)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        se[mloc][i][j] = e[j];
        sl[mloc][i][j] = l[j];
      }
    __syncthreads();
    cplx<double> te[NB], tl[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      cplx<double> ae = mk(0.0, 0.0), al = mk(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const cplx<double> eq = se[mloc][q][j];
        ae = cfma(e[q], eq, ae);
        al = cfma(l[q], eq, al);
        al = cfma(e[q], sl[mloc][q][j], al);
      }
      te[j] = ae;
      tl[j] = al;
    }
    if (s2 < sq)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        e[j] = te[j];
        l[j] = tl[j];
      }
    __syncthreads();
  }
  // Omega' = L(A, Omega): rows to LDS, then this matrix's K entries shared
  // out over its NB lanes (S.v holds 2 sigma)
  if (lane_used)
#pragma unroll
    for (int j = 0; j < NB; ++j) sl[mloc][i][j] = l[j];
  __syncthreads();
  if (valid) {
    for (int idx = i; idx < 6 * D * D; idx += NB) {
      const int p = idx / (D * D), b = (idx / D) % D, a2 = idx % D;
      cplx<double> acc = mk(0.0, 0.0);
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) acc = cfma(S.v[p][c][s][tt], sl[mloc][tt * D + b][s * D + a2], acc);
      K[(((size_t)(c * 6 + p) * D + b) * D + a2) * V + lex] = 0.5 * acc;
    }
  }
}

// Thread per (plane p, site x): for the four leaves l of Q_p(x), the matrix
// g = sum_b Re tr[T^b_R R(l) K_p] T^b = (H - tr(H)/N)/2 with H the Hermitian
// part of the pull-back of R(l) K_p, into G[p][k][N][N][V].
template <int N, int REP>
__global__ __launch_bounds__(64) void k_clover_leafgen(const cplx<double> *__restrict__ U,
                                                       const cplx<double> *__restrict__ K,
                                                       cplx<double> *__restrict__ G, Geom g) {
  constexpr int D = rep_dim(N, REP);
  const size_t V = 2 * (size_t)g.Vh;
  const size_t gid = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  // 64-site chunks, the six planes of a chunk in consecutive wavefronts (the
  // planes that share a link direction read it close together in time)
  const size_t chunk = gid / 384;
  const int r6 = (int)(gid - chunk * 384);
  const int p = r6 >> 6;
  const size_t lex = chunk * 64 + (r6 & 63);
  if (lex >= V) return;
  int mu, nu;
  plane_dirs(p, mu, nu);
  size_t r = lex;
  int c[4];
  c[3] = (int)(r % g.Z); r /= g.Z;
  c[2] = (int)(r % g.Y); r /= g.Y;
  c[1] = (int)(r % g.X);
  c[0] = (int)(r / g.X);
  const PlaneNb pn(g, c, lex, mu, nu);
  cplx<double> Kh[D][D];
  {
    cplx<double> lam[D][D];
    for (int b = 0; b < D; ++b)
      for (int a = 0; a < D; ++a)
        lam[b][a] = K[(((size_t)p * D + b) * D + a) * V + lex] + K[(((size_t)(6 + p) * D + b) * D + a) * V + lex];
    for (int b = 0; b < D; ++b)
      for (int a = 0; a < D; ++a) Kh[b][a] = mk(lam[b][a].re + lam[a][b].re, lam[b][a].im - lam[a][b].im);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    cplx<double> L[N][N];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const LeafStep s = kLeafC[k][f];
      cplx<double> u[N][N];
      load_link<N>(u, U, V, pn.at(s.a, s.b), s.dir ? nu : mu, s.dag != 0);
      if (f == 0) {
        for (int i = 0; i < N; ++i)
          for (int j = 0; j < N; ++j) L[i][j] = u[i][j];
      } else {
        mul_right<N>(L, u);
      }
    }
    cplx<double> R[D][D], M[D][D];
    for (int A = 0; A < D; ++A)
      for (int B = 0; B < D; ++B) R[A][B] = rep_entry<N, REP>(L, A, B);
    for (int A = 0; A < D; ++A)
      for (int B = 0; B < D; ++B) {
        cplx<double> sum = mk(0.0, 0.0);
        for (int C = 0; C < D; ++C) sum = cfma(R[A][C], Kh[C][B], sum);
        M[A][B] = sum;
      }
    cplx<double> Z[N][N];
    rep_pullback<N, REP>([&](int B, int A) { return M[B][A]; }, Z);
    double tr = 0.0;
    for (int i = 0; i < N; ++i) tr += Z[i][i].re;
    // g = (H - tr(H)/N) / 2, H = (Z + Z^+)/2, Hermitian: stored as N^2 reals
    // (g_ii, then Re g_ij and Im g_ij for i < j), see g_load
    double *gr = reinterpret_cast<double *>(G) + (size_t)(p * 4 + k) * N * N * V + lex;
#pragma unroll
    for (int i = 0; i < N; ++i) gr[(size_t)i * V] = 0.5 * (Z[i][i].re - tr / N);
    int t = N;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = i + 1; j < N; ++j) {
        gr[(size_t)t * V] = 0.25 * (Z[i][j].re + Z[j][i].re);
        gr[(size_t)(t + 1) * V] = 0.25 * (Z[i][j].im - Z[j][i].im);
        t += 2;
      }
  }
}

// The Hermitian leaf matrix g of (plane, leaf) p4k at site xl from its N^2
// stored reals (k_clover_leafgen).
template <int N>
__device__ __forceinline__ void g_load(cplx<double> (&gm)[N][N], const cplx<double> *G, int p4k, size_t xl, size_t V) {
  const double *gr = reinterpret_cast<const double *>(G) + (size_t)p4k * N * N * V + xl;
#pragma unroll
  for (int i = 0; i < N; ++i) gm[i][i] = mk(gr[(size_t)i * V], 0.0);
  int t = N;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i + 1; j < N; ++j) {
      const double re = gr[(size_t)t * V], im = gr[(size_t)(t + 1) * V];
      gm[i][j] = mk(re, im);
      gm[j][i] = mk(re, -im);
      t += 2;
    }
}

// X <- S^+ X S for a Hermitian X, S a fundamental link (dag: its adjoint)
// read from the structure-of-arrays copy; the upper triangle is formed and
// mirrored, so X stays exactly Hermitian.
template <int N>
__device__ __forceinline__ void herm_transport(cplx<double> (&X)[N][N], const cplx<double> *Us, size_t V, size_t lex,
                                               int mu, bool dag) {
  cplx<double> S[N][N], T[N][N];
  load_link<N>(S, Us, V, lex, mu, dag);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      cplx<double> s = mk(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < N; ++q) s = cfma(X[i][q], S[q][j], s);
      T[i][j] = s;
    }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      cplx<double> s = mk(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < N; ++q) s = cfma_conj(S[q][i], T[q][j], s);
      X[i][j] = i == j ? mk(s.re, 0.0) : s;
      if (j != i) X[j][i] = mk(s.re, -s.im);
    }
}

// The plaquette of plane p = (lo, hi) with lower corner z (offsets za, zb
// along lo, hi from y), traversed lo, hi, lo^+, hi^+: steps S_0 = U_lo(z),
// S_1 = U_hi(z+lo), S_2 = U_lo(z+hi)^+, S_3 = U_hi(z)^+, corners c_m = start
// of S_m.  The leaf k of a site is this loop started at c_k (leaf 0 at z,
// 1 at z+lo, 2 at z+lo+hi, 3 at z+hi), so for the link at step J every leaf
// of the plaquette contributes B^+ g_k B with B the path from c_k to step J,
// and the four nest as
//   H_J = g_J + S_{J+3}^+ [g_{J+3} + S_{J+2}^+ [g_{J+2} + S_{J+1}^+ g_{J+1} S_{J+1}] S_{J+2}] S_{J+3}
// (indices mod 4): three transports instead of four separate paths.  The
// link at a forward step receives +H_J, at a backward one -S_J^+ H_J S_J.
template <int N, int J>
__device__ __forceinline__ void plaquette_horner(cplx<double> (&acc)[N][N], const cplx<double> *Us,
                                                 const cplx<double> *Gl, size_t V, const PlaneNb &pn, int lo, int hi,
                                                 int p, int za, int zb) {
  constexpr int ca[4] = {0, 1, 1, 0}, cb[4] = {0, 0, 1, 1};   // corner c_m - z
  constexpr int sa[4] = {0, 1, 0, 0}, sb[4] = {0, 0, 1, 0};   // start of the link of S_m - z
  cplx<double> H[N][N], gm[N][N];
#pragma unroll
  for (int s = 1; s <= 3; ++s) {
    const int m = (J + s) & 3;
    g_load<N>(gm, Gl, p * 4 + m, pn.at(za + ca[m], zb + cb[m]), V);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) H[i][j] = s == 1 ? gm[i][j] : H[i][j] + gm[i][j];
    herm_transport<N>(H, Us, V, pn.at(za + sa[m], zb + sb[m]), (m & 1) ? hi : lo, m >= 2);
  }
  g_load<N>(gm, Gl, p * 4 + J, pn.at(za + ca[J], zb + cb[J]), V);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) acc[i][j] = acc[i][j] + H[i][j] + gm[i][j];
}

// Thread per link (y, rho): P = coef sum over the planes (rho, nu) of the
// contributions of the two plaquettes that hold the link (see
// plaquette_horner); out as in the hopping force: P, or G = 2i P U
// (gradient), stored or accumulated.
template <int N>
__global__ __launch_bounds__(128) void k_clover_gather(const cplx<double> *__restrict__ U,
                                                       const cplx<double> *__restrict__ Gl, double *P, Geom g,
                                                       double coef, int gradient, int accumulate) {
  const size_t V = 2 * (size_t)g.Vh;
  const size_t gid = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  // 64-site chunks, the four directions of a chunk in consecutive
  // wavefronts: the lanes of a wavefront hold one direction on consecutive
  // sites (coalesced structure-of-arrays link reads, the same planes in every
  // lane), and the two directions of a plane read its leaf matrices close
  // together in time
  const size_t chunk = gid / 256;
  const int r4 = (int)(gid - chunk * 256);
  const int rho = r4 >> 6;
  const size_t lex = chunk * 64 + (r4 & 63);
  if (lex >= V) return;
  size_t r = lex;
  int cy[4];
  cy[3] = (int)(r % g.Z); r /= g.Z;
  cy[2] = (int)(r % g.Y); r /= g.Y;
  cy[1] = (int)(r % g.X);
  cy[0] = (int)(r / g.X);
  // forward (af) and backward (ab) occurrences; the backward sum is
  // transported by the link itself once at the end
  cplx<double> af[N][N], ab[N][N];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) af[i][j] = ab[i][j] = mk(0.0, 0.0);
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == rho) continue;
    const int lo = rho < nu ? rho : nu, hi = rho < nu ? nu : rho;
    const int p = lo == 0 ? hi - 1 : lo == 1 ? hi + 1 : 5;
    const PlaneNb pn(g, cy, lex, lo, hi);
    if (rho == lo) {
      plaquette_horner<N, 0>(af, U, Gl, V, pn, lo, hi, p, 0, 0);    // S_0 of the plaquette at y
      plaquette_horner<N, 2>(ab, U, Gl, V, pn, lo, hi, p, 0, -1);   // S_2 of the one at y - hi
    } else {
      plaquette_horner<N, 1>(af, U, Gl, V, pn, lo, hi, p, -1, 0);   // S_1 of the one at y - lo
      plaquette_horner<N, 3>(ab, U, Gl, V, pn, lo, hi, p, 0, 0);    // S_3 of the one at y
    }
  }
  // S_J = U_rho(y)^+ for the backward steps: S_J^+ ab S_J = U ab U^+
  herm_transport<N>(ab, U, V, lex, rho, true);
  cplx<double> acc[N][N];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) acc[i][j] = af[i][j] - ab[i][j];
  cplx<double> Fo[N][N];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) Fo[i][j] = coef * acc[i][j];
  if (gradient) {
    const cplx<double> *u = U + (size_t)rho * N * N * V + lex;
    cplx<double> Gm[N][N];
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        cplx<double> s = mk(0.0, 0.0);
        for (int q = 0; q < N; ++q) s = cfma(Fo[i][q], u[(size_t)(q * N + j) * V], s);
        Gm[i][j] = mk(-2.0 * s.im, 2.0 * s.re);
      }
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) Fo[i][j] = Gm[i][j];
  }
  double *out = P + (lex * 4 + rho) * N * N * 2;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double re = Fo[i][j].re, im = Fo[i][j].im;
      if (accumulate) {
        re += out[2 * (i * N + j)];
        im += out[2 * (i * N + j) + 1];
      }
      out[2 * (i * N + j)] = re;
      out[2 * (i * N + j) + 1] = im;
    }
}

// log|det D_oo(x)| summed over the odd sites: thread per (odd site, block),
// Gaussian elimination with partial pivoting of the stored inverse block
// (log|det D_oo| = -log|det D_oo^{-1}|), block partial sums.
template <int D>
__global__ __launch_bounds__(64) void k_clover_logdet(const cplx<double> *__restrict__ clov, double *partial,
                                                      Geom g) {
  constexpr int NB = 2 * D;
  __shared__ double sh[1];
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (gid < 2 * (size_t)g.Vh) {
    const int c = (int)(gid / g.Vh);
    const size_t cb = gid - (size_t)c * g.Vh;
    const cplx<double> *Mi = clov + (size_t)(2 + c) * (NB * (NB + 1) / 2) * g.stride + cb;
    cplx<double> a[NB][NB];
    for (int i = 0; i < NB; ++i)
      for (int j = 0; j < NB; ++j) a[i][j] = herm_entry(Mi, g.stride, NB, i, j);
    double ld = 0.0;
    for (int col = 0; col < NB; ++col) {
      int piv = col;
      double best = a[col][col].re * a[col][col].re + a[col][col].im * a[col][col].im;
      for (int rr = col + 1; rr < NB; ++rr) {
        const double m2 = a[rr][col].re * a[rr][col].re + a[rr][col].im * a[rr][col].im;
        if (m2 > best) {
          best = m2;
          piv = rr;
        }
      }
      if (piv != col)
        for (int j = 0; j < NB; ++j) {
          const cplx<double> tmp = a[col][j];
          a[col][j] = a[piv][j];
          a[piv][j] = tmp;
        }
      ld += 0.5 * log(best);
      const cplx<double> d = a[col][col];
      const double dn = 1.0 / best;
      const cplx<double> di = mk(d.re * dn, -d.im * dn);
      for (int rr = col + 1; rr < NB; ++rr) {
        const cplx<double> fct = cmul(a[rr][col], di);
        for (int j = col; j < NB; ++j) a[rr][j] = a[rr][j] - cmul(fct, a[col][j]);
      }
    }
    v = -ld;
  }
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

constexpr bool clover_rep_ok(int N, int REP) {
  return (REP != 3 || N > 2) && (rep_dim(N, REP) == 2 || rep_dim(N, REP) == 3 || rep_dim(N, REP) == 4 ||
                                 rep_dim(N, REP) == 6);
}

template <int N, int REP>
static hipError_t clover_force_nr(void *P, const void *Xe, const void *Xo, const void *Ye, const void *Yo,
                                  const void *U0, const void *clov, double *F, double *K, double *Gl, double *Us,
                                  const Geom &g,
                                  double m0, double csw, int expo, double cdet, double coef, int gradient,
                                  int accumulate, hipStream_t st) {
  if constexpr (clover_rep_ok(N, REP)) {
    constexpr int D = rep_dim(N, REP);
    const size_t V = 2 * (size_t)g.Vh;
    {
      hipError_t e = links_soa_launch<N>(U0, Us, g, st);
      if (e != hipSuccess) return e;
    }
    const double *U = Us;
    if (expo) {
      hipError_t e = F_launch<N, REP>(U, F, g, st);
      if (e != hipSuccess) return e;
    }
    const SigmaBlocks S = sigma_blocks();
    const dim3 ig((unsigned)((2 * V + 63) / 64));
    if (expo) {
      constexpr int MPB = 64 / (2 * D);
      const dim3 rg((unsigned)((2 * V + MPB - 1) / MPB));
      hipLaunchKernelGGL((k_clover_insert_rows<D>), rg, dim3(64), 0, st, (const cplx<double> *)Xe,
                         (const cplx<double> *)Xo, (const cplx<double> *)Ye, (const cplx<double> *)Yo,
                         (const cplx<double> *)clov, (const cplx<double> *)F, (cplx<double> *)K, g, S, m0, csw, cdet);
    } else
      hipLaunchKernelGGL((k_clover_insert<D>), ig, dim3(64), 0, st, (const cplx<double> *)Xe,
                         (const cplx<double> *)Xo, (const cplx<double> *)Ye, (const cplx<double> *)Yo,
                         (const cplx<double> *)clov, (const cplx<double> *)F, (cplx<double> *)K, g, S, m0, csw, cdet);
    hipLaunchKernelGGL((k_clover_leafgen<N, REP>), dim3((unsigned)(6 * ((V + 63) / 64))), dim3(64), 0, st,
                       (const cplx<double> *)U, (const cplx<double> *)K, (cplx<double> *)Gl, g);
    hipLaunchKernelGGL((k_clover_gather<N>), dim3((unsigned)(2 * ((V + 63) / 64))), dim3(128), 0, st,
                       (const cplx<double> *)U, (const cplx<double> *)Gl, (double *)P, g, coef, gradient, accumulate);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int N>
static hipError_t clover_force_n(void *P, const void *Xe, const void *Xo, const void *Ye, const void *Yo,
                                 const void *U, const void *clov, double *F, double *K, double *Gl, double *Us,
                                 const Geom &g,
                                 int rep, double m0, double csw, int expo, double cdet, double coef, int gradient,
                                 int accumulate, hipStream_t st) {
  switch (rep) {
    case 0: return clover_force_nr<N, 0>(P, Xe, Xo, Ye, Yo, U, clov, F, K, Gl, Us, g, m0, csw, expo, cdet, coef, gradient, accumulate, st);
    case 1: return clover_force_nr<N, 1>(P, Xe, Xo, Ye, Yo, U, clov, F, K, Gl, Us, g, m0, csw, expo, cdet, coef, gradient, accumulate, st);
    case 2: return clover_force_nr<N, 2>(P, Xe, Xo, Ye, Yo, U, clov, F, K, Gl, Us, g, m0, csw, expo, cdet, coef, gradient, accumulate, st);
    case 3: return clover_force_nr<N, 3>(P, Xe, Xo, Ye, Yo, U, clov, F, K, Gl, Us, g, m0, csw, expo, cdet, coef, gradient, accumulate, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_clover_force(void *P, const void *Xe, const void *Xo, const void *Ye, const void *Yo, const void *U,
                               const void *clov, double *F, double *K, double *Gl, double *Us, const Geom &g, int N, int rep,
                               double m0, double csw, int expo, double cdet, double coef, int gradient, int accumulate,
                               hipStream_t st) {
  switch (N) {
    case 2: return clover_force_n<2>(P, Xe, Xo, Ye, Yo, U, clov, F, K, Gl, Us, g, rep, m0, csw, expo, cdet, coef, gradient, accumulate, st);
    case 3: return clover_force_n<3>(P, Xe, Xo, Ye, Yo, U, clov, F, K, Gl, Us, g, rep, m0, csw, expo, cdet, coef, gradient, accumulate, st);
    case 4: return clover_force_n<4>(P, Xe, Xo, Ye, Yo, U, clov, F, K, Gl, Us, g, rep, m0, csw, expo, cdet, coef, gradient, accumulate, st);
  }
  return hipErrorInvalidValue;
}

int clover_logdet_blocks(const Geom &g) { return (int)((2 * (size_t)g.Vh + 63) / 64); }

hipError_t launch_clover_logdet(const void *clov, double *partial, const Geom &g, int d, hipStream_t st) {
  const dim3 grid((unsigned)clover_logdet_blocks(g));
  switch (d) {
    case 2: hipLaunchKernelGGL(k_clover_logdet<2>, grid, dim3(64), 0, st, (const cplx<double> *)clov, partial, g); break;
    case 3: hipLaunchKernelGGL(k_clover_logdet<3>, grid, dim3(64), 0, st, (const cplx<double> *)clov, partial, g); break;
    case 4: hipLaunchKernelGGL(k_clover_logdet<4>, grid, dim3(64), 0, st, (const cplx<double> *)clov, partial, g); break;
    case 6: hipLaunchKernelGGL(k_clover_logdet<6>, grid, dim3(64), 0, st, (const cplx<double> *)clov, partial, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace wd
