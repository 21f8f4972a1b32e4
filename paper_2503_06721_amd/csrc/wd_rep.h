// Entry-wise map of a fundamental SU(N) matrix to the representations of the
// library (Sec. 2.3), shared by the represented-link and clover kernels.
//
// Bases (fixed conventions of this library):
//  * fundamental generators T^a: for each pair j < k in lexicographic order
//    (E_jk + E_kj)/2 then (-i E_jk + i E_kj)/2; then for k = 1..N-1
//    diag(1,..,1,-k,0,..)/sqrt(2k(k+1));
//  * ADJ: (U_R)_ab = 2 tr(T^a U T^b U^+), evaluated from the few non-zero
//    entries of each generator;
//  * SYM / 2AS: orthonormal basis of symmetric / antisymmetric matrices
//    e_(ab) (a <= b / a < b, lexicographic), e_(aa) = E_aa, e_(ab) =
//    (E_ab +- E_ba)/sqrt 2, acting as M -> U M U^T.  Expanding
//    tr(e_(ab)^+ U e_(cd) U^T) gives the closed forms used below:
//      SYM, a<b, c<d:   U_ac U_bd + U_ad U_bc
//      SYM, a<b, c=d:   sqrt2 U_ac U_bc
//      SYM, a=b, c<d:   sqrt2 U_ac U_ad
//      SYM, a=b, c=d:   U_ac^2
//      2AS, a<b, c<d:   U_ac U_bd - U_ad U_bc
#pragma once

#include "wd_common.h"

namespace wd {

constexpr int rep_dim(int N, int rep) {
  return rep == 0 ? N : rep == 1 ? N * N - 1 : rep == 2 ? N * (N + 1) / 2 : N * (N - 1) / 2;
}

// Non-zero entries of fundamental generator a: returns count, fills (row, col, value).
template <int N>
__device__ __forceinline__ int gen_nz(int a, int (&ri)[N], int (&ci)[N], cplx<double> (&v)[N]) {
  constexpr int noff = N * (N - 1);
  if (a < noff) {
    int p = a >> 1, j = 0;
    while (p >= N - 1 - j) {
      p -= N - 1 - j;
      ++j;
    }
    const int k = j + 1 + p;
    ri[0] = j; ci[0] = k;
    ri[1] = k; ci[1] = j;
    if ((a & 1) == 0) {
      v[0] = mk(0.5, 0.0);
      v[1] = mk(0.5, 0.0);
    } else {
      v[0] = mk(0.0, -0.5);
      v[1] = mk(0.0, 0.5);
    }
    return 2;
  }
  const int kk = a - noff + 1;
  const double nrm = 1.0 / sqrt(2.0 * kk * (kk + 1));
  for (int i = 0; i < kk; ++i) {
    ri[i] = i; ci[i] = i;
    v[i] = mk(nrm, 0.0);
  }
  ri[kk] = kk; ci[kk] = kk;
  v[kk] = mk(-kk * nrm, 0.0);
  return kk + 1;
}

// Index pair (a, b) of two-index basis element A (a <= b for SYM, a < b for 2AS).
template <int N, bool SYM>
__device__ __forceinline__ void pair_of(int A, int &a, int &b) {
  a = 0;
  int rem = A;
  while (rem >= (SYM ? N - a : N - 1 - a)) {
    rem -= SYM ? N - a : N - 1 - a;
    ++a;
  }
  b = a + rem + (SYM ? 0 : 1);
}

// (R(u))_AB for REP = 0 FUND, 1 ADJ (real: imaginary part 0), 2 SYM, 3 2AS.
template <int N, int REP>
__device__ __forceinline__ cplx<double> rep_entry(const cplx<double> (&u)[N][N], int A, int B) {
  if constexpr (REP == 0) {
    return u[A][B];
  } else if constexpr (REP == 1) {
    int ra[N], ca[N], rb[N], cbi[N];
    cplx<double> va[N], vb[N];
    const int na = gen_nz<N>(A, ra, ca, va);
    const int nb = gen_nz<N>(B, rb, cbi, vb);
    // 2 tr(T^A U T^B U^+) = 2 sum T^A_ij U_jk T^B_kl conj(U_il)
    cplx<double> s = mk(0.0, 0.0);
    for (int p = 0; p < na; ++p)
      for (int q = 0; q < nb; ++q) {
        const cplx<double> w = cmul(cmul(va[p], vb[q]), u[ca[p]][rb[q]]);
        s = cfma_conj(u[ra[p]][cbi[q]], w, s);
      }
    return mk(2.0 * s.re, 0.0);
  } else {
    constexpr bool SYM = REP == 2;
    const double rt2 = 1.4142135623730951;
    int a, b, cc, dd;
    pair_of<N, SYM>(A, a, b);
    pair_of<N, SYM>(B, cc, dd);
    if (!SYM) return cmul(u[a][cc], u[b][dd]) - cmul(u[a][dd], u[b][cc]);
    if (a < b && cc < dd) return cmul(u[a][cc], u[b][dd]) + cmul(u[a][dd], u[b][cc]);
    if (a < b) return rt2 * cmul(u[a][cc], u[b][cc]);
    if (cc < dd) return rt2 * cmul(u[a][cc], u[a][dd]);
    return cmul(u[a][cc], u[a][cc]);
  }
}

// Non-zero entries of two-index basis element A (SYM or 2AS): count, and
// (row, col, value) of each.
template <int N, bool SYM>
__device__ __forceinline__ int two_index_nz(int A, int (&ri)[2], int (&ci)[2], double (&v)[2]) {
  int a, b;
  pair_of<N, SYM>(A, a, b);
  if (a == b) {
    ri[0] = a; ci[0] = a; v[0] = 1.0;
    return 1;
  }
  const double s = 0.70710678118654752440;
  ri[0] = a; ci[0] = b; v[0] = s;
  ri[1] = b; ci[1] = a; v[1] = SYM ? s : -s;
  return 2;
}

// Pull-back of a d_R x d_R matrix M to an N x N matrix Z with
// tr(T^a_R M) = tr(T^a Z) for every generator a.  Mel(B, A) returns M_BA.
//   FUND: Z = M.
//   ADJ: (T^a_R)_bc = 2 tr(T^a [T^c, T^b]), so Z = 2 sum_bc M_cb [T^c, T^b].
//   two-index: T^a_R e = T^a e + e T^aT gives, for every non-zero (e_A)_ij
//   and (e_B)_kl, Z_ki += conj(e_A)_ij (e_B)_kj M_BA (l = j) and
//   Z_lj += conj(e_A)_ij (e_B)_il M_BA (k = i); the bases are real.
template <int N, int REP, typename MF>
__device__ __forceinline__ void rep_pullback(MF Mel, cplx<double> (&Z)[N][N]) {
  constexpr int D = rep_dim(N, REP);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) Z[i][j] = mk(0.0, 0.0);
  if constexpr (REP == 0) {
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) Z[i][j] = Mel(i, j);
  } else if constexpr (REP == 1) {
    int rb[N], cb[N], rc[N], cc[N];
    cplx<double> vb[N], vc[N];
    for (int c = 0; c < D; ++c) {
      const int nc = gen_nz<N>(c, rc, cc, vc);
      for (int b = 0; b < D; ++b) {
        const int nb = gen_nz<N>(b, rb, cb, vb);
        const cplx<double> m = 2.0 * Mel(c, b);
        for (int p = 0; p < nc; ++p)
          for (int q = 0; q < nb; ++q) {
            if (cc[p] == rb[q]) Z[rc[p]][cb[q]] = cfma(m, cmul(vc[p], vb[q]), Z[rc[p]][cb[q]]);
            if (cb[q] == rc[p]) Z[rb[q]][cc[p]] = cfma(mk(-m.re, -m.im), cmul(vb[q], vc[p]), Z[rb[q]][cc[p]]);
          }
      }
    }
  } else {
    constexpr bool SYM = REP == 2;
    int ra[2], ca[2], rb[2], cb[2];
    double va[2], vb[2];
    for (int A = 0; A < D; ++A) {
      const int na = two_index_nz<N, SYM>(A, ra, ca, va);
      for (int B = 0; B < D; ++B) {
        const int nb = two_index_nz<N, SYM>(B, rb, cb, vb);
        const cplx<double> m = Mel(B, A);
        for (int p = 0; p < na; ++p)
          for (int q = 0; q < nb; ++q) {
            const cplx<double> c = (va[p] * vb[q]) * m;
            if (cb[q] == ca[p]) Z[rb[q]][ra[p]] = Z[rb[q]][ra[p]] + c;
            if (rb[q] == ra[p]) Z[cb[q]][ca[p]] = Z[cb[q]][ca[p]] + c;
          }
      }
    }
  }
}

}  // namespace wd
