// Linear algebra on packed half spinors and the per-iteration kernels of the
// conjugate-gradient solver.  Sums are accumulated in FP64 whatever the field
// precision; block partial sums are combined by one block per right-hand
// side with Neumaier's compensated summation (Sec. 5.1.1), in a fixed order,
// so results are deterministic (no floating-point atomics).
#include "wd_common.h"
#include "wd_kernels.h"

namespace wd {

constexpr int BT = 256;   // threads per block of the streaming kernels

int blas_nblocks(const FieldShape &f) { return (f.maxvh + BT - 1) / BT; }

Counts uniform_counts(int n) {
  Counts c;
  for (int k = 0; k < MAXSYS; ++k) c.n[k] = n;
  return c;
}

// Row addressing of system s: element (component c, site i) is at
// f.off[s] + c * f.stride[s] + i.

template <typename T>
__device__ __forceinline__ cplx<T> ld(const void *p, size_t o) {
  return static_cast<const cplx<T> *>(p)[o];
}
template <typename T>
__device__ __forceinline__ void st(void *p, size_t o, cplx<double> v) {
  static_cast<cplx<T> *>(p)[o] = mk<T>((T)v.re, (T)v.im);
}
template <typename T>
__device__ __forceinline__ cplx<double> up(cplx<T> v) {
  return mk<double>((double)v.re, (double)v.im);
}

// Compensated accumulation (Neumaier): (s, c) += v.
__device__ __forceinline__ void neumaier_add(double &s, double &c, double v) {
  const double t = s + v;
  if (fabs(s) >= fabs(v)) c += (s - t) + v;
  else c += (v - t) + s;
  s = t;
}

// Error-free transformation: s + e == a + b exactly (Knuth's TwoSum, no
// ordering requirement on |a|, |b|).
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// One block per rhs: compensated sum of partial[0..nblk).  Each thread keeps a
// Neumaier (sum, compensation) pair over a strided subset; pairs are merged
// by a butterfly over the wavefront with TwoSum on the sums, then the four
// wavefronts are merged in a fixed order.  Deterministic: the result depends
// only on nblk and the values, not on timing.
__device__ double sum_partials(const double *partial, int nblk) {
  __shared__ double ws[BT / 64], wc[BT / 64];
  double s = 0.0, c = 0.0;
  for (int k = threadIdx.x; k < nblk; k += BT) neumaier_add(s, c, partial[k]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double so = __shfl_xor(s, off, 64), co = __shfl_xor(c, off, 64);
    double t, e;
    two_sum(s, so, t, e);
    s = t;
    c = (c + co) + e;
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    ws[threadIdx.x >> 6] = s;
    wc[threadIdx.x >> 6] = c;
  }
  __syncthreads();
  double tot = 0.0;
  if (threadIdx.x == 0) {
    double ts = ws[0], tc = wc[0];
    for (int w = 1; w < BT / 64; ++w) {
      double t, e;
      two_sum(ts, ws[w], t, e);
      ts = t;
      tc = (tc + wc[w]) + e;
    }
    tot = ts + tc;
  }
  __syncthreads();
  return tot;
}

__global__ __launch_bounds__(BT) void k_finalize_sum(double *out, const double *partial, int prow, Counts cnt,
                                                     int nsys) {
  const int r = blockIdx.x;
  const double s = sum_partials(partial + (size_t)r * prow, cnt.n[r % nsys]);
  if (threadIdx.x == 0) out[r] = s;
}

// One block per row; rows r >= nsys (the imaginary parts of dot products)
// use the counts of system r - nsys.
hipError_t launch_finalize_sum(double *out, const double *partial, int prow, const Counts &counts, int nrows,
                               int nsys, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_sum, dim3(nrows), dim3(BT), 0, st, out, partial, prow, counts, nsys);
  return hipGetLastError();
}

// ------------------------------------------------------------- streaming
template <typename T>
__global__ __launch_bounds__(BT) void k_lincomb(void *out, double a, const void *x, double b, const void *y,
                                                FieldShape f) {
  const int i = blockIdx.x * BT + threadIdx.x, sy = blockIdx.y;
  if (i >= f.vh[sy]) return;
  const size_t base = (size_t)f.off[sy] + i;
  for (int c = 0; c < f.ncomp; ++c) {
    const size_t o = base + (size_t)c * f.stride[sy];
    cplx<double> v = up(ld<T>(x, o));
    v = a * v;
    if (y) {
      const cplx<double> w = up(ld<T>(y, o));
      v.re = fma(b, w.re, v.re);
      v.im = fma(b, w.im, v.im);
    }
    st<T>(out, o, v);
  }
}

hipError_t launch_lincomb(void *out, double a, const void *x, double b, const void *y, const FieldShape &f, int prec,
                          hipStream_t st) {
  dim3 grid(blas_nblocks(f), f.nsys);
  if (prec == 0) hipLaunchKernelGGL(k_lincomb<double>, grid, dim3(BT), 0, st, out, a, x, b, y, f);
  else hipLaunchKernelGGL(k_lincomb<float>, grid, dim3(BT), 0, st, out, a, x, b, y, f);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(BT) void k_norm2_partial(double *partial, const void *v, FieldShape f) {
  __shared__ double sh[BT / 64];
  const int i = blockIdx.x * BT + threadIdx.x, sy = blockIdx.y;
  double s = 0.0;
  if (i < f.vh[sy]) {
    const size_t base = (size_t)f.off[sy] + i;
    for (int c = 0; c < f.ncomp; ++c) {
      const cplx<T> w = ld<T>(v, base + (size_t)c * f.stride[sy]);
      s += (double)w.re * w.re + (double)w.im * w.im;
    }
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

hipError_t launch_norm2_partial(double *partial, const void *v, const FieldShape &f, int prec, hipStream_t st) {
  dim3 grid(blas_nblocks(f), f.nsys);
  if (prec == 0) hipLaunchKernelGGL(k_norm2_partial<double>, grid, dim3(BT), 0, st, partial, v, f);
  else hipLaunchKernelGGL(k_norm2_partial<float>, grid, dim3(BT), 0, st, partial, v, f);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(BT) void k_dot_partial(double *partial, const void *a, const void *b, FieldShape f) {
  __shared__ double sh[BT / 64];
  const int i = blockIdx.x * BT + threadIdx.x, sy = blockIdx.y;
  double re = 0.0, im = 0.0;
  if (i < f.vh[sy]) {
    const size_t base = (size_t)f.off[sy] + i;
    for (int c = 0; c < f.ncomp; ++c) {
      const size_t o = base + (size_t)c * f.stride[sy];
      const cplx<double> x = up(ld<T>(a, o)), y = up(ld<T>(b, o));
      re = fma(x.re, y.re, re);
      re = fma(x.im, y.im, re);
      im = fma(x.re, y.im, im);
      im = fma(-x.im, y.re, im);
    }
  }
  re = block_sum(re, sh);
  im = block_sum(im, sh);
  if (threadIdx.x == 0) {
    partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = re;
    partial[(size_t)(gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = im;
  }
}

hipError_t launch_dot_partial(double *partial, const void *a, const void *b, const FieldShape &f, int prec,
                              hipStream_t st) {
  dim3 grid(blas_nblocks(f), f.nsys);
  if (prec == 0) hipLaunchKernelGGL(k_dot_partial<double>, grid, dim3(BT), 0, st, partial, a, b, f);
  else hipLaunchKernelGGL(k_dot_partial<float>, grid, dim3(BT), 0, st, partial, a, b, f);
  return hipGetLastError();
}

template <typename TO, typename TI>
__global__ __launch_bounds__(BT) void k_convert(void *out, const void *in, FieldShape f) {
  const int i = blockIdx.x * BT + threadIdx.x, sy = blockIdx.y;
  if (i >= f.vh[sy]) return;
  const size_t base = (size_t)f.off[sy] + i;
  for (int c = 0; c < f.ncomp; ++c) {
    const size_t o = base + (size_t)c * f.stride[sy];
    st<TO>(out, o, up(ld<TI>(in, o)));
  }
}

hipError_t launch_convert(void *out, int prec_out, const void *in, int prec_in, const FieldShape &f,
                          hipStream_t st) {
  dim3 grid(blas_nblocks(f), f.nsys);
  if (prec_out == 0 && prec_in == 1) hipLaunchKernelGGL((k_convert<double, float>), grid, dim3(BT), 0, st, out, in, f);
  else if (prec_out == 1 && prec_in == 0) hipLaunchKernelGGL((k_convert<float, double>), grid, dim3(BT), 0, st, out, in, f);
  else if (prec_out == 0) hipLaunchKernelGGL((k_convert<double, double>), grid, dim3(BT), 0, st, out, in, f);
  else hipLaunchKernelGGL((k_convert<float, float>), grid, dim3(BT), 0, st, out, in, f);
  return hipGetLastError();
}

// ------------------------------------------------------------------- CG
__global__ __launch_bounds__(BT) void k_cg_alpha(CgScalars *S, const double *partial, int prow, Counts cnt) {
  const int r = blockIdx.x;
  CgScalars &s = S[r];
  if (!s.active) return;
  const double pAp = sum_partials(partial + (size_t)r * prow, cnt.n[r]);
  if (threadIdx.x == 0) {
    s.pAp = pAp;
    if (!(pAp > 0.0) || !isfinite(pAp) || !isfinite(s.rho)) {
      s.status = -5;   // breakdown
      s.active = 0;
      s.alpha = 0.0;
    } else {
      s.alpha = s.rho / pAp;
    }
  }
}

hipError_t launch_cg_alpha(CgScalars *s, const double *pAp_partial, int prow, const Counts &counts, int nsys,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_cg_alpha, dim3(nsys), dim3(BT), 0, st, s, pAp_partial, prow, counts);
  return hipGetLastError();
}

template <typename T, typename TX>
__global__ __launch_bounds__(BT) void k_cg_update_xr(void *x, void *r, const void *p, const void *q,
                                                     const CgScalars *S, double *partial, FieldShape f) {
  __shared__ double sh[BT / 64];
  const CgScalars &s = S[blockIdx.y];
  if (!s.active) return;
  const double a = s.alpha;
  const int i = blockIdx.x * BT + threadIdx.x, sy = blockIdx.y;
  double nrm = 0.0;
  if (i < f.vh[sy]) {
    const size_t base = (size_t)f.off[sy] + i;
    for (int c = 0; c < f.ncomp; ++c) {
      const size_t o = base + (size_t)c * f.stride[sy];
      const cplx<double> pv = up(ld<T>(p, o)), qv = up(ld<T>(q, o));
      cplx<double> xv = up(ld<TX>(x, o)), rv = up(ld<T>(r, o));
      xv.re = fma(a, pv.re, xv.re);
      xv.im = fma(a, pv.im, xv.im);
      rv.re = fma(-a, qv.re, rv.re);
      rv.im = fma(-a, qv.im, rv.im);
      st<TX>(x, o, xv);
      const cplx<T> rs = mk<T>((T)rv.re, (T)rv.im);   // the stored (rounded) residual
      static_cast<cplx<T> *>(r)[o] = rs;
      nrm += (double)rs.re * rs.re + (double)rs.im * rs.im;
    }
  }
  nrm = block_sum(nrm, sh);
  if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = nrm;
}

hipError_t launch_cg_update_xr(void *x, int prec_x, void *r, const void *p, const void *q, const CgScalars *s,
                               double *partial, const FieldShape &f, int prec, hipStream_t st) {
  dim3 grid(blas_nblocks(f), f.nsys);
  if (prec == 0 && prec_x == 0)
    hipLaunchKernelGGL((k_cg_update_xr<double, double>), grid, dim3(BT), 0, st, x, r, p, q, s, partial, f);
  else if (prec == 1 && prec_x == 1)
    hipLaunchKernelGGL((k_cg_update_xr<float, float>), grid, dim3(BT), 0, st, x, r, p, q, s, partial, f);
  else if (prec == 1 && prec_x == 0)
    hipLaunchKernelGGL((k_cg_update_xr<float, double>), grid, dim3(BT), 0, st, x, r, p, q, s, partial, f);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// beta = rho'/rho; convergence and (mixed mode) reliable-update triggers.
// The p update of an iteration is due exactly when this kernel ran for the rhs
// (do_p), including the iteration that pauses it for a residual replacement:
// the recurrence resumes afterwards from a consistent (r, p) pair.
__global__ __launch_bounds__(BT) void k_cg_beta(CgScalars *S, const double *partial, int nblk, double delta) {
  const int r = blockIdx.x;
  CgScalars &s = S[r];
  const int act = s.active;
  __syncthreads();
  if (threadIdx.x == 0) s.do_p = 0;
  if (!act) return;
  const double rr = sum_partials(partial + (size_t)r * nblk, nblk);
  if (threadIdx.x == 0) {
    s.iters += 1;
    if (!isfinite(rr)) {
      s.status = -5;
      s.active = 0;
      return;
    }
    s.beta = rr / s.rho;
    s.rho = rr;
    s.do_p = 1;
    const double rn = sqrt(rr);
    if (rn > s.rmax) s.rmax = rn;
    if (rr <= s.stop2) {
      s.active = 0;          // recursive residual converged: verify in FP64
      s.need_update = 1;
    } else if (delta > 0.0 && rn < delta * s.rmax) {
      // mixed mode: ask for a reliable update and keep iterating until every
      // other active system asks too, so that no system idles while the
      // batched hops still stream its field
      s.need_update = 1;
    }
  }
}

hipError_t launch_cg_beta(CgScalars *s, const double *rr_partial, int nblk, int nrhs, double delta,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_cg_beta, dim3(nrhs), dim3(BT), 0, st, s, rr_partial, nblk, delta);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(BT) void k_cg_update_p(void *p, const void *r, const CgScalars *S, FieldShape f) {
  const CgScalars &s = S[blockIdx.y];
  if (!s.do_p) return;
  const double b = s.beta;
  const int i = blockIdx.x * BT + threadIdx.x, sy = blockIdx.y;
  if (i >= f.vh[sy]) return;
  const size_t base = (size_t)f.off[sy] + i;
  for (int c = 0; c < f.ncomp; ++c) {
    const size_t o = base + (size_t)c * f.stride[sy];
    const cplx<double> rv = up(ld<T>(r, o));
    cplx<double> pv = up(ld<T>(p, o));
    pv.re = fma(b, pv.re, rv.re);
    pv.im = fma(b, pv.im, rv.im);
    st<T>(p, o, pv);
  }
}

hipError_t launch_cg_update_p(void *p, const void *r, const CgScalars *s, const FieldShape &f, int prec,
                              hipStream_t st) {
  dim3 grid(blas_nblocks(f), f.nsys);
  if (prec == 0) hipLaunchKernelGGL(k_cg_update_p<double>, grid, dim3(BT), 0, st, p, r, s, f);
  else hipLaunchKernelGGL(k_cg_update_p<float>, grid, dim3(BT), 0, st, p, r, s, f);
  return hipGetLastError();
}

__global__ __launch_bounds__(BT) void k_residual(void *r, const void *b, const void *q, double *partial,
                                                 FieldShape f) {
  __shared__ double sh[BT / 64];
  const int i = blockIdx.x * BT + threadIdx.x, sy = blockIdx.y;
  double nrm = 0.0;
  if (i < f.vh[sy]) {
    const size_t base = (size_t)f.off[sy] + i;
    for (int c = 0; c < f.ncomp; ++c) {
      const size_t o = base + (size_t)c * f.stride[sy];
      const cplx<double> v = ld<double>(b, o) - ld<double>(q, o);
      st<double>(r, o, v);
      nrm += v.re * v.re + v.im * v.im;
    }
  }
  nrm = block_sum(nrm, sh);
  if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = nrm;
}

hipError_t launch_residual(void *r, const void *b, const void *q, double *partial, const FieldShape &f,
                           hipStream_t st) {
  dim3 grid(blas_nblocks(f), f.nsys);
  hipLaunchKernelGGL(k_residual, grid, dim3(BT), 0, st, r, b, q, partial, f);
  return hipGetLastError();
}

// After a (re)computation of r = b - A x in FP64: rho = ||r||^2.  With set_b2
// the partial sums are those of b itself and only b2 / stop2 are set.
// Otherwise rhs that are not finished are (re)activated: finished means
// converged (rho <= stop2), broken down, or b = 0.  reset_p_mask != 0 marks
// that p must be reset to r by the caller (first start).
__global__ __launch_bounds__(BT) void k_cg_restart(CgScalars *S, const double *partial, int nblk, double tol,
                                                   int set_b2, int first) {
  const int r = blockIdx.x;
  CgScalars &s = S[r];
  const double v = sum_partials(partial + (size_t)r * nblk, nblk);
  if (threadIdx.x != 0) return;
  if (set_b2) {
    s.b2 = v;
    s.stop2 = tol * tol * v;
    s.iters = 0;
    s.status = 0;
    s.active = 0;
    s.need_update = 0;
    s.do_p = 0;
    s.rmax = 0.0;
    return;
  }
  s.rho = v;
  s.rho64 = v;
  s.rmax = sqrt(v);
  s.need_update = 0;
  if (first) s.beta = 0.0;
  if (s.status != 0) {
    s.active = 0;
    return;
  }
  if (!isfinite(v)) {
    s.status = -5;
    s.active = 0;
    return;
  }
  s.active = (s.b2 > 0.0 && v > s.stop2) ? 1 : 0;
}

hipError_t launch_cg_restart(CgScalars *s, const double *partial, int nblk, int nrhs, double tol, int set_b2,
                             int first, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_restart, dim3(nrhs), dim3(BT), 0, st, s, partial, nblk, tol, set_b2, first);
  return hipGetLastError();
}

// x64 += x32 and x32 = 0 (mixed-mode accumulation of the inner solution).
__global__ __launch_bounds__(BT) void k_accum_x(void *x64, void *x32, FieldShape f) {
  const int i = blockIdx.x * BT + threadIdx.x, sy = blockIdx.y;
  if (i >= f.vh[sy]) return;
  const size_t base = (size_t)f.off[sy] + i;
  for (int c = 0; c < f.ncomp; ++c) {
    const size_t o = base + (size_t)c * f.stride[sy];
    const cplx<double> v = ld<double>(x64, o) + up(ld<float>(x32, o));
    st<double>(x64, o, v);
    st<float>(x32, o, mk(0.0, 0.0));
  }
}

hipError_t launch_accum_x(void *x64, void *x32, const FieldShape &f, hipStream_t st) {
  dim3 grid(blas_nblocks(f), f.nsys);
  hipLaunchKernelGGL(k_accum_x, grid, dim3(BT), 0, st, x64, x32, f);
  return hipGetLastError();
}

// out = gamma_5 x + i c y (y nullable), gamma_5 = diag(1, 1, -1, -1) on the
// spin index (components spin * d + colour); out may alias x or y.
template <typename T>
__global__ __launch_bounds__(BT) void k_gamma5_axpy(void *out, const void *x, double c, const void *y,
                                                    FieldShape f) {
  const int i = blockIdx.x * BT + threadIdx.x, sy = blockIdx.y;
  if (i >= f.vh[sy]) return;
  const size_t base = (size_t)f.off[sy] + i;
  const int d = f.ncomp / 4;
  for (int comp = 0; comp < f.ncomp; ++comp) {
    const size_t o = base + (size_t)comp * f.stride[sy];
    cplx<double> v = up(ld<T>(x, o));
    if (comp >= 2 * d) v = mk(-v.re, -v.im);
    if (y) {
      const cplx<double> w = up(ld<T>(y, o));
      v.re = fma(-c, w.im, v.re);
      v.im = fma(c, w.re, v.im);
    }
    st<T>(out, o, v);
  }
}

hipError_t launch_gamma5_axpy(void *out, const void *x, double c, const void *y, const FieldShape &f, int prec,
                              hipStream_t st) {
  dim3 grid(blas_nblocks(f), f.nsys);
  if (prec == 0) hipLaunchKernelGGL(k_gamma5_axpy<double>, grid, dim3(BT), 0, st, out, x, c, y, f);
  else hipLaunchKernelGGL(k_gamma5_axpy<float>, grid, dim3(BT), 0, st, out, x, c, y, f);
  return hipGetLastError();
}

// ------------------------------------------------------------ multi-shift CG
// Recursion of the base system (smallest shift sigma0) plus, for every shift
// k with delta_k = sigma_k - sigma0 >= 0, the collinear shifted residual
// r_k = zeta_k r.  With a_{-1} = 1, b_{-1} = 0, zeta_{-1} = zeta_0 = 1:
//   zeta_k' = zeta_k zeta_k^old a_old / (a b_old (zeta_k^old - zeta_k)
//                                        + zeta_k^old a_old (1 + delta_k a)),
//   alpha_k = a zeta_k' / zeta_k,   beta_k = b (zeta_k' / zeta_k)^2,
//   x_k += alpha_k p_k,   p_k = zeta_k' r' + beta_k p_k.
__global__ void k_ms_init(MsScalars *S, const double *b2_partial, int nblk, ShiftList d, int nshift, int base,
                          double sigma0, double tol) {
  const double b2 = sum_partials(b2_partial, nblk);
  if (threadIdx.x != 0) return;
  MsScalars &s = *S;
  s.b2 = b2;
  s.stop2 = tol * tol * b2;
  s.rr = b2;
  s.pAp = 0.0;
  s.alpha = 0.0;
  s.alpha_old = 1.0;
  s.beta = 0.0;
  s.beta_old = 0.0;
  s.sigma0 = sigma0;
  s.iters = 0;
  s.nshift = nshift;
  s.base = base;
  // a non-finite right-hand side is a breakdown, not a zero source
  s.status = isfinite(b2) ? 0 : -5;
  s.active = (b2 > 0.0 && isfinite(b2)) ? 1 : 0;
  for (int k = 0; k < MAXSHIFT; ++k) {
    s.delta[k] = k < nshift ? d.v[k] : 0.0;
    s.zeta[k] = s.zeta_old[k] = s.zeta_new[k] = 1.0;
    s.as[k] = s.bs[k] = 0.0;
    s.sact[k] = k < nshift ? s.active : 0;
    s.upd[k] = 0;
    s.siters[k] = 0;
  }
}

hipError_t launch_ms_init(MsScalars *s, const double *b2_partial, int nblk, const ShiftList &delta, int nshift,
                          int base, double sigma0, double tol, hipStream_t st) {
  hipLaunchKernelGGL(k_ms_init, dim3(1), dim3(BT), 0, st, s, b2_partial, nblk, delta, nshift, base, sigma0, tol);
  return hipGetLastError();
}

// <p, (A + sigma0) p> = ||D-hat p||^2 + sigma0 ||p||^2, base step length and
// the shifted step lengths.
__global__ void k_ms_alpha(MsScalars *S, const double *uu, int prow, int cnt, const double *pp, int nblk_pp) {
  MsScalars &s = *S;
  const int act = s.active;
  __syncthreads();
  // the x updates flagged by the previous iteration's beta step are done:
  // iterations launched after convergence must not repeat them
  if (threadIdx.x == 0)
    for (int k = 0; k < MAXSHIFT; ++k) s.upd[k] = 0;
  if (!act) return;
  double pAp = sum_partials(uu, cnt);
  if (pp) {
    const double p2 = sum_partials(pp, nblk_pp);
    pAp += s.sigma0 * p2;
  }
  (void)prow;
  if (threadIdx.x != 0) return;
  s.pAp = pAp;
  if (!(pAp > 0.0) || !isfinite(pAp)) {
    s.status = -5;
    s.active = 0;
    for (int k = 0; k < s.nshift; ++k) s.sact[k] = s.upd[k] = 0;
    return;
  }
  const double a = s.rr / pAp;
  s.alpha = a;
  for (int k = 0; k < s.nshift; ++k) {
    if (!s.sact[k]) continue;
    const double z = s.zeta[k], zo = s.zeta_old[k];
    const double den = a * s.beta_old * (zo - z) + zo * s.alpha_old * (1.0 + s.delta[k] * a);
    const double zn = z * zo * s.alpha_old / den;
    s.zeta_new[k] = zn;
    s.as[k] = a * zn / z;
  }
}

hipError_t launch_ms_alpha(MsScalars *s, const double *uu_partial, int prow, const Counts &counts,
                           const double *pp_partial, int nblk_pp, hipStream_t st) {
  hipLaunchKernelGGL(k_ms_alpha, dim3(1), dim3(BT), 0, st, s, uu_partial, prow, counts.n[0], pp_partial, nblk_pp);
  return hipGetLastError();
}

// r -= alpha q (FP64), per-block partial sums of |r|^2.
__global__ __launch_bounds__(BT) void k_ms_update_r(void *r, const void *q, const MsScalars *S, double *partial,
                                                    FieldShape f) {
  __shared__ double sh[BT / 64];
  if (!S->active) return;
  const double a = S->alpha;
  const int i = blockIdx.x * BT + threadIdx.x;
  double nrm = 0.0;
  if (i < f.vh[0]) {
    const size_t base = (size_t)f.off[0] + i;
    for (int c = 0; c < f.ncomp; ++c) {
      const size_t o = base + (size_t)c * f.stride[0];
      const cplx<double> qv = ld<double>(q, o);
      cplx<double> rv = ld<double>(r, o);
      rv.re = fma(-a, qv.re, rv.re);
      rv.im = fma(-a, qv.im, rv.im);
      static_cast<cplx<double> *>(r)[o] = rv;
      nrm += rv.re * rv.re + rv.im * rv.im;
    }
  }
  nrm = block_sum(nrm, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = nrm;
}

hipError_t launch_ms_update_r(void *r, const void *q, const MsScalars *s, double *partial, const FieldShape &f,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_ms_update_r, dim3(blas_nblocks(f)), dim3(BT), 0, st, r, q, s, partial, f);
  return hipGetLastError();
}

// beta, the shifted beta_k, rotation of the zeta history, and convergence of
// each shift (|zeta_k| ||r|| <= tol ||b||: its update of this iteration is its
// last).  The base recursion runs while any shift is still being updated.
__global__ void k_ms_beta(MsScalars *S, const double *rr_partial, int nblk) {
  MsScalars &s = *S;
  if (!s.active) return;
  const double rr = sum_partials(rr_partial, nblk);
  if (threadIdx.x != 0) return;
  s.iters += 1;
  if (!isfinite(rr)) {
    s.status = -5;
    s.active = 0;
    for (int k = 0; k < s.nshift; ++k) s.sact[k] = s.upd[k] = 0;
    return;
  }
  const double b = rr / s.rr;
  int any = 0;
  for (int k = 0; k < s.nshift; ++k) {
    s.upd[k] = s.sact[k];
    if (!s.sact[k]) continue;
    const double q = s.zeta_new[k] / s.zeta[k];
    s.bs[k] = b * q * q;
    s.siters[k] += 1;
    s.zeta_old[k] = s.zeta[k];
    s.zeta[k] = s.zeta_new[k];
    if (s.zeta[k] * s.zeta[k] * rr <= s.stop2) s.sact[k] = 0;
    any |= s.sact[k];
  }
  s.alpha_old = s.alpha;
  s.beta_old = b;
  s.beta = b;
  s.rr = rr;
  s.active = any;
}

hipError_t launch_ms_beta(MsScalars *s, const double *rr_partial, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_ms_beta, dim3(1), dim3(BT), 0, st, s, rr_partial, nblk);
  return hipGetLastError();
}

// x_k += alpha_k p_k (shifts whose x update is due) and p_k = zeta_k r +
// beta_k p_k (shifts still active; the base shift while any is), one thread
// per site with the shifts in the inner loop, so that r is read once for all
// of them (per shift 4 half-field passes instead of 5).  Shift fields are
// `fstride` complex elements apart.
__global__ __launch_bounds__(BT) void k_ms_update_xp(void *__restrict__ x, void *__restrict__ p,
                                                     const void *__restrict__ r, const MsScalars *__restrict__ S,
                                                     long long fstride, FieldShape f) {
  const MsScalars &s = *S;
  const int i = blockIdx.x * BT + threadIdx.x;
  if (i >= f.vh[0]) return;
  const int ns = s.nshift, kb = s.base, bact = s.active;
  cplx<double> *xs = static_cast<cplx<double> *>(x);
  cplx<double> *ps = static_cast<cplx<double> *>(p);
  const cplx<double> *rr = static_cast<const cplx<double> *>(r);
  const size_t base = (size_t)f.off[0] + i;
  for (int c = 0; c < f.ncomp; ++c) {
    const size_t o = base + (size_t)c * f.stride[0];
    const cplx<double> rv = rr[o];
    for (int k = 0; k < ns; ++k) {
      const bool ux = s.upd[k] != 0;
      const bool upd_p = k == kb ? bact != 0 : s.sact[k] != 0;
      if (!ux && !upd_p) continue;   // uniform over the grid
      const size_t ok = (size_t)k * fstride + o;
      const cplx<double> pv = ps[ok];
      if (ux) {
        const double a = s.as[k];
        cplx<double> xv = xs[ok];
        xv.re = fma(a, pv.re, xv.re);
        xv.im = fma(a, pv.im, xv.im);
        xs[ok] = xv;
      }
      if (upd_p) {
        const double z = s.zeta[k], b = s.bs[k];
        cplx<double> pn;
        pn.re = fma(z, rv.re, b * pv.re);
        pn.im = fma(z, rv.im, b * pv.im);
        ps[ok] = pn;
      }
    }
  }
}

hipError_t launch_ms_update_xp(void *x, void *p, const void *r, const MsScalars *s, long long fstride,
                               const FieldShape &f, int, hipStream_t st) {
  hipLaunchKernelGGL(k_ms_update_xp, dim3(blas_nblocks(f)), dim3(BT), 0, st, x, p, r, s, fstride, f);
  return hipGetLastError();
}

}  // namespace wd
