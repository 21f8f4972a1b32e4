// Host-side launchers of the libwdirac kernels (internal interface).
#pragma once

#include <hip/hip_runtime.h>

#include "wd_common.h"

namespace wd {

enum { HOP_SITE = 0, HOP_COLOUR = 1, HOP_COLOUR_PAIR = 2 };

// Arguments of one hopping-term launch.  Pointers are device memory; fields
// are packed half spinors, links the packed represented field.
struct HopArgs {
  void *out;
  const void *in;
  const void *links;
  const void *xadd;   // nullable
  Geom g;
  int parity;         // parity of the output sites
  int xcd_remap;      // map consecutive tiles to one XCD
  double alpha, beta; // out = alpha * xadd + beta * H in
  double *partial;    // nullable: per-block partial sums of |out|^2, [rhs][tile]
  int ntiles, ngroups;  // set by the launcher (colour-split form)
};

// nr: right-hand sides per block of the colour-split form (1..4; reduced to
// one that divides nrhs and fits LDS).  *nblk receives the number of tiles,
// the row length of `partial`.
hipError_t launch_hop(const HopArgs &a, int d, int real, int prec, int dagger, int nrhs, int variant, int nr,
                      hipStream_t st, int *nblk);
int hop_max_nr(int d, int prec, int variant);
int hop_nblocks(int Vh, int d, int variant);
bool hop_variant_ok(int d, int variant);

// rep.hip
hipError_t launch_rep_links(const void *U, void *UR, const Geom &g, int N, int rep, int prec, hipStream_t st);
hipError_t launch_unpack_links(void *canon, const void *UR, const Geom &g, int d, int real, int prec,
                               hipStream_t st);
hipError_t launch_pack_spinor(void *packed, const void *canon, const Geom &g, int d, int parity, int nrhs,
                              int prec, int unpack, hipStream_t st);

// blas.hip -- packed half-spinor linear algebra and reductions.  `ncomp` is
// 4 d_R; fields hold nrhs rows of ncomp * stride complex numbers.
struct FieldShape {
  int Vh, stride, ncomp, nrhs;
};
int blas_nblocks(const FieldShape &f);
// out = a * x + b * y (y nullable); precision of all three = prec
hipError_t launch_lincomb(void *out, double a, const void *x, double b, const void *y, const FieldShape &f, int prec,
                          hipStream_t st);
// partial[r][blk] = sum |v|^2 over the block's sites, all components
hipError_t launch_norm2_partial(double *partial, const void *v, const FieldShape &f, int prec, hipStream_t st);
// out[r] = compensated sum of partial[r][0..nblk)
hipError_t launch_finalize_sum(double *out, const double *partial, int nblk, int nrhs, hipStream_t st);
// partial[r][blk] = Re sum conj(a) b, partial[nrhs + r][blk] = Im sum conj(a) b
hipError_t launch_dot_partial(double *partial, const void *a, const void *b, const FieldShape &f, int prec,
                              hipStream_t st);
// convert between precisions: out (prec_out) = in (prec_in)
hipError_t launch_convert(void *out, int prec_out, const void *in, int prec_in, const FieldShape &f,
                          hipStream_t st);

// CG (see api.hip for the algorithm).  One record per right-hand side.
struct CgScalars {
  double rho;       // <r, r>
  double pAp;       // <p, A p> = ||D-hat p||^2
  double alpha, beta;
  double b2;        // ||b||^2
  double stop2;     // tol^2 ||b||^2 (recursive-residual target)
  double rmax;      // largest ||r|| since the last reliable update (mixed mode)
  double rho64;     // FP64 residual norm^2 at the last reliable update (mixed mode)
  int active;       // 1 while iterating
  int iters;
  int status;       // wdirac_status
  int need_update;  // mixed mode: reliable update requested
  int do_p;         // the last beta step ran for this rhs: p = r + beta p is due
  int pad;
};
hipError_t launch_cg_alpha(CgScalars *s, const double *pAp_partial, int nblk, int nrhs, hipStream_t st);
// x += alpha p (x in prec_x), r -= alpha q, partial |r|^2.  p, q, r in prec.
hipError_t launch_cg_update_xr(void *x, int prec_x, void *r, const void *p, const void *q, const CgScalars *s,
                               double *partial, const FieldShape &f, int prec, hipStream_t st);
hipError_t launch_cg_beta(CgScalars *s, const double *rr_partial, int nblk, int nrhs, double delta,
                          hipStream_t st);
hipError_t launch_cg_update_p(void *p, const void *r, const CgScalars *s, const FieldShape &f, int prec,
                              hipStream_t st);
// r = b - q and partial |r|^2 (FP64)
hipError_t launch_residual(void *r, const void *b, const void *q, double *partial, const FieldShape &f,
                           hipStream_t st);
// With set_b2: b2 = sum(partial), stop2 = tol^2 b2, counters reset.  Otherwise
// rho = sum(partial) for a freshly computed FP64 residual, and every rhs that
// is neither converged nor broken down is (re)activated.
hipError_t launch_cg_restart(CgScalars *s, const double *partial, int nblk, int nrhs, double tol, int set_b2,
                             int first, hipStream_t st);
// x64 += x32, then x32 = 0
hipError_t launch_accum_x(void *x64, void *x32, const FieldShape &f, hipStream_t st);

// force.hip
// U nullable: if given, the output is 2i P U instead of P
hipError_t launch_force_links(void *P, const void *X_e, const void *X_o, const void *Y_e, const void *Y_o,
                              const void *UR, const void *U, const Geom &g, int N, int rep, double scale,
                              int accumulate, hipStream_t st);

}  // namespace wd
