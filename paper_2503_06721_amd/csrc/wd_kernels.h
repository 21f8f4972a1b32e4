// Host-side launchers of the libwdirac kernels (internal interface).
//
// A context holds one lattice or a batch of up to MAXLAT lattices of
// different shapes (each with its own geometry).  Packed fields of a batch are
// the concatenation of the per-lattice fields, lattice by lattice.  A
// "system" is one independent field of a packed object: a right-hand side of
// a single lattice, or one lattice of a batch (batches carry one right-hand
// side).  Reductions and CG scalars are per system.
#pragma once

#include <hip/hip_runtime.h>

#include "wd_common.h"

namespace wd {

constexpr int MAXSYS = 12;
constexpr int MAXLAT = 8;

// HOP_COMPACT / HOP_COMPACT_PAIR: the colour-split forms reading the
// fundamental links and rebuilding the two-index represented entries in
// registers (SYM and 2AS only, where N^2 < d_R^2).
// HOP_COLOUR_QUAD: the colour-split form staging two directions (four hops)
// per barrier phase (one rhs per block, d_R <= 4).
// HOP_MULTI: several right-hand sides per block, one wavefront each, with the
// tile's link entries staged once per block in LDS (hop_mr.hip).
enum {
  HOP_SITE = 0,
  HOP_COLOUR = 1,
  HOP_COLOUR_PAIR = 2,
  HOP_COMPACT = 3,
  HOP_COMPACT_PAIR = 4,
  HOP_COLOUR_QUAD = 5,
  HOP_MULTI = 6
};

// One lattice of a launch.
struct LatDesc {
  Geom g;
  int tile0;        // first tile of this lattice in the launch (set by the launcher)
  int ntiles;       // tiles of this lattice (set by the launcher)
  long long soff;   // offset of this lattice in packed half spinors, complex elements
  long long loff;   // offset of this lattice in packed links, link elements
  long long floff;  // offset of this lattice in the compact fundamental links, complex elements
};

// Arguments of one hopping-term launch.  Pointers are device memory; fields
// are packed half spinors, links the packed represented field.
struct HopArgs {
  void *out;
  const void *in;
  const void *links;
  const void *flinks; // compact fundamental links (HOP_COMPACT forms), boundary phase folded as sqrt(bc)
  const void *xadd;   // nullable
  int nlat;
  LatDesc lat[MAXLAT];
  int parity;         // parity of the output sites
  int xcd_remap;      // map consecutive tiles to one XCD
  double alpha, beta; // out = alpha * xadd + beta * H in
  double *partial;    // nullable: per-tile partial sums of |out|^2, [system][prow]
  int prow;           // row length of `partial` (set by the launcher: the largest tile count)
  int ntiles, ngroups;  // total tiles and rhs groups (set by the launcher)
  int tblock;           // t-blocked tile order (0 = lexicographic; single lattices only), see hop.hip
  int tiles_per_tx;     // set by the launcher
};

// Number of valid partial sums per system (rows of a [system][prow] array).
struct Counts {
  int n[MAXSYS];
};

// nr: right-hand sides per block of the colour-split form (1..4; reduced to
// one that divides nrhs and fits LDS); of the site-parallel form 1 or 4 (4 rhs
// across the lanes of each wavefront).  On return counts->n[s] holds the
// number of partial sums written for system s (the tiles of its lattice) and
// *prow their row length.
hipError_t launch_hop(const HopArgs &a, int N, int rep, int d, int real, int prec, int dagger, int nrhs, int variant,
                      int nr, hipStream_t st, Counts *counts, int *prow);
// Whether the colour-split form of the given variant takes nr right-hand
// sides per block (nr in 1..4, or 6 for the unpaired form with d_R <= 4)
// within the LDS budget.
bool hop_nr_supported(int N, int d, int prec, int variant, int nr);
bool hop_variant_ok(int N, int rep, int d, int variant);
// hop_mr.hip: the HOP_MULTI form (nr = right-hand sides per block, one of
// 1, 2, 3, 4, 6, 12, dividing nrhs); built for complex d_R = 3, 6 and real
// d_R = 3.
bool hop_mr_ok(int d, int real);
hipError_t launch_hop_mr(const HopArgs &a, int d, int real, int prec, int dagger, int nrhs, int nr, hipStream_t st,
                         Counts *counts, int *prow);
// Whether the compact forms exist for (N, rep): SYM for N = 2, 3, 4 and 2AS
// for N = 4 (where they read fewer bytes than the represented links).
bool compact_links_ok(int N, int rep);

// rep.hip (one lattice per call; the caller offsets the pointers)
// F (nullable): also write the compact fundamental links [parity][mu][N*N][stride]
// complex, multiplied by i where the boundary phase is -1 (the two-index maps
// are quadratic, so R(i U) = -R(U)).
hipError_t launch_rep_links(const void *U, void *UR, void *F, const Geom &g, int N, int rep, int prec,
                            hipStream_t st);
hipError_t launch_unpack_links(void *canon, const void *UR, const Geom &g, int d, int real, int prec,
                               hipStream_t st);
hipError_t launch_pack_spinor(void *packed, const void *canon, const Geom &g, int d, int parity, int nrhs,
                              int prec, int unpack, hipStream_t st);

// blas.hip -- packed half-spinor linear algebra and reductions.
struct FieldShape {
  int nsys, ncomp, maxvh;
  int vh[MAXSYS];          // sites of the system
  int stride[MAXSYS];      // padded length of one component row
  long long off[MAXSYS];   // complex elements from the field start to the system's first row
};
int blas_nblocks(const FieldShape &f);   // blocks per system of the streaming kernels (row length of partials)
Counts uniform_counts(int n);
// out = a * x + b * y (y nullable); precision of all three = prec
hipError_t launch_lincomb(void *out, double a, const void *x, double b, const void *y, const FieldShape &f, int prec,
                          hipStream_t st);
// partial[s][blk] = sum |v|^2 over the block's sites, all components
hipError_t launch_norm2_partial(double *partial, const void *v, const FieldShape &f, int prec, hipStream_t st);
// out[r] = compensated sum of partial[r][0..counts.n[r % nsys]) for r < nrows,
// rows of length prow (nrows = 2 nsys for the real and imaginary rows of a dot)
hipError_t launch_finalize_sum(double *out, const double *partial, int prow, const Counts &counts, int nrows,
                               int nsys, hipStream_t st);
// partial[s][blk] = Re sum conj(a) b, partial[nsys + s][blk] = Im sum conj(a) b
hipError_t launch_dot_partial(double *partial, const void *a, const void *b, const FieldShape &f, int prec,
                              hipStream_t st);
// out = gamma_5 x + i c y (y nullable); out may alias x or y
hipError_t launch_gamma5_axpy(void *out, const void *x, double c, const void *y, const FieldShape &f, int prec,
                              hipStream_t st);
// convert between precisions: out (prec_out) = in (prec_in)
hipError_t launch_convert(void *out, int prec_out, const void *in, int prec_in, const FieldShape &f,
                          hipStream_t st);

// CG (see api.hip for the algorithm).  One record per system.
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
  int do_p;         // the last beta step ran for this system: p = r + beta p is due
  int pad;
};
hipError_t launch_cg_alpha(CgScalars *s, const double *pAp_partial, int prow, const Counts &counts, int nsys,
                           hipStream_t st);
// x += alpha p (x in prec_x), r -= alpha q, partial |r|^2.  p, q, r in prec.
hipError_t launch_cg_update_xr(void *x, int prec_x, void *r, const void *p, const void *q, const CgScalars *s,
                               double *partial, const FieldShape &f, int prec, hipStream_t st);
hipError_t launch_cg_beta(CgScalars *s, const double *rr_partial, int nblk, int nsys, double delta,
                          hipStream_t st);
hipError_t launch_cg_update_p(void *p, const void *r, const CgScalars *s, const FieldShape &f, int prec,
                              hipStream_t st);
// r = b - q and partial |r|^2 (FP64)
hipError_t launch_residual(void *r, const void *b, const void *q, double *partial, const FieldShape &f,
                           hipStream_t st);
// With set_b2: b2 = sum(partial), stop2 = tol^2 b2, counters reset.  Otherwise
// rho = sum(partial) for a freshly computed FP64 residual, and every system
// that is neither converged nor broken down is (re)activated.
hipError_t launch_cg_restart(CgScalars *s, const double *partial, int nblk, int nsys, double tol, int set_b2,
                             int first, hipStream_t st);
// x64 += x32, then x32 = 0
hipError_t launch_accum_x(void *x64, void *x32, const FieldShape &f, hipStream_t st);

// Multi-shift CG (see blas.hip for the recurrences).  One system (one rhs of
// a single lattice); shift k's fields are `fstride` complex elements apart.
constexpr int MAXSHIFT = 32;
struct ShiftList {
  double v[MAXSHIFT];
};
struct MsScalars {
  double rr;          // <r, r> of the base recursion
  double pAp;         // <p, (A + sigma0) p>
  double alpha, alpha_old, beta, beta_old;
  double b2, stop2;   // ||b||^2, tol^2 ||b||^2
  double sigma0;      // base (smallest) shift
  int iters, active, status, nshift, base, pad;
  double delta[MAXSHIFT];   // sigma_k - sigma0
  double zeta[MAXSHIFT], zeta_old[MAXSHIFT], zeta_new[MAXSHIFT];
  double as[MAXSHIFT], bs[MAXSHIFT];   // shifted alpha_k, beta_k
  int sact[MAXSHIFT];     // shift k is still updated
  int upd[MAXSHIFT];      // shift k's x update is due in this iteration
  int siters[MAXSHIFT];   // iterations that updated shift k
};
hipError_t launch_ms_init(MsScalars *s, const double *b2_partial, int nblk, const ShiftList &delta, int nshift,
                          int base, double sigma0, double tol, hipStream_t st);
hipError_t launch_ms_alpha(MsScalars *s, const double *uu_partial, int prow, const Counts &counts,
                           const double *pp_partial, int nblk_pp, hipStream_t st);
hipError_t launch_ms_update_r(void *r, const void *q, const MsScalars *s, double *partial, const FieldShape &f,
                              hipStream_t st);
hipError_t launch_ms_beta(MsScalars *s, const double *rr_partial, int nblk, hipStream_t st);
hipError_t launch_ms_update_xp(void *x, void *p, const void *r, const MsScalars *s, long long fstride,
                               const FieldShape &f, int nshift, hipStream_t st);

// clover.hip (one lattice per call; the caller offsets the pointers).
// Clover field: [parity][chirality block][d(2d+1)][stride] complex, the upper
// triangle (row-major, diagonal included) of the Hermitian 2d x 2d block; even
// sites holding D_ee, odd sites D_oo^{-1}.  F: scratch of 6 d^2 complex FP64
// per site; Us: scratch of 4 N^2 complex FP64 per site (a structure-of-arrays
// copy of the links).
bool clover_supported(int d);
hipError_t launch_clover_field(void *clov, const void *U, double *F, double *Us, const Geom &g, int N, int rep, int d,
                               double m0, double csw, int expo, int prec, hipStream_t st);
// out = D_ee in (parity 0) or D_oo^{-1} in (parity 1); out may alias in
hipError_t launch_clover_apply(void *out, const void *in, const void *clov, const Geom &g, int d, int parity,
                               int nrhs, int prec, hipStream_t st);
// Clover contribution to the link force of a functional with variation
// -2 Re sum_x tr[dM Omega], Omega = X Y^+ (Xe non-null) + cdet D_oo^{-1} on odd
// sites; P (+)= coef * force (or its gradient form).  F: 6 d^2 V, K: 12 d^2 V,
// Gl: 24 N^2 V complex FP64 scratch (F only for the exponential form), Us:
// 4 N^2 V complex FP64 (structure-of-arrays copy of the links).
hipError_t launch_clover_force(void *P, const void *Xe, const void *Xo, const void *Ye, const void *Yo, const void *U,
                               const void *clov, double *F, double *K, double *Gl, double *Us, const Geom &g, int N, int rep,
                               double m0, double csw, int expo, double cdet, double coef, int gradient, int accumulate,
                               hipStream_t st);
// Partial sums of log|det D_oo(x)| over the odd sites (clover_logdet_blocks of them).
int clover_logdet_blocks(const Geom &g);
hipError_t launch_clover_logdet(const void *clov, double *partial, const Geom &g, int d, hipStream_t st);

// hmc.hip (one lattice per call; canonical fundamental links and momenta)
hipError_t launch_gauge_force(const void *U, void *F, const Geom &g, int N, double beta, double scale,
                              int accumulate, hipStream_t st);
int plaquette_blocks(const Geom &g);
hipError_t launch_plaquette_partial(const void *U, double *partial, const Geom &g, int N, hipStream_t st);
hipError_t launch_link_update(void *U, const void *pi, const Geom &g, int N, double eps, hipStream_t st);
int kinetic_blocks(const Geom &g);
hipError_t launch_kinetic_partial(const void *pi, double *partial, const Geom &g, int N, hipStream_t st);
hipError_t launch_algebra(void *pi, const double *w, const Geom &g, int N, hipStream_t st);

// force.hip (one lattice per call; the caller offsets the pointers)
// U nullable: if given, the output is 2i P U instead of P
hipError_t launch_force_links(void *P, const void *X_e, const void *X_o, const void *Y_e, const void *Y_o,
                              const void *UR, const void *U, const Geom &g, int N, int rep, double scale,
                              int accumulate, hipStream_t st);

}  // namespace wd
