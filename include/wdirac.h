/*
 * libwdirac -- even-odd preconditioned Wilson-Dirac operator for fermions in a
 * representation R of SU(N) (fundamental, adjoint, two-index symmetric and
 * antisymmetric), its conjugate-gradient solve and its fermion force, on AMD
 * MI355X (gfx950).  Definitions follow arXiv:2503.06721 (HiRep v2).
 *
 * C ABI.  Every `void *` field argument is DEVICE memory owned by the caller
 * (for example the data pointer of a torch tensor on the GPU); `stream` is a
 * hipStream_t passed as `void *` (NULL = the null stream).  No call allocates
 * device memory: scratch space is passed in as `workspace`, sized by
 * wdirac_workspace_bytes().  All calls are asynchronous on `stream` except
 * wdirac_cg_eo() and wdirac_force_eo(), which synchronise `stream`.  No call
 * aborts or throws; each returns a wdirac_status code, and on error the
 * thread-local message of wdirac_last_error() says what was wrong.
 *
 * Geometry.  dims = {T, X, Y, Z}, direction mu = 0 is time (Sec. 2.1); every
 * extent must be even and >= 2.  The lexicographic site index is
 * ((t*X + x)*Y + y)*Z + z; a site is even when (t+x+y+z) is even (Sec. 5.3.3).
 * bc[mu] = +1 periodic, -1 antiperiodic for the fermion field (Sec. 6.3.1).
 *
 * Canonical layouts (the caller's), all row-major, complex = (re, im) pairs:
 *   fundamental links  complex128 [T][X][Y][Z][4][N][N]
 *   represented links  complex128 [T][X][Y][Z][4][d][d] (ADJ: float64, real)
 *   spinor (full)      [nrhs][T][X][Y][Z][4][d], complex128 for WDIRAC_F64
 *                      and complex64 for WDIRAC_F32 (spin index, then colour)
 *   force              complex128 [T][X][Y][Z][4][N][N]
 * Packed layouts (the library's, opaque sizes from wdirac_field_bytes()):
 *   half spinor  one parity, structure of arrays: component (spin*d + colour)
 *                major, site (index among sites of that parity, in
 *                lexicographic order) minor, so that consecutive GPU lanes
 *                touch consecutive addresses.
 *   links        U_R for both parities and the four positive directions in the
 *                same site-minor order, with the fermion boundary phase folded
 *                in (Sec. 6.3.1).
 *   clover       per parity, the two 2d x 2d chirality blocks of every site
 *                (row-major entries, site minor).
 */
#ifndef WDIRAC_H
#define WDIRAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wdirac_ctx wdirac_ctx;

typedef enum {
  WDIRAC_OK = 0,
  WDIRAC_EINVAL = -1,       /* bad argument: null pointer, odd extent, nrhs out of range, ... */
  WDIRAC_EUNSUPPORTED = -2, /* (N, representation) pair not built, e.g. SU(2) 2AS (d = 1)     */
  WDIRAC_EHIP = -3,         /* HIP runtime error (message in wdirac_last_error)              */
  WDIRAC_ENOCONV = -4,      /* solver reached maxit; x holds the last iterate, stats filled   */
  WDIRAC_EBREAKDOWN = -5    /* solver met a non-finite value or <p, A p> <= 0                 */
} wdirac_status;

typedef enum { WDIRAC_FUND = 0, WDIRAC_ADJ = 1, WDIRAC_SYM = 2, WDIRAC_ASYM = 3 } wdirac_rep;
typedef enum { WDIRAC_F64 = 0, WDIRAC_F32 = 1 } wdirac_prec;
typedef enum { WDIRAC_CG_F64 = 0, WDIRAC_CG_MIXED = 1 } wdirac_cg_mode;

/* Kinds of packed objects, for wdirac_field_bytes(). */
typedef enum { WDIRAC_FIELD_HALF_SPINOR = 0, WDIRAC_FIELD_LINKS = 1, WDIRAC_FIELD_CLOVER = 2 } wdirac_field_kind;
/* Operations that need scratch memory, for wdirac_workspace_bytes(). */
typedef enum {
  WDIRAC_OP_DHAT = 0,
  WDIRAC_OP_CG = 1,
  WDIRAC_OP_FORCE = 2,
  WDIRAC_OP_NORM = 3,
  WDIRAC_OP_DOT = 4,
  WDIRAC_OP_TUNE = 5,
  WDIRAC_OP_MSHIFT = 6,  /* `nrhs` argument = number of shifts (1..32) */
  WDIRAC_OP_CLOVER = 7,  /* construction of a clover field */
  WDIRAC_OP_GAUGE = 8,   /* gauge action and kinetic-energy reductions */
  WDIRAC_OP_CLOVER_FORCE = 9 /* clover force and clover determinant */
} wdirac_op;

typedef struct {
  int32_t dims[4]; /* T, X, Y, Z: even, >= 2                                */
  int32_t bc[4];   /* +1 periodic or -1 antiperiodic fermion BC per direction */
} wdirac_geom;

typedef struct {
  int32_t iters;            /* CG iterations (outer plus inner for mixed)            */
  int32_t reliable_updates; /* FP64 residual replacements                            */
  int32_t hops;             /* hopping-term applications issued for this solve       */
  int32_t status;           /* wdirac_status of this right-hand side                 */
  double true_rel_resid;    /* ||b - A x|| / ||b|| recomputed in FP64 at the end      */
  double seconds;           /* wall time of the solve: from the point where the work
                               queued on the stream before the call has finished to
                               the return                                            */
} wdirac_cg_stats;

/* Create a context for SU(Ng) fermions in representation `rep` on the lattice
 * `geom`.  Host only: validates arguments and records the geometry; touches no
 * GPU.  Supported: Ng in {2, 3, 4} with every representation of the paper's
 * table of representations (Sec. 2.3) except SU(2) 2AS, whose d_R = 1.
 * *ctx receives the new context (owned by the caller, released with
 * wdirac_destroy).  Errors: EINVAL, EUNSUPPORTED. */
int wdirac_create(wdirac_ctx **ctx, int Ng, int rep, const wdirac_geom *geom);

/* Create a context for a batch of nlat (1..8) lattices of possibly different
 * extents and boundary conditions, same Ng and representation: every call on
 * the context processes all lattices at once (one launch per kernel).  Packed
 * fields and links of a batch are the per-lattice objects one after the
 * other, lattice by lattice; canonical batch layouts are the per-lattice
 * canonical arrays one after the other ([lattice][T][X][Y][Z]...).  A batch
 * carries one right-hand side per lattice (nrhs = 1 in every call); results
 * that are per right-hand side (norms, dots, CG statistics) are per lattice.
 * Same errors as wdirac_create; EINVAL also for nlat out of range. */
int wdirac_create_batch(wdirac_ctx **ctx, int Ng, int rep, const wdirac_geom *geoms, int nlat);

/* Release a context (NULL is accepted). */
int wdirac_destroy(wdirac_ctx *ctx);

/* Tuning options (host only; they change speed, never results beyond
 * rounding):
 *   WDIRAC_OPT_HOP_VARIANT_F64 / _F32  0 = one lane per site (d_R <= 6 only),
 *                                      1 = one wavefront per colour row of a
 *                                          64-site tile (default),
 *                                      2 = as 1 with the forward and backward
 *                                          hop of each direction staged
 *                                          together (half the barriers),
 *                                      3, 4 = as 1, 2 reading the compact
 *                                          fundamental links and rebuilding
 *                                          the entries of U_R in registers
 *                                          (SYM for N = 2..4, 2AS for N = 4;
 *                                          1 or 2 rhs per block)
 *                                      5 = as 1 with two directions (four
 *                                          hops) staged per barrier phase
 *                                          (d_R <= 6; 1 rhs per block)
 *                                      6 = several right-hand sides per
 *                                          block, one wavefront each, the
 *                                          tile's link entries staged once
 *                                          per block in LDS (complex d_R = 3
 *                                          and 6, real d_R = 3; 1, 2, 3, 4,
 *                                          6 or 12 rhs per block)
 *   WDIRAC_OPT_XCD_REMAP               1 (default) = give each XCD a
 *                                      contiguous range of site tiles
 *   WDIRAC_OPT_CG_CHECK_EVERY          CG iterations between host checks of
 *                                      convergence (default 4, 1..1000)
 *   WDIRAC_OPT_MIXED_DELTA             reliable-update trigger of mixed CG,
 *                                      ||r|| < delta max ||r|| (default 0.01)
 *   WDIRAC_OPT_TILE_TBLOCK             0 (default) = site tiles in lexicographic
 *                                      order; b > 0 = in t-blocks of b slices
 *                                      (t-neighbours close in time), used
 *                                      when b divides T; b = -(10 bx + by) < 0
 *                                      = sub-lattices of bx x-rows by by
 *                                      tiles of a (t, x) row, each swept
 *                                      along t, used when bx, by > 0 divide
 *                                      X and the tiles of a row (values in
 *                                      [-99, 64]); both need tiles that do
 *                                      not straddle (t, x) rows
 *   WDIRAC_OPT_HOP_NR_F64 / _F32       right-hand sides sharing each link load
 *                                      (1..12).  Form 6: the largest of 1,
 *                                      2, 3, 4, 6, 12 not above it that
 *                                      divides nrhs.  Colour-split form: the
 *                                      largest divisor of nrhs not above it
 *                                      that the form supports is used (1..4
 *                                      within the LDS budget; 6 in the
 *                                      unpaired form for d_R <= 4).
 *                                      Site-parallel form: 4 (4 rhs across
 *                                      the lanes of a wavefront) when it is 4
 *                                      and divides nrhs, else 1
 *   WDIRAC_OPT_CG_GRAPH                1 (default): the CG iterations between
 *                                      host checks are captured once per
 *                                      solve into a HIP graph and replayed
 *                                      on a stream of the library's own
 *                                      (after the caller's stream has
 *                                      drained); 0: direct launches on the
 *                                      caller's stream
 *   WDIRAC_OPT_TUNE_COMPACT            1 (default): wdirac_autotune() also
 *                                      times the compact-link forms 3, 4;
 *                                      0: stored-link forms only
 * Options set here apply to every nrhs except those that wdirac_autotune()
 * has tuned.  Errors: EINVAL (unknown option or value), EUNSUPPORTED. */
typedef enum {
  WDIRAC_OPT_HOP_VARIANT_F64 = 0,
  WDIRAC_OPT_HOP_VARIANT_F32 = 1,
  WDIRAC_OPT_XCD_REMAP = 2,
  WDIRAC_OPT_CG_CHECK_EVERY = 3,
  WDIRAC_OPT_MIXED_DELTA = 4,
  WDIRAC_OPT_HOP_NR_F64 = 5,
  WDIRAC_OPT_HOP_NR_F32 = 6,
  WDIRAC_OPT_TILE_TBLOCK = 7,
  WDIRAC_OPT_CG_GRAPH = 8,
  WDIRAC_OPT_TUNE_COMPACT = 9
} wdirac_option;
int wdirac_set_option(wdirac_ctx *ctx, int option, double value);

/* Launch shape of the hopping kernel chosen by wdirac_autotune(). */
typedef struct {
  int32_t variant;    /* WDIRAC_OPT_HOP_VARIANT_F64 values (0..6)        */
  int32_t nr;         /* right-hand sides per block (colour-split form)  */
  int32_t xcd_remap;  /* 1 = contiguous tile ranges per XCD               */
  int32_t tblock;     /* tile order (WDIRAC_OPT_TILE_TBLOCK values)      */
  int32_t candidates; /* number of shapes timed                           */
  double us;          /* mean time of one hop launch with that shape (best
                         round of the second pass)                        */
  double spread;      /* (slowest - fastest) / fastest over the chosen
                         shape's five second-pass rounds                  */
  double runner_up_us;/* best round of the second-fastest finalist        */
} wdirac_tuning;

/* Autotuner: times every available launch shape of the hopping kernel
 * (variant x right-hand sides per block x XCD tile mapping x tile order) for
 * nrhs right-hand sides in precision prec on the links UR (HIP events,
 * after ~50 ms of untimed launches: 4 warm-up and 10 timed launches each,
 * repeated over ~5 ms, then the six
 * fastest again in five interleaved rounds of max(20, ~25 ms) launches, each
 * keeping its fastest round; launches
 * alternate D_eo and D_oe over three fields so that every other launch reads
 * the output just written, as between the hops of a solver), and makes the
 * fastest the one used for this (prec, nrhs) by every later call on ctx (CG
 * included).  Results never change
 * beyond rounding.  workspace: wdirac_workspace_bytes(ctx, WDIRAC_OP_TUNE,
 * nrhs, prec) bytes (overwritten).  best (host, nullable) receives the choice.
 * Synchronises.  Errors: EINVAL, EHIP. */
int wdirac_autotune(wdirac_ctx *ctx, const void *UR, int prec, int nrhs, void *workspace, wdirac_tuning *best,
                    void *stream);

/* Representation dimension d_R and whether links are stored as real numbers
 * (ADJ; Sec. 4.1.2).  Host only. */
int wdirac_rep_info(const wdirac_ctx *ctx, int *d_R, int *real_links);

/* Bytes of one packed object of `kind` holding `nrhs` right-hand sides (1 for
 * links) in precision `prec`.  Returns 0 for invalid arguments.  Host only. */
size_t wdirac_field_bytes(const wdirac_ctx *ctx, int kind, int nrhs, int prec);

/* Bytes of scratch memory `op` needs for `nrhs` right-hand sides (for
 * WDIRAC_OP_CG, `prec` is a wdirac_cg_mode).  Returns 0 for invalid arguments. */
size_t wdirac_workspace_bytes(const wdirac_ctx *ctx, int op, int nrhs, int prec);

/* Pack the sites of parity `parity` of the canonical full spinor `canon`
 * ([nrhs][T][X][Y][Z][4][d]) into the packed half spinor `packed`.  Both in
 * precision `prec`.  Errors: EINVAL, EHIP. */
int wdirac_pack_spinor(const wdirac_ctx *ctx, void *packed, const void *canon, int parity, int nrhs,
                       int prec, void *stream);

/* Inverse of wdirac_pack_spinor: writes the sites of parity `parity` of the
 * canonical full spinor `canon`; sites of the other parity are left as they
 * are.  Errors: EINVAL, EHIP. */
int wdirac_unpack_spinor(const wdirac_ctx *ctx, void *canon, const void *packed, int parity, int nrhs,
                         int prec, void *stream);

/* Represented links (Sec. 2.3): U_R(x,mu) = R(U(x,mu)) for every link of the
 * canonical fundamental field `U`, written packed to `UR` in precision
 * `prec`, with the fermion boundary phase bc[mu] multiplied into the links
 * U_R(x,mu) whose x_mu = L_mu - 1 (the hops that cross the boundary; Sec.
 * 6.3.1 applies the antiperiodic sign to one slice of the represented field).
 * Bases of R: generalised Gell-Mann generators, ADJ (U_R)_ab =
 * 2 tr(T^a U T^b U^+), SYM/2AS on the orthonormal (anti)symmetric basis
 * matrices in lexicographic pair order.  For SYM with N = 2, 3, 4 and 2AS
 * with N = 4 the field also holds, after U_R, a compact copy of the
 * fundamental links (N^2 instead of d_R^2 entries per link; i U on the links
 * whose phase is -1, since the two-index maps are quadratic) from which the
 * compact hop forms rebuild U_R in registers; wdirac_field_bytes(
 * WDIRAC_FIELD_LINKS) counts both.  Errors: EINVAL, EHIP. */
int wdirac_rep_links(const wdirac_ctx *ctx, void *UR, const void *U, int prec, void *stream);

/* Unpack packed links `UR` (precision `prec`) to the canonical represented
 * layout in float64/complex128 (boundary phase included).  For checks. */
int wdirac_unpack_links(const wdirac_ctx *ctx, void *UR_canon, const void *UR, int prec, void *stream);

/* Hopping block of the Wilson-Dirac operator (Sec. 2.3, even-odd split of
 * Sec. 5.3.3), applied to `nrhs` packed half spinors at once:
 *   out = alpha * x_add + beta * H in,
 *   H in (x) = -1/2 sum_mu [ (1 - g_mu) U_R(x,mu) in(x+mu)
 *                            + (1 + g_mu) U_R(x-mu,mu)^+ in(x-mu) ]
 * for the sites x of parity `out_parity` (0: D_eo, input odd; 1: D_oe, input
 * even).  With dagger = 1, H is replaced by the (out_parity, 1-out_parity)
 * block of H^+, i.e. the adjoint of the opposite block (the two spin
 * projectors trade places).  x_add may be NULL (then alpha is ignored); it may
 * alias `out` but `in` may not.  `UR` comes from wdirac_rep_links in the same
 * precision `prec`.  Errors: EINVAL, EHIP. */
int wdirac_dslash_eo(const wdirac_ctx *ctx, void *out, const void *in, const void *UR, int out_parity,
                     int dagger, int nrhs, double alpha, const void *x_add, double beta, int prec,
                     void *stream);

/* Diagonal blocks of the unimproved Wilson operator (Sec. 5.3.3):
 * D_ee = D_oo = (4 + m0) 1; out = (4 + m0) in, or in / (4 + m0) when
 * inverse = 1.  out may alias in.  Errors: EINVAL (also m0 = -4 with
 * inverse), EHIP. */
int wdirac_apply_Mee(const wdirac_ctx *ctx, void *out, const void *in, double m0, int inverse, int nrhs,
                     int prec, void *stream);
int wdirac_apply_Moo(const wdirac_ctx *ctx, void *out, const void *in, double m0, int inverse, int nrhs,
                     int prec, void *stream);

/* Preconditioned operator (Sec. 5.3.3) on packed even half spinors:
 *   dagger = 0: out = D-hat in   = (4+m0)^2 in - D_eo D_oe in,
 *   dagger = 1: out = D-hat^+ in = (4+m0)^2 in - D_oe^+ D_eo^+ in.
 * workspace: wdirac_workspace_bytes(ctx, WDIRAC_OP_DHAT, nrhs, prec) bytes.
 * Errors: EINVAL, EHIP. */
int wdirac_apply_dhat(const wdirac_ctx *ctx, void *out, const void *in, const void *UR, double m0,
                      int dagger, int nrhs, int prec, void *workspace, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * out = D-hat in / D-hat^+ in as wdirac_apply_dhat, with no workspace
 * argument.  The odd half field between the two hops lives in a fixed
 * device array inside the library, wdirac_noalloc_scratch_bytes() = 64 MiB
 * per GPU, held from the first call on that GPU until the process ends.
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine); the caller owns in, out and UR as for wdirac_apply_dhat.
 * Every call on one GPU shares that GPU's array and overwrites it before
 * reading it, so calls that overlap on one GPU (other streams, other
 * threads, other contexts) race and must be serialised by the caller.
 * Asynchronous on `stream`.  Errors: EINVAL (as wdirac_apply_dhat, and when
 * the odd half field, wdirac_field_bytes(ctx, WDIRAC_FIELD_HALF_SPINOR,
 * nrhs, prec) bytes, exceeds the scratch size), EHIP. */
int wdirac_apply_dhat_noalloc(const wdirac_ctx *ctx, void *out, const void *in, const void *UR, double m0,
                              int dagger, int nrhs, int prec, void *stream);
size_t wdirac_noalloc_scratch_bytes(void);

/* Even-odd source preparation (Sec. 5.3.3, from the block form of D_m psi =
 * eta): b_e = (4+m0) eta_e - D_eo eta_o.  Packed FP64 halves.  Errors: EINVAL, EHIP. */
int wdirac_eo_source(const wdirac_ctx *ctx, void *b_e, const void *eta_e, const void *eta_o,
                     const void *UR, double m0, int nrhs, void *stream);

/* Odd half of the solution: psi_o = (eta_o - D_oe psi_e) / (4 + m0).  Packed
 * FP64 halves.  Errors: EINVAL, EHIP. */
int wdirac_eo_reconstruct(const wdirac_ctx *ctx, void *psi_o, const void *psi_e, const void *eta_o,
                          const void *UR, double m0, int nrhs, void *stream);

/* Squared norms ||v_k||^2 of the nrhs packed half spinors v (precision prec),
 * summed in FP64 with compensated (Neumaier, Sec. 5.1.1) accumulation of the
 * block partial sums; written to the host array out[nsys] (nsys = nrhs, or
 * the number of lattices of a batch).  Synchronises.
 * workspace: wdirac_workspace_bytes(ctx, WDIRAC_OP_NORM, nrhs, prec). */
int wdirac_norm2(const wdirac_ctx *ctx, double *out, const void *v, int nrhs, int prec, void *workspace,
                 void *stream);

/* Inner products <a_k, b_k> = sum over sites, spins and colours of
 * conj(a) b (Sec. 4.2.2) for the nrhs packed half spinors a, b (precision
 * prec), summed in FP64 with compensated accumulation of the block partial
 * sums; written to the host array out[2 nsys] as (re, im) pairs (nsys =
 * nrhs, or the number of lattices of a batch).
 * Synchronises.  workspace: wdirac_workspace_bytes(ctx, WDIRAC_OP_DOT, nrhs,
 * prec).  Errors: EINVAL, EHIP. */
int wdirac_dot(const wdirac_ctx *ctx, double *out, const void *a, const void *b, int nrhs, int prec,
               void *workspace, void *stream);

/* Conjugate gradient (Sec. 5.1.2) on (D-hat^+ D-hat) x = b over the even sites,
 * independently for each of nrhs right-hand sides.  x (packed FP64, in: the
 * initial guess, out: the solution), b (packed FP64).  Stops when the FP64
 * true residual ||b - A x|| <= tol ||b|| (recomputed, not the recursive one).
 * mode WDIRAC_CG_F64: all in FP64, UR32 unused (may be NULL).  mode
 * WDIRAC_CG_MIXED: FP32 hops and vectors inside, FP64 solution, FP64
 * residual replacements ("reliable updates") and FP64 inner-product sums;
 * UR32 = the FP32 links.  stats: host array of nsys records (nsys = nrhs,
 * or the number of lattices of a batch).  Returns OK,
 * ENOCONV (some rhs reached maxit), EBREAKDOWN, EINVAL or EHIP.  workspace:
 * wdirac_workspace_bytes(ctx, WDIRAC_OP_CG, nrhs, mode).  Synchronises. */
int wdirac_cg_eo(const wdirac_ctx *ctx, void *x, const void *b, const void *UR64, const void *UR32,
                 double m0, double tol, int maxit, int nrhs, int mode, void *workspace,
                 wdirac_cg_stats *stats, void *stream);

/* Clover improvement (Sec. 6.1.2, exponential form Sec. 6.1.3).  Builds the site-diagonal blocks of the
 * clover-improved operator from the fundamental links U (canonical complex128
 * [T][X][Y][Z][4][N][N], lattice after lattice for a batch):
 *   D_ee + D_oo = (4 + m0) + csw (i/4) sum_{mu,nu} sigma_mu,nu F_mu,nu(x),
 * or with exponential = 1 the exponential form
 *   (4 + m0) exp(csw / (4 + m0) (i/4) sum_{mu,nu} sigma_mu,nu F_mu,nu(x)),
 * sigma_mu,nu = (i/2)[gamma_mu, gamma_nu], F_mu,nu = (Q_mu,nu - Q_mu,nu^+)/8,
 * Q the sum of the four plaquette leaves of the (mu, nu) plane at x (all
 * starting at x, turning from mu to nu), in the fermion representation.  The
 * packed clover field (wdirac_field_bytes(ctx, WDIRAC_FIELD_CLOVER, 1, prec)
 * bytes, precision prec) holds, per site, the two 2d x 2d chirality blocks:
 * D_ee on the even sites and D_oo^{-1} on the odd sites, which is what
 * D-hat = D_ee - D_eo D_oo^{-1} D_oe (Sec. 5.3.3) applies.  The blocks are
 * Hermitian and only their upper triangles (d(2d+1) complex entries each)
 * are stored.  Computed in FP64.
 * workspace: wdirac_workspace_bytes(ctx, WDIRAC_OP_CLOVER, 1, WDIRAC_F64).
 * Errors: EINVAL, EUNSUPPORTED (d_R not in {2, 3, 4, 6}), EHIP. */
int wdirac_clover_field(const wdirac_ctx *ctx, void *clov, const void *U, double m0, double csw, int exponential,
                        int prec, void *workspace, void *stream);

/* out = D_ee in (parity 0, even half fields) or D_oo^{-1} in (parity 1, odd
 * half fields) with the clover field clov, for nrhs packed half spinors of
 * precision prec (clov of the same precision).  out may alias in.  Errors:
 * EINVAL, EUNSUPPORTED, EHIP. */
int wdirac_apply_clover(const wdirac_ctx *ctx, void *out, const void *in, const void *clov, int parity, int nrhs,
                        int prec, void *stream);

/* Clover even-odd operator out = D-hat in, D-hat = D_ee - D_eo D_oo^{-1} D_oe
 * (Sec. 5.3.3; dagger = 1: D-hat^+ = D_ee - D_oe^+ D_oo^{-1} D_eo^+, the
 * blocks being Hermitian).  The mass enters through the clover field.  Note
 * the normalisation: with csw = 0 this is the D-hat of wdirac_apply_dhat
 * divided by (4 + m0).  workspace: wdirac_workspace_bytes(ctx, WDIRAC_OP_DHAT,
 * nrhs, prec).  out must not alias in.  Errors: EINVAL, EUNSUPPORTED, EHIP. */
int wdirac_apply_dhat_clover(const wdirac_ctx *ctx, void *out, const void *in, const void *UR, const void *clov,
                             int dagger, int nrhs, int prec, void *workspace, void *stream);

/* Conjugate gradient on (D-hat^+ D-hat) x = b with the clover D-hat above;
 * otherwise exactly as wdirac_cg_eo (mode, stopping on the FP64 true
 * residual, reliable updates, statistics, workspace WDIRAC_OP_CG).  clov64:
 * the FP64 clover field; clov32: the FP32 one (mode WDIRAC_CG_MIXED only,
 * may be NULL otherwise). */
int wdirac_cg_eo_clover(const wdirac_ctx *ctx, void *x, const void *b, const void *UR64, const void *UR32,
                        const void *clov64, const void *clov32, double tol, int maxit, int nrhs, int mode,
                        void *workspace, wdirac_cg_stats *stats, void *stream);

/* Fermion force of S_f = phi^+ (D-hat^+ D-hat)^{-1} phi with the clover
 * D-hat = D_ee - D_eo D_oo^{-1} D_oe (regular clover, Sec. 6.1.2, or the
 * exponential form, Sec. 6.1.3), given x = (D-hat^+ D-hat)^{-1} phi (packed
 * FP64 even half).  With X = (x, D_oo^{-1} D_oe x), Y = (D-hat x,
 * D_oo^{-1} D_eo^+ D-hat x):
 *   dS = 2 Re(Y^+ dH X) - 2 Re sum_x tr[dM(x) X(x) Y(x)^+],
 * the hopping part as in wdirac_force_bilinear_eo and the variation of the
 * diagonal blocks M through the clover leaves (exponential form: through the
 * derivative of the exponential).  Link variation, output P or G = 2i P U
 * (gradient = 1), scale and accumulate as in wdirac_force_eo.  U: canonical
 * fundamental links; clov64: the FP64 clover field of wdirac_clover_field for
 * the same U, m0, csw and exponential.  workspace: wdirac_workspace_bytes(ctx,
 * WDIRAC_OP_CLOVER_FORCE, 1, WDIRAC_F64).  Synchronises.  Errors: EINVAL,
 * EUNSUPPORTED (d_R not in {2, 3, 4, 6}), EHIP. */
int wdirac_force_eo_clover(const wdirac_ctx *ctx, void *out, const void *x_e, const void *UR64, const void *U,
                           const void *clov64, double m0, double csw, int exponential, double scale, int gradient,
                           int accumulate, void *workspace, void *stream);

/* Force of the odd-block determinant term S_det = -2 sum_{x odd} log|det
 * D_oo(x)| that completes the two-flavour determinant, det D = det D_oo
 * det D-hat (Sec. 5.3.3): dS_det = -2 Re sum_{x odd} tr[dM(x) D_oo(x)^{-1}].
 * For the exponential form det D_oo is constant and the result vanishes up to
 * rounding.  Arguments as in wdirac_force_eo_clover (no spinors).
 * Synchronises.  Errors: EINVAL, EUNSUPPORTED, EHIP. */
int wdirac_force_clover_logdet(const wdirac_ctx *ctx, void *out, const void *U, const void *clov64, double m0,
                               double csw, int exponential, double scale, int gradient, int accumulate,
                               void *workspace, void *stream);

/* logdet[l] (host array of one value per lattice) = sum over the odd sites
 * of lattice l of log|det D_oo(x)|, from the FP64 clover field (which stores
 * D_oo^{-1} there); S_det = -2 logdet.  workspace: wdirac_workspace_bytes(ctx,
 * WDIRAC_OP_CLOVER_FORCE, 1, WDIRAC_F64).  Synchronises.  Errors: EINVAL,
 * EUNSUPPORTED, EHIP. */
int wdirac_clover_logdet(const wdirac_ctx *ctx, double *logdet, const void *clov64, void *workspace, void *stream);

/* Multi-shift conjugate gradient (the multi-shift inversion of the RHMC,
 * Sec. 5.3.2): x_k = (D-hat^+ D-hat + sigma_k)^{-1} b for the nshift shifts
 * sigma_k >= 0 (host array, any order, 1 <= nshift <= 32), all from one
 * Krylov space: the recursion runs on the smallest shift; the solution of
 * every other shift is updated through the collinearity of the shifted
 * residuals (r_k = zeta_k r), and a shift stops being updated once
 * |zeta_k| ||r|| <= tol ||b|| / 2 (the margin covers the drift of the
 * recursive residuals).  One right-hand side, FP64, single lattice
 * (EUNSUPPORTED for a batch).  x: nshift packed FP64 even fields one after
 * the other (out; every field overwritten, no initial guess), b: packed FP64
 * even field.  stats: host array of nshift records, true_rel_resid =
 * ||b - (A + sigma_k) x_k|| / ||b|| recomputed in FP64; status ENOCONV if it
 * is above tol.  workspace: wdirac_workspace_bytes(ctx, WDIRAC_OP_MSHIFT,
 * nshift, WDIRAC_F64).  Synchronises.  Errors: EINVAL, EUNSUPPORTED, EHIP,
 * ENOCONV, EBREAKDOWN. */
int wdirac_cg_mshift_eo(const wdirac_ctx *ctx, void *x, const void *b, const void *UR64, double m0,
                        const double *shifts, int nshift, double tol, int maxit, void *workspace,
                        wdirac_cg_stats *stats, void *stream);

/* out = a x + b y for nrhs packed half spinors of precision prec (y may be
 * NULL: out = a x; out may alias x or y).  The linear combinations of
 * solver outputs that a rational function needs, e.g. r(A) phi =
 * gamma_0 phi + sum_k gamma_k x_k (Sec. 5.3.2).  Errors: EINVAL, EHIP. */
int wdirac_axpby(const wdirac_ctx *ctx, void *out, double a, const void *x, double b, const void *y, int nrhs,
                 int prec, void *stream);

/* Fermion force of S_f = phi^+ (D-hat^+ D-hat)^{-1} phi (Sec. 5.3.1, force of
 * Sec. 2.5 in even-odd form) given the solution x = (D-hat^+ D-hat)^{-1} phi
 * (packed FP64 even half): for every link, the Hermitian traceless matrix
 *   P_mu(x) = sum_a (dS/dw^a_mu(x)) T^a_F,  dS/dw^a = Im tr[T^a_R U_R Sigma_mu],
 *   Sigma_mu(x) = tr_spin[(1 - g_mu) X(x+mu) Y(x)^+ + (1 + g_mu) Y(x+mu) X(x)^+],
 * X = (x, D_oe x), Y = (D-hat x, D_eo^+ D-hat x), for the variation
 * U -> exp(i w^a T^a_F) U.  `out` (canonical complex128 [T][X][Y][Z][4][N][N])
 * receives scale * F (accumulate = 0) or out += scale * F (accumulate = 1),
 * where F = P when U is NULL, and F = G = 2i P U (U: the canonical
 * fundamental links) otherwise: G is the gradient in the convention
 * dS = Re tr(G^+ dU) for tangent variations dU = i w^a T^a U.  The same
 * formula gives the force of one pole of a rational action (Sec. 5.3.2),
 * phi^+ (D-hat^+ D-hat + sigma)^{-1} phi, with x = (D-hat^+ D-hat + sigma)^{-1}
 * phi: scale = gamma_k and accumulate = 1 sum the poles.  workspace:
 * wdirac_workspace_bytes(ctx, WDIRAC_OP_FORCE, 1, WDIRAC_F64).  Synchronises.
 * Errors: EINVAL, EHIP. */
int wdirac_force_eo(const wdirac_ctx *ctx, void *out, const void *x_e, const void *UR64, const void *U,
                    double m0, double scale, int accumulate, void *workspace, void *stream);

/* Measurement aid for the roofline (not part of the operator): sustained
 * bandwidth of a pure streaming kernel with nread input streams and one output
 * stream of `elems` 16-byte elements each, out[i] = sum_s in_s[i], one element
 * per lane, non-temporal loads and stores -- the practical ceiling of a
 * kernel with that read:write mix (the hop reads about 7 bytes per byte it
 * writes).  bufs: caller-owned device memory of (nread + 1) * elems * 16
 * bytes (inputs first, contents irrelevant; the output part is overwritten).
 * One warm-up launch, then `reps` launches timed with HIP events on stream;
 * *gbps (host) receives (bytes read + written) / time.  Synchronises.
 * Errors: EINVAL (null pointer, nread outside [1, 8], elems outside
 * [1, 2^31], reps outside [1, 1000]), EHIP. */
int wdirac_stream_probe(void *bufs, size_t elems, int nread, int reps, double *gbps, void *stream);

/* out = gamma_5 in on nrhs packed half spinors (gamma_5 = diag(1, 1, -1, -1)
 * in the basis of Sec. 2.2); out may alias in.  Errors: EINVAL, EHIP. */
int wdirac_gamma5(const wdirac_ctx *ctx, void *out, const void *in, int nrhs, int prec, void *stream);

/* Twisted-mass operators of the even-odd preconditioned Hasenbusch
 * factorisation (Sec. 6.2.1): out = W_sign(mu) in = (Q-hat + i sign mu) in,
 * Q-hat = gamma_5 D-hat with the D-hat of wdirac_apply_dhat (one factor of
 * 4 + m0 absorbed), sign = +1 or -1.  W_- = W_+^+ and W_+ W_- = D-hat^+ D-hat
 * + mu^2, so the twisted-mass monomial is a shifted solve
 * (wdirac_cg_mshift_eo with shift mu^2).  workspace: wdirac_workspace_bytes(
 * ctx, WDIRAC_OP_DHAT, nrhs, prec).  out must not alias in.  Errors: EINVAL,
 * EHIP. */
int wdirac_apply_W(const wdirac_ctx *ctx, void *out, const void *in, const void *UR, double m0, double mu, int sign,
                   int nrhs, int prec, void *workspace, void *stream);

/* Link derivative of a bilinear in the hopping term: for fixed full-lattice
 * fields X = (X_e, X_o) and Y = (Y_e, Y_o) (packed FP64 half fields), the
 * force of the functional 2 Re(Y^+ H X), in the convention of
 * wdirac_force_eo (P, or G = 2i P U when U is given; scale, accumulate).
 * wdirac_force_eo is the case X = (x, D_oe x), Y = (D-hat x, D_eo^+ D-hat x);
 * other monomials (Hasenbusch, Sec. 6.2.1) combine it with other fields.
 * Synchronises.  Errors: EINVAL, EHIP. */
int wdirac_force_bilinear_eo(const wdirac_ctx *ctx, void *out, const void *X_e, const void *X_o, const void *Y_e,
                             const void *Y_o, const void *UR64, const void *U, double scale, int accumulate,
                             void *stream);

/* HMC molecular-dynamics pieces (Sec. 5.2, 5.3) on the canonical fundamental
 * links U and momenta pi, both complex128 [T][X][Y][Z][4][N][N] (lattice
 * after lattice for a batch); momenta are Hermitian traceless matrices
 * pi = pi^a T^a (generators of wdirac_create's basis), the molecular dynamics
 * is dU/dtau = i pi U, dpi/dtau = -F, H = sum tr(pi^2) + S.
 *
 * wdirac_gauge_force: F (+)= scale * sum_a (dS_g/dw^a) T^a for the Wilson
 *   plaquette action S_g = beta sum_x sum_{mu<nu} (1 - Re tr P_mu,nu(x)/N)
 *   and the variation U -> exp(i w^a T^a) U (the convention of
 *   wdirac_force_eo's P, so fermion and gauge forces add).  F must not alias
 *   U.  Asynchronous.
 * wdirac_gauge_action: S[l] = S_g of lattice l (host array of nlat values).
 *   workspace: wdirac_workspace_bytes(ctx, WDIRAC_OP_GAUGE, 1, WDIRAC_F64).
 *   Synchronises.
 * wdirac_link_update: U <- exp(i eps pi) U on every link (exponential by
 *   scaling and squaring of the Taylor series, FP64).  Asynchronous.
 * wdirac_kinetic: K[l] = sum over the links of lattice l of tr(pi^2).
 *   workspace as for the gauge action.  Synchronises.
 * wdirac_algebra_from_components: pi = sum_a w^a T^a from the components w
 *   (device float64 [T][X][Y][Z][4][N^2-1]; e.g. Gaussian draws for the
 *   momentum refresh).  Asynchronous.
 * Errors: EINVAL, EHIP. */
int wdirac_gauge_force(const wdirac_ctx *ctx, void *F, const void *U, double beta, double scale, int accumulate,
                       void *stream);
int wdirac_gauge_action(const wdirac_ctx *ctx, double *S, const void *U, double beta, void *workspace,
                        void *stream);
int wdirac_link_update(const wdirac_ctx *ctx, void *U, const void *pi, double eps, void *stream);
int wdirac_kinetic(const wdirac_ctx *ctx, double *K, const void *pi, void *workspace, void *stream);
int wdirac_algebra_from_components(const wdirac_ctx *ctx, void *pi, const double *w, void *stream);

/* Thread-local description of the last error (empty string if none). */
const char *wdirac_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WDIRAC_H */
