// C ABI of libwdirac: argument checking, dispatch to the kernels, and the
// host loop of the conjugate-gradient solver.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/wdirac.h"
#include "wd_common.h"
#include "wd_kernels.h"

struct wdirac_tuned {
  int valid, variant, nr, xcd_remap, tblock;
};

struct wdirac_ctx {
  int N, rep, d, real;
  int nlat;                        // lattices of a batch (1 for a single lattice)
  wd::Geom g[wd::MAXLAT];
  long long spre[wd::MAXLAT + 1];  // prefix sums of the packed row strides (sites)
  long long vpre[wd::MAXLAT + 1];  // prefix sums of the lattice volumes (canonical sites)
  int hop_variant[2];   // per precision (F64, F32): one of the wd::HOP_* forms
  int hop_nr[2];        // preferred right-hand sides per colour-split block
  wdirac_tuned tuned[2][13];   // autotuned shape per (precision, nrhs)
  int xcd_remap;
  int tblock;           // t-blocked tile order (0 = lexicographic)
  int cg_check_every;   // CG iterations between host convergence checks
  double mixed_delta;   // reliable-update trigger ||r|| < delta max||r||
  int cg_graph;         // replay the CG iterations between checks as a HIP graph
  int tune_compact;     // the autotuner also times the compact-link forms
  mutable hipStream_t own = nullptr;   // the library's stream for graph capture (created on first use)
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define WD_HIP(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(WDIRAC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define WD_TRY(expr)            \
  do {                          \
    int rc_ = (expr);           \
    if (rc_ != WDIRAC_OK) return rc_; \
  } while (0)

int rep_dim(int N, int rep) {
  switch (rep) {
    case WDIRAC_FUND: return N;
    case WDIRAC_ADJ: return N * N - 1;
    case WDIRAC_SYM: return N * (N + 1) / 2;
    case WDIRAC_ASYM: return N * (N - 1) / 2;
  }
  return 0;
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

size_t half_bytes(const wdirac_ctx *c, int nrhs, int prec) {
  return (size_t)nrhs * 4 * c->d * c->spre[c->nlat] * (prec == WDIRAC_F64 ? 16 : 8);
}

// Independent systems of a packed field: the right-hand sides of a single
// lattice, or the lattices of a batch (one right-hand side each).
int nsys_of(const wdirac_ctx *c, int nrhs) { return c->nlat == 1 ? nrhs : c->nlat; }

wd::FieldShape shape(const wdirac_ctx *c, int nrhs) {
  wd::FieldShape f{};
  f.ncomp = 4 * c->d;
  f.nsys = nsys_of(c, nrhs);
  f.maxvh = 0;
  for (int s = 0; s < f.nsys; ++s) {
    const int l = c->nlat == 1 ? 0 : s;
    f.vh[s] = c->g[l].Vh;
    f.stride[s] = c->g[l].stride;
    f.off[s] = c->nlat == 1 ? (long long)s * f.ncomp * c->g[0].stride : (long long)f.ncomp * c->spre[l];
    f.maxvh = std::max(f.maxvh, f.vh[s]);
  }
  return f;
}

hipStream_t S(void *s) { return static_cast<hipStream_t>(s); }

int check_ctx(const wdirac_ctx *c) {
  if (!c) return fail(WDIRAC_EINVAL, "ctx is NULL");
  return WDIRAC_OK;
}
int check_prec(int prec) {
  if (prec != WDIRAC_F64 && prec != WDIRAC_F32) return fail(WDIRAC_EINVAL, "prec must be WDIRAC_F64 or WDIRAC_F32");
  return WDIRAC_OK;
}
int check_nrhs(int nrhs) {
  if (nrhs < 1 || nrhs > 12) return fail(WDIRAC_EINVAL, "nrhs must be in [1, 12]");
  return WDIRAC_OK;
}
int check_nrhs(const wdirac_ctx *c, int nrhs) {
  WD_TRY(check_nrhs(nrhs));
  if (c->nlat > 1 && nrhs != 1) return fail(WDIRAC_EINVAL, "a batch of lattices carries one right-hand side");
  return WDIRAC_OK;
}
int check_parity(int p) {
  if (p != 0 && p != 1) return fail(WDIRAC_EINVAL, "parity must be 0 (even) or 1 (odd)");
  return WDIRAC_OK;
}
int check_ptr(const void *p, const char *name) {
  if (!p) return fail(WDIRAC_EINVAL, std::string(name) + " is NULL");
  return WDIRAC_OK;
}

// Workspace carving: consecutive 256-byte aligned pieces.
struct Carver {
  char *base;
  size_t off = 0;
  void *take(size_t n) {
    void *p = base ? base + off : nullptr;
    off += align256(n);
    return p;
  }
};

size_t partial_doubles(const wdirac_ctx *c, int nrhs) {
  // rows (one per system, twice for the real and imaginary rows of a dot) of
  // the longest per-tile row any producer writes: the smallest tiles are the
  // 32-site tiles of the multi-rhs hop with two lanes per site
  int mx = 0;
  for (int l = 0; l < c->nlat; ++l) mx = std::max(mx, (c->g[l].Vh + 31) / 32);
  return (size_t)2 * nsys_of(c, nrhs) * mx;
}

struct CgWork {
  void *r, *p, *q, *t, *u, *v;            // FP64
  void *r32, *p32, *x32, *q32, *t32, *u32, *v32;  // FP32 (mixed)
  double *P1, *P2;
  wd::CgScalars *sc;
  size_t bytes;
};

CgWork carve_cg(const wdirac_ctx *c, int nrhs, int mode, void *ws) {
  Carver cv{static_cast<char *>(ws)};
  CgWork w{};
  const size_t h64 = half_bytes(c, nrhs, WDIRAC_F64), h32 = half_bytes(c, nrhs, WDIRAC_F32);
  w.r = cv.take(h64); w.p = cv.take(h64); w.q = cv.take(h64);
  w.t = cv.take(h64); w.u = cv.take(h64); w.v = cv.take(h64);
  if (mode == WDIRAC_CG_MIXED) {
    w.r32 = cv.take(h32); w.p32 = cv.take(h32); w.x32 = cv.take(h32); w.q32 = cv.take(h32);
    w.t32 = cv.take(h32); w.u32 = cv.take(h32); w.v32 = cv.take(h32);
  }
  w.P1 = static_cast<double *>(cv.take(partial_doubles(c, nrhs) * sizeof(double)));
  w.P2 = static_cast<double *>(cv.take(partial_doubles(c, nrhs) * sizeof(double)));
  w.sc = static_cast<wd::CgScalars *>(cv.take(nsys_of(c, nrhs) * sizeof(wd::CgScalars)));
  w.bytes = cv.off;
  return w;
}

struct MsWork {
  void *r, *q, *t, *u, *v, *p;   // FP64 half fields; p holds nshift fields
  double *P1, *P2, *P3;
  wd::MsScalars *sc;
  size_t bytes;
};

MsWork carve_ms(const wdirac_ctx *c, int nshift, void *ws) {
  Carver cv{static_cast<char *>(ws)};
  MsWork w{};
  const size_t h = half_bytes(c, 1, WDIRAC_F64);
  w.r = cv.take(h); w.q = cv.take(h); w.t = cv.take(h); w.u = cv.take(h); w.v = cv.take(h);
  w.p = cv.take((size_t)nshift * h);
  w.P1 = static_cast<double *>(cv.take(partial_doubles(c, 1) * sizeof(double)));
  w.P2 = static_cast<double *>(cv.take(partial_doubles(c, 1) * sizeof(double)));
  w.P3 = static_cast<double *>(cv.take(partial_doubles(c, 1) * sizeof(double)));
  w.sc = static_cast<wd::MsScalars *>(cv.take(sizeof(wd::MsScalars)));
  w.bytes = cv.off;
  return w;
}

// Bytes of the represented links of the whole context in precision prec; the
// compact fundamental copy (two-index representations with compact forms)
// follows them in the same links field.
size_t rep_links_bytes(const wdirac_ctx *c, int prec) {
  return (size_t)8 * c->d * c->d * c->spre[c->nlat] * (prec == WDIRAC_F64 ? 8 : 4) * (c->real ? 1 : 2);
}
size_t compact_links_bytes(const wdirac_ctx *c, int prec) {
  if (!wd::compact_links_ok(c->N, c->rep)) return 0;
  return (size_t)8 * c->N * c->N * c->spre[c->nlat] * (prec == WDIRAC_F64 ? 16 : 8);
}

// Right-hand sides per colour-split block: the largest supported divisor of
// nrhs not above the preference.
int effective_nr(const wdirac_ctx *c, int pref, int nrhs, int prec, int variant) {
  // site-parallel form: 4 right-hand sides across the lanes of a wavefront, or 1
  if (variant == wd::HOP_SITE) return (pref >= 4 && nrhs % 4 == 0) ? 4 : 1;
  for (int nr = std::min(pref, variant == wd::HOP_MULTI ? 12 : 6); nr > 1; --nr)
    if (nrhs % nr == 0 && wd::hop_nr_supported(c->N, c->d, prec, variant, nr)) return nr;
  return 1;
}

// One hopping-term launch over every lattice of the context.  counts/prow
// (nullable) receive the layout of the per-tile partial sums.
int hop(const wdirac_ctx *c, void *out, const void *in, const void *UR, int out_parity, int dagger, int nrhs,
        double alpha, const void *xadd, double beta, int prec, double *partial, hipStream_t st,
        wd::Counts *counts = nullptr, int *prow = nullptr) {
  int variant = c->hop_variant[prec], pref = c->hop_nr[prec], remap = c->xcd_remap, tblock = c->tblock;
  const wdirac_tuned &tn = c->tuned[prec][nrhs];
  if (tn.valid) {
    variant = tn.variant;
    pref = tn.nr;
    remap = tn.xcd_remap;
    tblock = tn.tblock;
  }
  wd::HopArgs a;
  a.out = out;
  a.in = in;
  a.links = UR;
  a.flinks = wd::compact_links_ok(c->N, c->rep) ? static_cast<const char *>(UR) + rep_links_bytes(c, prec) : nullptr;
  a.xadd = xadd;
  a.nlat = c->nlat;
  for (int l = 0; l < c->nlat; ++l) {
    a.lat[l].g = c->g[l];
    a.lat[l].tile0 = a.lat[l].ntiles = 0;
    a.lat[l].soff = c->nlat == 1 ? 0 : (long long)4 * c->d * c->spre[l];
    a.lat[l].loff = (long long)8 * c->d * c->d * c->spre[l];
    a.lat[l].floff = (long long)8 * c->N * c->N * c->spre[l];
  }
  a.parity = out_parity;
  a.xcd_remap = remap;
  a.alpha = alpha;
  a.beta = beta;
  a.partial = partial;
  a.prow = a.ntiles = a.ngroups = 0;
  a.tblock = c->nlat == 1 ? tblock : 0;
  a.tiles_per_tx = 0;
  wd::Counts cnt{};
  int pr = 0;
  WD_HIP(wd::launch_hop(a, c->N, c->rep, c->d, c->real, prec, dagger, nrhs, variant,
                        effective_nr(c, pref, nrhs, prec, variant), st, &cnt, &pr));
  if (counts) *counts = cnt;
  if (prow) *prow = pr;
  return WDIRAC_OK;
}

// D_ee in (parity 0) or D_oo^{-1} in (parity 1) with a clover field, lattice
// by lattice; out may alias in.
int clover_apply(const wdirac_ctx *c, void *out, const void *in, const void *clov, int parity, int nrhs, int prec,
                 hipStream_t st) {
  const size_t cb = prec == WDIRAC_F64 ? 16 : 8;
  for (int l = 0; l < c->nlat; ++l) {
    const size_t so = (size_t)4 * c->d * c->spre[l] * cb;
    const size_t co = (size_t)4 * c->d * (2 * c->d + 1) * c->spre[l] * cb;
    WD_HIP(wd::launch_clover_apply(static_cast<char *>(out) + so, static_cast<const char *>(in) + so,
                                   static_cast<const char *>(clov) + co, c->g[l], c->d, parity, nrhs, prec, st));
  }
  return WDIRAC_OK;
}

// out = D-hat in (dagger = 0) or D-hat^+ in (dagger = 1); tmp is an odd half field.
// Without a clover field: D-hat = (4+m)^2 - D_eo D_oe (Sec. 5.3.3, one factor
// of 4+m absorbed).  With one: D-hat = D_ee - D_eo D_oo^{-1} D_oe, whose
// diagonal blocks are Hermitian, so the adjoint only swaps to the dagger hops.
int dhat(const wdirac_ctx *c, void *out, const void *in, const void *UR, double m0, int dagger, int nrhs, int prec,
         void *tmp, double *partial, hipStream_t st, wd::Counts *counts = nullptr, int *prow = nullptr,
         const void *clov = nullptr) {
  if (clov) {
    WD_TRY(hop(c, tmp, in, UR, 1, dagger, nrhs, 0.0, nullptr, 1.0, prec, nullptr, st));
    WD_TRY(clover_apply(c, tmp, tmp, clov, 1, nrhs, prec, st));
    WD_TRY(clover_apply(c, out, in, clov, 0, nrhs, prec, st));
    WD_TRY(hop(c, out, tmp, UR, 0, dagger, nrhs, 1.0, out, -1.0, prec, partial, st, counts, prow));
    return WDIRAC_OK;
  }
  const double m4 = (4.0 + m0) * (4.0 + m0);
  WD_TRY(hop(c, tmp, in, UR, 1, dagger, nrhs, 0.0, nullptr, 1.0, prec, nullptr, st));
  WD_TRY(hop(c, out, tmp, UR, 0, dagger, nrhs, m4, in, -1.0, prec, partial, st, counts, prow));
  return WDIRAC_OK;
}

// Canonical <-> packed half spinors, lattice by lattice.  Canonical batch
// layout: [lattice][T][X][Y][Z][4][d] (one right-hand side).
int pack(const wdirac_ctx *c, void *packed, void *canon, int parity, int nrhs, int prec, int unpack, hipStream_t st) {
  const size_t cb = prec == WDIRAC_F64 ? 16 : 8;
  for (int l = 0; l < c->nlat; ++l) {
    char *P = static_cast<char *>(packed) + (size_t)4 * c->d * c->spre[l] * cb;
    char *C = static_cast<char *>(canon) + (size_t)4 * c->d * c->vpre[l] * cb;
    WD_HIP(wd::launch_pack_spinor(P, C, c->g[l], c->d, parity, nrhs, prec, unpack, st));
  }
  return WDIRAC_OK;
}

// Workspace of the clover force: the three FP64 half fields of the
// pseudofermion force (whole batch), then the per-lattice scratch of the
// largest lattice: F (6 d^2 V), K (12 d^2 V), leaf matrices (24 N^2 V) complex
// FP64, and the log-det partial sums.
struct CloverForceWs {
  void *z_o, *y_e, *w_o;
  double *F, *K, *G, *Us, *part, *dtmp;
  size_t bytes;
};

CloverForceWs carve_clover_force(const wdirac_ctx *c, void *base) {
  Carver cv{static_cast<char *>(base)};
  CloverForceWs w;
  const size_t h = half_bytes(c, 1, WDIRAC_F64);
  w.z_o = cv.take(h);
  w.y_e = cv.take(h);
  w.w_o = cv.take(h);
  size_t V = 0;
  int nb = 0;
  for (int l = 0; l < c->nlat; ++l) {
    V = std::max(V, 2 * (size_t)c->g[l].Vh);
    nb = std::max(nb, wd::clover_logdet_blocks(c->g[l]));
  }
  const size_t d2 = (size_t)c->d * c->d, n2 = (size_t)c->N * c->N;
  w.F = static_cast<double *>(cv.take(6 * d2 * V * 16));
  w.K = static_cast<double *>(cv.take(12 * d2 * V * 16));
  w.G = static_cast<double *>(cv.take(24 * n2 * V * 16));
  w.Us = static_cast<double *>(cv.take(4 * n2 * V * 16));
  w.part = static_cast<double *>(cv.take((size_t)nb * sizeof(double)));
  w.dtmp = static_cast<double *>(cv.take(sizeof(double)));
  w.bytes = cv.off;
  return w;
}

}  // namespace

extern "C" {

const char *wdirac_last_error(void) { return g_err.c_str(); }

int wdirac_create_batch(wdirac_ctx **ctx, int Ng, int rep, const wdirac_geom *geoms, int nlat) {
  g_err.clear();
  if (!ctx) return fail(WDIRAC_EINVAL, "ctx is NULL");
  *ctx = nullptr;
  if (!geoms) return fail(WDIRAC_EINVAL, "geom is NULL");
  if (nlat < 1 || nlat > wd::MAXLAT) return fail(WDIRAC_EINVAL, "a batch holds 1 to 8 lattices");
  if (rep < WDIRAC_FUND || rep > WDIRAC_ASYM) return fail(WDIRAC_EINVAL, "unknown representation");
  if (Ng < 2 || Ng > 4) return fail(WDIRAC_EUNSUPPORTED, "Ng must be 2, 3 or 4");
  if (Ng == 2 && rep == WDIRAC_ASYM) return fail(WDIRAC_EUNSUPPORTED, "SU(2) 2AS is one-dimensional (d_R = 1)");
  const int d = rep_dim(Ng, rep);
  int64_t total = 0;
  for (int l = 0; l < nlat; ++l) {
    int64_t V = 1;
    for (int mu = 0; mu < 4; ++mu) {
      const int L = geoms[l].dims[mu];
      if (L < 2 || (L & 1)) return fail(WDIRAC_EINVAL, "every lattice extent must be even and >= 2");
      if (geoms[l].bc[mu] != 1 && geoms[l].bc[mu] != -1) return fail(WDIRAC_EINVAL, "bc must be +1 or -1");
      V *= L;
    }
    if (V > (int64_t)1 << 30) return fail(WDIRAC_EINVAL, "lattice volume above 2^30 sites");
    total += V;
  }
  // every packed offset must stay addressable by the kernels' 64-bit arithmetic
  // and every per-lattice row index by 32-bit ints (checked per lattice above)
  if (total * 12 * d * d > ((int64_t)1 << 45)) return fail(WDIRAC_EINVAL, "batch too large");
  wdirac_ctx *c = new wdirac_ctx();
  c->N = Ng;
  c->rep = rep;
  c->d = d;
  c->real = rep == WDIRAC_ADJ;
  c->nlat = nlat;
  c->spre[0] = c->vpre[0] = 0;
  for (int l = 0; l < nlat; ++l) {
    wd::Geom &g = c->g[l];
    g.T = geoms[l].dims[0];
    g.X = geoms[l].dims[1];
    g.Y = geoms[l].dims[2];
    g.Z = geoms[l].dims[3];
    const int64_t V = (int64_t)g.T * g.X * g.Y * g.Z;
    g.Vh = (int)(V / 2);
    // Rows of whole 256-site tiles (see hop.hip).  A row pitch that is a
    // multiple of 16 KB (1024 FP64 complex entries) puts the component rows
    // a wavefront streams together on the same HBM channel pattern; such
    // strides are padded by 256 entries (7-read/1-write streaming probe with
    // 256 MiB rows: 5.74 TB/s, rows 4 KB off a 16 KB multiple: 6.04 TB/s).
    g.stride = (g.Vh + 255) & ~255;
    if (g.stride % 1024 == 0) g.stride += 256;
    for (int mu = 0; mu < 4; ++mu) g.bc[mu] = geoms[l].bc[mu];
    c->spre[l + 1] = c->spre[l] + g.stride;
    c->vpre[l + 1] = c->vpre[l] + V;
  }
  c->hop_variant[0] = wd::HOP_COLOUR;
  c->hop_variant[1] = wd::HOP_COLOUR;
  c->hop_nr[0] = c->hop_nr[1] = 4;
  std::memset(c->tuned, 0, sizeof(c->tuned));
  c->xcd_remap = 1;
  c->tblock = 0;
  c->cg_check_every = 4;
  c->mixed_delta = 0.01;
  c->cg_graph = 1;
  c->tune_compact = 1;
  *ctx = c;
  return WDIRAC_OK;
}

int wdirac_create(wdirac_ctx **ctx, int Ng, int rep, const wdirac_geom *geom) {
  return wdirac_create_batch(ctx, Ng, rep, geom, 1);
}

int wdirac_destroy(wdirac_ctx *ctx) {
  if (ctx && ctx->own) (void)hipStreamDestroy(ctx->own);
  delete ctx;
  return WDIRAC_OK;
}

int wdirac_rep_info(const wdirac_ctx *ctx, int *d_R, int *real_links) {
  WD_TRY(check_ctx(ctx));
  if (d_R) *d_R = ctx->d;
  if (real_links) *real_links = ctx->real;
  return WDIRAC_OK;
}

size_t wdirac_field_bytes(const wdirac_ctx *ctx, int kind, int nrhs, int prec) {
  if (!ctx || (prec != WDIRAC_F64 && prec != WDIRAC_F32)) return 0;
  const size_t el = prec == WDIRAC_F64 ? 8 : 4;
  if (kind == WDIRAC_FIELD_HALF_SPINOR) {
    if (nrhs < 1 || nrhs > 12) return 0;
    return half_bytes(ctx, nrhs, prec);
  }
  if (kind == WDIRAC_FIELD_LINKS) return rep_links_bytes(ctx, prec) + compact_links_bytes(ctx, prec);
  if (kind == WDIRAC_FIELD_CLOVER)
    return wd::clover_supported(ctx->d) ? (size_t)4 * ctx->d * (2 * ctx->d + 1) * ctx->spre[ctx->nlat] * 2 * el : 0;
  return 0;
}

size_t wdirac_workspace_bytes(const wdirac_ctx *ctx, int op, int nrhs, int prec) {
  if (!ctx) return 0;
  if (op == WDIRAC_OP_GAUGE) {   // reductions over links and sites
    int mx = 0;
    for (int l = 0; l < ctx->nlat; ++l) mx = std::max(mx, wd::kinetic_blocks(ctx->g[l]));
    return align256((size_t)mx * sizeof(double)) + align256(sizeof(double));
  }
  if (op == WDIRAC_OP_CLOVER) {   // scratch of the clover-field construction
    if (!wd::clover_supported(ctx->d)) return 0;
    int mx = 0;
    for (int l = 0; l < ctx->nlat; ++l) mx = std::max(mx, ctx->g[l].Vh);
    // F, then the structure-of-arrays copy of the links
    return align256((size_t)6 * ctx->d * ctx->d * 2 * mx * 16) + align256((size_t)4 * ctx->N * ctx->N * 2 * mx * 16);
  }
  if (op == WDIRAC_OP_CLOVER_FORCE) {
    if (!wd::clover_supported(ctx->d)) return 0;
    return carve_clover_force(ctx, nullptr).bytes;
  }
  if (op == WDIRAC_OP_MSHIFT) {   // nrhs = number of shifts
    if (nrhs < 1 || nrhs > wd::MAXSHIFT || prec != WDIRAC_F64 || ctx->nlat != 1) return 0;
    return carve_ms(ctx, nrhs, nullptr).bytes;
  }
  if (nrhs < 1 || nrhs > 12 || (ctx->nlat > 1 && nrhs != 1)) return 0;
  switch (op) {
    case WDIRAC_OP_DHAT:
      if (prec != WDIRAC_F64 && prec != WDIRAC_F32) return 0;
      return align256(half_bytes(ctx, nrhs, prec));
    case WDIRAC_OP_CG:
      if (prec != WDIRAC_CG_F64 && prec != WDIRAC_CG_MIXED) return 0;
      return carve_cg(ctx, nrhs, prec, nullptr).bytes;
    case WDIRAC_OP_FORCE:
      return 3 * align256(half_bytes(ctx, 1, WDIRAC_F64));
    case WDIRAC_OP_NORM:
    case WDIRAC_OP_DOT:
      return align256(partial_doubles(ctx, nrhs) * sizeof(double)) + align256(2 * wd::MAXSYS * sizeof(double));
    case WDIRAC_OP_TUNE:
      if (prec != WDIRAC_F64 && prec != WDIRAC_F32) return 0;
      return 3 * align256(half_bytes(ctx, nrhs, prec));
  }
  return 0;
}

int wdirac_set_option(wdirac_ctx *ctx, int option, double value) {
  WD_TRY(check_ctx(ctx));
  switch (option) {
    case WDIRAC_OPT_HOP_VARIANT_F64:
    case WDIRAC_OPT_HOP_VARIANT_F32: {
      const int v = (int)value;
      if (v < wd::HOP_SITE || v > wd::HOP_MULTI) return fail(WDIRAC_EINVAL, "hop variant out of range");
      if (!wd::hop_variant_ok(ctx->N, ctx->rep, ctx->d, v))
        return fail(WDIRAC_EUNSUPPORTED, "hop variant not available for this representation");
      ctx->hop_variant[option == WDIRAC_OPT_HOP_VARIANT_F64 ? 0 : 1] = v;
      return WDIRAC_OK;
    }
    case WDIRAC_OPT_XCD_REMAP:
      ctx->xcd_remap = value != 0.0;
      return WDIRAC_OK;
    case WDIRAC_OPT_CG_CHECK_EVERY:
      if (value < 1 || value > 1000) return fail(WDIRAC_EINVAL, "check interval must be in [1, 1000]");
      ctx->cg_check_every = (int)value;
      return WDIRAC_OK;
    case WDIRAC_OPT_MIXED_DELTA:
      if (!(value > 0.0 && value < 1.0)) return fail(WDIRAC_EINVAL, "delta must be in (0, 1)");
      ctx->mixed_delta = value;
      return WDIRAC_OK;
    case WDIRAC_OPT_CG_GRAPH:
      if (value != 0.0 && value != 1.0) return fail(WDIRAC_EINVAL, "CG graph option must be 0 or 1");
      ctx->cg_graph = (int)value;
      return WDIRAC_OK;
    case WDIRAC_OPT_TILE_TBLOCK:
      if (!(value >= -99 && value <= 64)) return fail(WDIRAC_EINVAL, "t-block must be in [-99, 64]");
      ctx->tblock = (int)value;
      return WDIRAC_OK;
    case WDIRAC_OPT_TUNE_COMPACT:
      if (value != 0.0 && value != 1.0) return fail(WDIRAC_EINVAL, "compact tuning option must be 0 or 1");
      ctx->tune_compact = (int)value;
      return WDIRAC_OK;
    case WDIRAC_OPT_HOP_NR_F64:
    case WDIRAC_OPT_HOP_NR_F32:
      if (!(value >= 1 && value <= 12)) return fail(WDIRAC_EINVAL, "right-hand sides per block must be in [1, 12]");
      ctx->hop_nr[option == WDIRAC_OPT_HOP_NR_F64 ? 0 : 1] = (int)value;
      return WDIRAC_OK;
  }
  return fail(WDIRAC_EINVAL, "unknown option");
}

int wdirac_autotune(wdirac_ctx *ctx, const void *UR, int prec, int nrhs, void *workspace, wdirac_tuning *best,
                    void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(UR, "UR"));
  WD_TRY(check_ptr(workspace, "workspace"));
  WD_TRY(check_prec(prec));
  WD_TRY(check_nrhs(ctx, nrhs));
  const hipStream_t st = S(stream);
  Carver cv{static_cast<char *>(workspace)};
  const size_t hb = half_bytes(ctx, nrhs, prec);
  void *f0 = cv.take(hb), *f1 = cv.take(hb), *f2 = cv.take(hb);
  WD_HIP(hipMemsetAsync(f0, 0, hb, st));
  WD_HIP(hipMemsetAsync(f1, 0, hb, st));
  WD_HIP(hipMemsetAsync(f2, 0, hb, st));
  struct Cand {
    int variant, nr, remap, tblock;
  };
  std::vector<Cand> cands;
  // sub-lattice sweeps (negative codes -(10 bx + by)) only where a work item
  // holds several right-hand sides; shapes whose code does not fit the
  // lattice fall back to lexicographic order in the launch
  const int tbs[] = {0, 2, 4, 8, -23, -33, -43, -63, -39};
  for (int tb : tbs) {
    if (tb < 0 && nrhs < 4) continue;
    if (tb > 0 && (ctx->nlat > 1 || ctx->g[0].T % tb)) continue;
    if (tb < 0 && (ctx->nlat > 1 || ctx->g[0].X % ((-tb) / 10))) continue;
    for (int remap = 0; remap < 2; ++remap) {
      for (int v = wd::HOP_COLOUR; v <= wd::HOP_MULTI; ++v) {
        if (!wd::hop_variant_ok(ctx->N, ctx->rep, ctx->d, v)) continue;
        if (!ctx->tune_compact && (v == wd::HOP_COMPACT || v == wd::HOP_COMPACT_PAIR)) continue;
        // the multi-rhs form only where it shares links (nr > 1)
        for (int nr : {1, 2, 3, 4, 6, 12})
          if ((v != wd::HOP_MULTI || nr > 1) && effective_nr(ctx, nr, nrhs, prec, v) == nr)
            cands.push_back({v, nr, remap, tb});
      }
      if (wd::hop_variant_ok(ctx->N, ctx->rep, ctx->d, wd::HOP_SITE)) {
        cands.push_back({wd::HOP_SITE, 1, remap, tb});
        if (nrhs % 4 == 0) cands.push_back({wd::HOP_SITE, 4, remap, tb});
      }
    }
  }
  hipEvent_t e0, e1;
  WD_HIP(hipEventCreate(&e0));
  WD_HIP(hipEventCreate(&e1));
  wdirac_tuned &slot = ctx->tuned[prec][nrhs];
  int rc = WDIRAC_OK;
  // Mean time of `reps` back-to-back launches of candidate cd (after 4
  // untimed), alternating D_eo f0 -> f1 and D_oe f1 -> f2: every other
  // launch reads the output just written, as between the hops of a solver.
  auto time_cand = [&](const Cand &cd, int reps, float *ms) {
    slot = wdirac_tuned{1, cd.variant, cd.nr, cd.remap, cd.tblock};
    auto launch = [&](int k) {
      return hop(ctx, (k & 1) ? f2 : f1, (k & 1) ? f1 : f0, UR, k & 1, 0, nrhs, 0.0, nullptr, 1.0, prec, nullptr,
                 st);
    };
    for (int k = 0; k < 4 && rc == WDIRAC_OK; ++k) rc = launch(k);
    if (rc == WDIRAC_OK && hipEventRecord(e0, st) != hipSuccess) rc = fail(WDIRAC_EHIP, "hipEventRecord");
    for (int k = 0; k < reps && rc == WDIRAC_OK; ++k) rc = launch(k);
    if (rc == WDIRAC_OK && hipEventRecord(e1, st) != hipSuccess) rc = fail(WDIRAC_EHIP, "hipEventRecord");
    if (rc == WDIRAC_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(WDIRAC_EHIP, "hipEventSynchronize");
    *ms = 0.0f;
    if (rc == WDIRAC_OK && hipEventElapsedTime(ms, e0, e1) != hipSuccess) rc = fail(WDIRAC_EHIP, "hipEventElapsedTime");
    *ms /= (float)reps;
  };
  // Pass 1: every candidate, 10 launches, then again over about 5 ms (at
  // most 100 launches), keeping the faster.  Pass 2: the best six again,
  // five interleaved rounds of at least 20 launches and about 25 ms each (so
  // that millisecond-scale kernels are timed over many launches), keeping
  // each one's fastest round; the spread of the pick's rounds is reported.
  std::vector<std::pair<float, int>> t1;
  {
    // untimed: about 50 ms of launches first, so that no candidate is timed
    // while the clocks are still ramping up
    float ms;
    time_cand(cands.front(), 4, &ms);
    if (rc == WDIRAC_OK) time_cand(cands.front(), std::min(1000, std::max(4, (int)(50.0f / std::max(ms, 1e-3f)))), &ms);
  }
  for (size_t i = 0; i < cands.size() && rc == WDIRAC_OK; ++i) {
    float ms, ms2 = 1e30f;
    time_cand(cands[i], 10, &ms);
    const int n2 = std::min(100, (int)(5.0f / std::max(ms, 1e-3f)));
    if (rc == WDIRAC_OK && n2 > 10) time_cand(cands[i], n2, &ms2);
    t1.push_back({std::min(ms, ms2), (int)i});
  }
  float best_ms = 1e30f, best_worst = 0.0f, second_ms = 0.0f;
  Cand pick = cands.front();
  if (rc == WDIRAC_OK) {
    std::sort(t1.begin(), t1.end());
    const size_t nfin = std::min<size_t>(6, t1.size());
    std::vector<float> t2(nfin, 1e30f), t2w(nfin, 0.0f);
    std::vector<int> reps(nfin);
    for (size_t j = 0; j < nfin; ++j)
      reps[j] = std::min(1000, std::max(20, (int)(25.0f / std::max(t1[j].first, 1e-3f))));
    for (int round = 0; round < 5 && rc == WDIRAC_OK; ++round)
      for (size_t j = 0; j < nfin && rc == WDIRAC_OK; ++j) {
        float ms;
        time_cand(cands[t1[j].second], reps[j], &ms);
        t2[j] = std::min(t2[j], ms);
        t2w[j] = std::max(t2w[j], ms);
      }
    size_t jb = 0;
    for (size_t j = 0; j < nfin; ++j)
      if (t2[j] < best_ms) {
        best_ms = t2[j];
        jb = j;
      }
    pick = cands[t1[jb].second];
    best_worst = t2w[jb];
    second_ms = 1e30f;
    for (size_t j = 0; j < nfin; ++j)
      if (j != jb) second_ms = std::min(second_ms, t2[j]);
    if (nfin < 2) second_ms = best_ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != WDIRAC_OK) {
    slot.valid = 0;
    return rc;
  }
  slot = wdirac_tuned{1, pick.variant, pick.nr, pick.remap, pick.tblock};
  if (best) {
    best->variant = pick.variant;
    best->nr = pick.nr;
    best->xcd_remap = pick.remap;
    best->tblock = pick.tblock;
    best->candidates = (int)cands.size();
    best->us = best_ms * 1e3;
    best->spread = best_ms > 0.0f ? (best_worst - best_ms) / best_ms : 0.0;
    best->runner_up_us = second_ms * 1e3;
  }
  return WDIRAC_OK;
}

int wdirac_pack_spinor(const wdirac_ctx *ctx, void *packed, const void *canon, int parity, int nrhs, int prec,
                       void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(packed, "packed"));
  WD_TRY(check_ptr(canon, "canon"));
  WD_TRY(check_parity(parity));
  WD_TRY(check_nrhs(ctx, nrhs));
  WD_TRY(check_prec(prec));
  return pack(ctx, packed, const_cast<void *>(canon), parity, nrhs, prec, 0, S(stream));
}

int wdirac_unpack_spinor(const wdirac_ctx *ctx, void *canon, const void *packed, int parity, int nrhs, int prec,
                         void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(packed, "packed"));
  WD_TRY(check_ptr(canon, "canon"));
  WD_TRY(check_parity(parity));
  WD_TRY(check_nrhs(ctx, nrhs));
  WD_TRY(check_prec(prec));
  return pack(ctx, const_cast<void *>(packed), canon, parity, nrhs, prec, 1, S(stream));
}

int wdirac_rep_links(const wdirac_ctx *ctx, void *UR, const void *U, int prec, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(UR, "UR"));
  WD_TRY(check_ptr(U, "U"));
  WD_TRY(check_prec(prec));
  const size_t el = (prec == WDIRAC_F64 ? 8 : 4) * (ctx->real ? 1 : 2);
  for (int l = 0; l < ctx->nlat; ++l) {
    const char *Ul = static_cast<const char *>(U) + (size_t)ctx->vpre[l] * 4 * ctx->N * ctx->N * 16;
    char *URl = static_cast<char *>(UR) + (size_t)8 * ctx->d * ctx->d * ctx->spre[l] * el;
    char *Fl = nullptr;
    if (wd::compact_links_ok(ctx->N, ctx->rep))
      Fl = static_cast<char *>(UR) + rep_links_bytes(ctx, prec) +
           (size_t)8 * ctx->N * ctx->N * ctx->spre[l] * (prec == WDIRAC_F64 ? 16 : 8);
    WD_HIP(wd::launch_rep_links(Ul, URl, Fl, ctx->g[l], ctx->N, ctx->rep, prec, S(stream)));
  }
  return WDIRAC_OK;
}

int wdirac_unpack_links(const wdirac_ctx *ctx, void *UR_canon, const void *UR, int prec, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(UR, "UR"));
  WD_TRY(check_ptr(UR_canon, "UR_canon"));
  WD_TRY(check_prec(prec));
  const size_t el = (prec == WDIRAC_F64 ? 8 : 4) * (ctx->real ? 1 : 2);
  const size_t cel = ctx->real ? 8 : 16;
  for (int l = 0; l < ctx->nlat; ++l) {
    char *Cl = static_cast<char *>(UR_canon) + (size_t)ctx->vpre[l] * 4 * ctx->d * ctx->d * cel;
    const char *URl = static_cast<const char *>(UR) + (size_t)8 * ctx->d * ctx->d * ctx->spre[l] * el;
    WD_HIP(wd::launch_unpack_links(Cl, URl, ctx->g[l], ctx->d, ctx->real, prec, S(stream)));
  }
  return WDIRAC_OK;
}

int wdirac_dslash_eo(const wdirac_ctx *ctx, void *out, const void *in, const void *UR, int out_parity, int dagger,
                     int nrhs, double alpha, const void *x_add, double beta, int prec, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(out, "out"));
  WD_TRY(check_ptr(in, "in"));
  WD_TRY(check_ptr(UR, "UR"));
  WD_TRY(check_parity(out_parity));
  WD_TRY(check_nrhs(ctx, nrhs));
  WD_TRY(check_prec(prec));
  if (dagger != 0 && dagger != 1) return fail(WDIRAC_EINVAL, "dagger must be 0 or 1");
  if (in == out) return fail(WDIRAC_EINVAL, "in and out must not alias");
  return hop(ctx, out, in, UR, out_parity, dagger, nrhs, alpha, x_add, beta, prec, nullptr, S(stream));
}

static int apply_M(const wdirac_ctx *ctx, void *out, const void *in, double m0, int inverse, int nrhs, int prec,
                   void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(out, "out"));
  WD_TRY(check_ptr(in, "in"));
  WD_TRY(check_nrhs(ctx, nrhs));
  WD_TRY(check_prec(prec));
  if (inverse && 4.0 + m0 == 0.0) return fail(WDIRAC_EINVAL, "4 + m0 = 0 has no inverse");
  const double f = inverse ? 1.0 / (4.0 + m0) : 4.0 + m0;
  WD_HIP(wd::launch_lincomb(out, f, in, 0.0, nullptr, shape(ctx, nrhs), prec, S(stream)));
  return WDIRAC_OK;
}

int wdirac_apply_Mee(const wdirac_ctx *ctx, void *out, const void *in, double m0, int inverse, int nrhs, int prec,
                     void *stream) {
  return apply_M(ctx, out, in, m0, inverse, nrhs, prec, stream);
}

int wdirac_apply_Moo(const wdirac_ctx *ctx, void *out, const void *in, double m0, int inverse, int nrhs, int prec,
                     void *stream) {
  return apply_M(ctx, out, in, m0, inverse, nrhs, prec, stream);
}

int wdirac_apply_dhat(const wdirac_ctx *ctx, void *out, const void *in, const void *UR, double m0, int dagger,
                      int nrhs, int prec, void *workspace, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(out, "out"));
  WD_TRY(check_ptr(in, "in"));
  WD_TRY(check_ptr(UR, "UR"));
  WD_TRY(check_ptr(workspace, "workspace"));
  WD_TRY(check_nrhs(ctx, nrhs));
  WD_TRY(check_prec(prec));
  if (dagger != 0 && dagger != 1) return fail(WDIRAC_EINVAL, "dagger must be 0 or 1");
  if (in == out) return fail(WDIRAC_EINVAL, "in and out must not alias");
  return dhat(ctx, out, in, UR, m0, dagger, nrhs, prec, workspace, nullptr, S(stream));
}

}  // extern "C"

// Scratch of wdirac_apply_dhat_noalloc: the odd half field between the two
// hops, in a device array of fixed size that every call on a GPU shares (each
// GPU holds its own copy from the first call until the process ends).  In
// host code `scratch` names a host-side stand-in; kernels receive the device
// address that hipGetSymbolAddress returns for the current device.
static constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int scratch_address(void **out) {
  int dev = -1;
  WD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(WDIRAC_EHIP, "device index out of range for the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    WD_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(WDIRAC_EHIP, "hipGetSymbolAddress returned a null scratch address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return WDIRAC_OK;
}
}  // namespace

extern "C" {

size_t wdirac_noalloc_scratch_bytes(void) { return kNoallocScratchBytes; }

int wdirac_apply_dhat_noalloc(const wdirac_ctx *ctx, void *out, const void *in, const void *UR, double m0,
                              int dagger, int nrhs, int prec, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(out, "out"));
  WD_TRY(check_ptr(in, "in"));
  WD_TRY(check_ptr(UR, "UR"));
  WD_TRY(check_nrhs(ctx, nrhs));
  WD_TRY(check_prec(prec));
  if (dagger != 0 && dagger != 1) return fail(WDIRAC_EINVAL, "dagger must be 0 or 1");
  if (in == out) return fail(WDIRAC_EINVAL, "in and out must not alias");
  const size_t need = half_bytes(ctx, nrhs, prec);
  if (need > kNoallocScratchBytes)
    return fail(WDIRAC_EINVAL, "apply_dhat_noalloc: the odd half field needs " + std::to_string(need) +
                                   " bytes, more than the " + std::to_string(kNoallocScratchBytes) +
                                   "-byte scratch; use wdirac_apply_dhat with a workspace");
  void *tmp = nullptr;
  WD_TRY(scratch_address(&tmp));
  // the first hop writes every element of tmp that the second reads: nothing
  // left by an earlier call needs clearing
  return dhat(ctx, out, in, UR, m0, dagger, nrhs, prec, tmp, nullptr, S(stream));
}

int wdirac_eo_source(const wdirac_ctx *ctx, void *b_e, const void *eta_e, const void *eta_o, const void *UR,
                     double m0, int nrhs, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(b_e, "b_e"));
  WD_TRY(check_ptr(eta_e, "eta_e"));
  WD_TRY(check_ptr(eta_o, "eta_o"));
  WD_TRY(check_ptr(UR, "UR"));
  WD_TRY(check_nrhs(ctx, nrhs));
  if (b_e == eta_o) return fail(WDIRAC_EINVAL, "b_e must not alias eta_o");
  return hop(ctx, b_e, eta_o, UR, 0, 0, nrhs, 4.0 + m0, eta_e, -1.0, WDIRAC_F64, nullptr, S(stream));
}

int wdirac_eo_reconstruct(const wdirac_ctx *ctx, void *psi_o, const void *psi_e, const void *eta_o, const void *UR,
                          double m0, int nrhs, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(psi_o, "psi_o"));
  WD_TRY(check_ptr(psi_e, "psi_e"));
  WD_TRY(check_ptr(eta_o, "eta_o"));
  WD_TRY(check_ptr(UR, "UR"));
  WD_TRY(check_nrhs(ctx, nrhs));
  if (4.0 + m0 == 0.0) return fail(WDIRAC_EINVAL, "4 + m0 = 0 has no inverse");
  if (psi_o == psi_e) return fail(WDIRAC_EINVAL, "psi_o must not alias psi_e");
  const double f = 1.0 / (4.0 + m0);
  return hop(ctx, psi_o, psi_e, UR, 1, 0, nrhs, f, eta_o, -f, WDIRAC_F64, nullptr, S(stream));
}

int wdirac_norm2(const wdirac_ctx *ctx, double *out, const void *v, int nrhs, int prec, void *workspace,
                 void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(out, "out"));
  WD_TRY(check_ptr(v, "v"));
  WD_TRY(check_ptr(workspace, "workspace"));
  WD_TRY(check_nrhs(ctx, nrhs));
  WD_TRY(check_prec(prec));
  Carver cv{static_cast<char *>(workspace)};
  double *part = static_cast<double *>(cv.take(partial_doubles(ctx, nrhs) * sizeof(double)));
  double *dout = static_cast<double *>(cv.take(2 * wd::MAXSYS * sizeof(double)));
  const wd::FieldShape f = shape(ctx, nrhs);
  const int nb = wd::blas_nblocks(f);
  WD_HIP(wd::launch_norm2_partial(part, v, f, prec, S(stream)));
  WD_HIP(wd::launch_finalize_sum(dout, part, nb, wd::uniform_counts(nb), f.nsys, f.nsys, S(stream)));
  WD_HIP(hipMemcpyAsync(out, dout, f.nsys * sizeof(double), hipMemcpyDeviceToHost, S(stream)));
  WD_HIP(hipStreamSynchronize(S(stream)));
  return WDIRAC_OK;
}

int wdirac_dot(const wdirac_ctx *ctx, double *out, const void *a, const void *b, int nrhs, int prec, void *workspace,
               void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(out, "out"));
  WD_TRY(check_ptr(a, "a"));
  WD_TRY(check_ptr(b, "b"));
  WD_TRY(check_ptr(workspace, "workspace"));
  WD_TRY(check_nrhs(ctx, nrhs));
  WD_TRY(check_prec(prec));
  Carver cv{static_cast<char *>(workspace)};
  double *part = static_cast<double *>(cv.take(partial_doubles(ctx, nrhs) * sizeof(double)));
  double *dout = static_cast<double *>(cv.take(2 * wd::MAXSYS * sizeof(double)));
  const wd::FieldShape f = shape(ctx, nrhs);
  const int nb = wd::blas_nblocks(f), ns = f.nsys;
  WD_HIP(wd::launch_dot_partial(part, a, b, f, prec, S(stream)));
  WD_HIP(wd::launch_finalize_sum(dout, part, nb, wd::uniform_counts(nb), 2 * ns, ns, S(stream)));
  std::vector<double> tmp(2 * ns);
  WD_HIP(hipMemcpyAsync(tmp.data(), dout, 2 * ns * sizeof(double), hipMemcpyDeviceToHost, S(stream)));
  WD_HIP(hipStreamSynchronize(S(stream)));
  for (int k = 0; k < ns; ++k) {
    out[2 * k] = tmp[k];
    out[2 * k + 1] = tmp[ns + k];
  }
  return WDIRAC_OK;
}

// ------------------------------------------------------------------- CG
// Per right-hand side, the Hestenes-Stiefel recurrence on A = D-hat^+ D-hat:
//   q = A p (u = D-hat p gives <p, A p> = ||u||^2, then q = D-hat^+ u),
//   alpha = rho / <p,Ap>;  x += alpha p;  r -= alpha q;  rho' = ||r||^2;
//   beta = rho'/rho;  p = r + beta p.
// All scalars stay on the device; kernels of right-hand sides that are done
// return at once, so the host only reads the scalars every few iterations.
// When the recursive residual reaches the target, r is recomputed as b - A x
// in FP64 (the "true" residual); if it is above target the recurrence resumes
// from it with p kept (residual replacement).  Mixed mode runs the
// recurrence in FP32 (hops, vectors; sums in FP64) on the correction
// equation and replaces the residual in FP64 whenever ||r|| drops below
// delta times its largest value since the previous replacement (reliable
// updates), accumulating the FP32 correction into the FP64 solution.
static int cg_impl(const wdirac_ctx *ctx, void *x, const void *b, const void *UR64, const void *UR32,
                   const void *clov64, const void *clov32, double m0, double tol, int maxit, int nrhs, int mode,
                   void *workspace, wdirac_cg_stats *stats, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(x, "x"));
  WD_TRY(check_ptr(b, "b"));
  WD_TRY(check_ptr(UR64, "UR64"));
  WD_TRY(check_ptr(workspace, "workspace"));
  WD_TRY(check_ptr(stats, "stats"));
  WD_TRY(check_nrhs(ctx, nrhs));
  if (mode != WDIRAC_CG_F64 && mode != WDIRAC_CG_MIXED) return fail(WDIRAC_EINVAL, "unknown CG mode");
  if (mode == WDIRAC_CG_MIXED) WD_TRY(check_ptr(UR32, "UR32"));
  if (!(tol > 0.0) || maxit < 0) return fail(WDIRAC_EINVAL, "tol must be > 0 and maxit >= 0");
  if (x == b) return fail(WDIRAC_EINVAL, "x and b must not alias");
  hipStream_t st = S(stream);
  // the solve starts once the caller's queued work is done: the reported
  // time is that of the solve alone
  WD_HIP(hipStreamSynchronize(st));
  const auto t0 = std::chrono::steady_clock::now();
  if (ctx->cg_graph) {
    // the iterations between host checks are captured once and replayed as
    // a graph; capture needs a stream of the library's own (the caller's may
    // be the null stream), ordered after the caller's work (drained above)
    if (!ctx->own && hipStreamCreateWithFlags(&ctx->own, hipStreamNonBlocking) != hipSuccess) ctx->own = nullptr;
    if (ctx->own) st = ctx->own;
  }
  const bool mixed = mode == WDIRAC_CG_MIXED;
  CgWork w = carve_cg(ctx, nrhs, mode, workspace);
  const wd::FieldShape f = shape(ctx, nrhs);
  const int nbb = wd::blas_nblocks(f), ns = f.nsys;
  std::vector<wd::CgScalars> hs(ns);
  std::vector<int> rel(ns, 0);
  int hop_count = 0, updates = 0;

  // b2, stop2
  WD_HIP(wd::launch_norm2_partial(w.P2, b, f, WDIRAC_F64, st));
  WD_HIP(wd::launch_cg_restart(w.sc, w.P2, nbb, ns, tol, 1, 1, st));
  // r = b - A x (FP64)
  auto true_residual = [&]() -> int {
    WD_TRY(dhat(ctx, w.u, x, UR64, m0, 0, nrhs, WDIRAC_F64, w.t, nullptr, st, nullptr, nullptr, clov64));
    WD_TRY(dhat(ctx, w.q, w.u, UR64, m0, 1, nrhs, WDIRAC_F64, w.v, nullptr, st, nullptr, nullptr, clov64));
    WD_HIP(wd::launch_residual(w.r, b, w.q, w.P2, f, st));
    hop_count += 4;
    return WDIRAC_OK;
  };
  WD_TRY(true_residual());
  WD_HIP(wd::launch_cg_restart(w.sc, w.P2, nbb, ns, tol, 0, 1, st));
  void *r = w.r, *p = w.p, *q = w.q, *t = w.t, *u = w.u, *v = w.v, *xi = x;
  const void *UR = UR64, *clov = clov64;
  int prec = WDIRAC_F64;
  if (mixed) {
    WD_HIP(wd::launch_convert(w.r32, WDIRAC_F32, w.r, WDIRAC_F64, f, st));
    WD_HIP(wd::launch_lincomb(w.x32, 0.0, w.r32, 0.0, nullptr, f, WDIRAC_F32, st));
    r = w.r32; p = w.p32; q = w.q32; t = w.t32; u = w.u32; v = w.v32; xi = w.x32;
    UR = UR32;
    clov = clov32;
    prec = WDIRAC_F32;
  }
  WD_HIP(wd::launch_lincomb(p, 1.0, r, 0.0, nullptr, f, prec, st));
  const double delta = mixed ? ctx->mixed_delta : 0.0;
  const int check = ctx->cg_check_every;
  int rc = WDIRAC_OK;
  int launched = 0;   // iterations launched since start
  bool use_graph = ctx->cg_graph && st == ctx->own;
  hipGraphExec_t exec = nullptr;
  for (;;) {
    WD_HIP(hipMemcpyAsync(hs.data(), w.sc, ns * sizeof(wd::CgScalars), hipMemcpyDeviceToHost, st));
    WD_HIP(hipStreamSynchronize(st));
    // a residual replacement runs once every system that is still iterating
    // has asked for one (mixed mode) or has stopped (converged recursion,
    // breakdown)
    bool any_active = false, any_update = false, all_ready = true;
    for (int k = 0; k < ns; ++k) {
      any_active |= hs[k].active != 0;
      any_update |= hs[k].need_update != 0;
      all_ready &= hs[k].active == 0 || hs[k].need_update != 0;
    }
    int max_iters = 0;
    for (int k = 0; k < ns; ++k) max_iters = std::max(max_iters, hs[k].iters);
    if (any_update && all_ready) {
      // residual replacement in FP64 (verifies convergence of the recursion)
      if (mixed) WD_HIP(wd::launch_accum_x(x, w.x32, f, st));
      WD_TRY(true_residual());
      WD_HIP(wd::launch_cg_restart(w.sc, w.P2, nbb, ns, tol, 0, 0, st));
      if (mixed) WD_HIP(wd::launch_convert(w.r32, WDIRAC_F32, w.r, WDIRAC_F64, f, st));
      ++updates;
      for (int k = 0; k < ns; ++k)
        if (hs[k].need_update) ++rel[k];
      continue;
    }
    if (!any_active) break;
    if (max_iters >= maxit) {
      rc = WDIRAC_ENOCONV;
      break;
    }
    const int nit = std::min(check, std::max(1, maxit - max_iters));
    auto launch_iters = [&](int n) -> int {
      for (int it = 0; it < n; ++it) {
        wd::Counts cnt{};
        int prow = 0;
        WD_TRY(dhat(ctx, u, p, UR, m0, 0, nrhs, prec, t, w.P1, st, &cnt, &prow, clov));
        WD_HIP(wd::launch_cg_alpha(w.sc, w.P1, prow, cnt, ns, st));
        WD_TRY(dhat(ctx, q, u, UR, m0, 1, nrhs, prec, v, nullptr, st, nullptr, nullptr, clov));
        WD_HIP(wd::launch_cg_update_xr(xi, prec, r, p, q, w.sc, w.P2, f, prec, st));
        WD_HIP(wd::launch_cg_beta(w.sc, w.P2, nbb, ns, delta, st));
        WD_HIP(wd::launch_cg_update_p(p, r, w.sc, f, prec, st));
      }
      return WDIRAC_OK;
    };
    if (use_graph && nit == check && !exec) {
      hipGraph_t graph = nullptr;
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        const int crc = launch_iters(nit);
        const hipError_t ce = hipStreamEndCapture(st, &graph);
        if (crc != WDIRAC_OK || ce != hipSuccess || !graph ||
            hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
          exec = nullptr;
        if (graph) (void)hipGraphDestroy(graph);
      }
      if (!exec) {
        use_graph = false;   // capture unavailable: launch directly from now on
        g_err.clear();
      }
    }
    if (use_graph && nit == check && exec) WD_HIP(hipGraphLaunch(exec, st));
    else WD_TRY(launch_iters(nit));
    hop_count += 4 * nit;
    launched += nit;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (mixed) WD_HIP(wd::launch_accum_x(x, w.x32, f, st));
  // final FP64 true residual of the returned x
  WD_TRY(true_residual());
  WD_HIP(wd::launch_finalize_sum(w.P1, w.P2, nbb, wd::uniform_counts(nbb), ns, ns, st));
  std::vector<double> res2(ns);
  WD_HIP(hipMemcpyAsync(res2.data(), w.P1, ns * sizeof(double), hipMemcpyDeviceToHost, st));
  WD_HIP(hipMemcpyAsync(hs.data(), w.sc, ns * sizeof(wd::CgScalars), hipMemcpyDeviceToHost, st));
  WD_HIP(hipStreamSynchronize(st));
  // b = 0: the solution is x = 0 whatever the initial guess
  for (int k = 0; k < ns; ++k)
    if (!(hs[k].b2 > 0.0)) {
      const size_t bytes = (size_t)f.ncomp * f.stride[k] * 16;
      WD_HIP(hipMemsetAsync(static_cast<char *>(x) + (size_t)f.off[k] * 16, 0, bytes, st));
      res2[k] = 0.0;
    }
  WD_HIP(hipStreamSynchronize(st));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = WDIRAC_OK;
  for (int k = 0; k < ns; ++k) {
    wdirac_cg_stats &s = stats[k];
    s.iters = hs[k].iters;
    s.reliable_updates = rel[k];
    s.hops = hop_count;
    s.true_rel_resid = hs[k].b2 > 0.0 ? std::sqrt(res2[k] / hs[k].b2) : 0.0;
    s.seconds = secs;
    int stk = hs[k].status;
    if (stk == WDIRAC_OK && hs[k].b2 > 0.0 && !(s.true_rel_resid <= tol)) stk = WDIRAC_ENOCONV;
    s.status = stk;
    if (stk == WDIRAC_EBREAKDOWN) worst = WDIRAC_EBREAKDOWN;
    else if (stk == WDIRAC_ENOCONV && worst == WDIRAC_OK) worst = WDIRAC_ENOCONV;
  }
  (void)launched;
  (void)updates;
  if (rc == WDIRAC_ENOCONV && worst == WDIRAC_OK) worst = WDIRAC_ENOCONV;
  if (worst == WDIRAC_ENOCONV) fail(worst, "CG did not reach the tolerance within maxit");
  if (worst == WDIRAC_EBREAKDOWN) fail(worst, "CG breakdown (non-finite value or <p,Ap> <= 0)");
  return worst;
}

int wdirac_cg_eo(const wdirac_ctx *ctx, void *x, const void *b, const void *UR64, const void *UR32, double m0,
                 double tol, int maxit, int nrhs, int mode, void *workspace, wdirac_cg_stats *stats, void *stream) {
  return cg_impl(ctx, x, b, UR64, UR32, nullptr, nullptr, m0, tol, maxit, nrhs, mode, workspace, stats, stream);
}

// ------------------------------------------------------------------ clover
int wdirac_clover_field(const wdirac_ctx *ctx, void *clov, const void *U, double m0, double csw, int exponential,
                        int prec, void *workspace, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(clov, "clov"));
  WD_TRY(check_ptr(U, "U"));
  WD_TRY(check_ptr(workspace, "workspace"));
  WD_TRY(check_prec(prec));
  if (!wd::clover_supported(ctx->d)) return fail(WDIRAC_EUNSUPPORTED, "clover term available for d_R in {2,3,4,6}");
  if (!std::isfinite(m0) || !std::isfinite(csw) || 4.0 + m0 == 0.0)
    return fail(WDIRAC_EINVAL, "m0 and csw must be finite and 4 + m0 != 0");
  if (exponential != 0 && exponential != 1) return fail(WDIRAC_EINVAL, "exponential must be 0 or 1");
  const size_t el = prec == WDIRAC_F64 ? 8 : 4;
  for (int l = 0; l < ctx->nlat; ++l) {
    const char *Ul = static_cast<const char *>(U) + (size_t)ctx->vpre[l] * 4 * ctx->N * ctx->N * 16;
    char *cl = static_cast<char *>(clov) + (size_t)4 * ctx->d * (2 * ctx->d + 1) * ctx->spre[l] * 2 * el;
    int mx = 0;
    for (int k = 0; k < ctx->nlat; ++k) mx = std::max(mx, ctx->g[k].Vh);
    double *Fw = static_cast<double *>(workspace);
    double *Us = reinterpret_cast<double *>(static_cast<char *>(workspace) +
                                            align256((size_t)6 * ctx->d * ctx->d * 2 * mx * 16));
    WD_HIP(wd::launch_clover_field(cl, Ul, Fw, Us, ctx->g[l], ctx->N, ctx->rep, ctx->d, m0, csw, exponential, prec,
                                   S(stream)));
  }
  return WDIRAC_OK;
}

int wdirac_apply_clover(const wdirac_ctx *ctx, void *out, const void *in, const void *clov, int parity, int nrhs,
                        int prec, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(out, "out"));
  WD_TRY(check_ptr(in, "in"));
  WD_TRY(check_ptr(clov, "clov"));
  WD_TRY(check_parity(parity));
  WD_TRY(check_nrhs(ctx, nrhs));
  WD_TRY(check_prec(prec));
  if (!wd::clover_supported(ctx->d)) return fail(WDIRAC_EUNSUPPORTED, "clover term available for d_R in {2,3,4,6}");
  return clover_apply(ctx, out, in, clov, parity, nrhs, prec, S(stream));
}

int wdirac_apply_dhat_clover(const wdirac_ctx *ctx, void *out, const void *in, const void *UR, const void *clov,
                             int dagger, int nrhs, int prec, void *workspace, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(out, "out"));
  WD_TRY(check_ptr(in, "in"));
  WD_TRY(check_ptr(UR, "UR"));
  WD_TRY(check_ptr(clov, "clov"));
  WD_TRY(check_ptr(workspace, "workspace"));
  WD_TRY(check_nrhs(ctx, nrhs));
  WD_TRY(check_prec(prec));
  if (dagger != 0 && dagger != 1) return fail(WDIRAC_EINVAL, "dagger must be 0 or 1");
  if (!wd::clover_supported(ctx->d)) return fail(WDIRAC_EUNSUPPORTED, "clover term available for d_R in {2,3,4,6}");
  if (out == in) return fail(WDIRAC_EINVAL, "out must not alias in");
  return dhat(ctx, out, in, UR, 0.0, dagger, nrhs, prec, workspace, nullptr, S(stream), nullptr, nullptr, clov);
}

int wdirac_cg_eo_clover(const wdirac_ctx *ctx, void *x, const void *b, const void *UR64, const void *UR32,
                        const void *clov64, const void *clov32, double tol, int maxit, int nrhs, int mode,
                        void *workspace, wdirac_cg_stats *stats, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(clov64, "clov64"));
  if (mode == WDIRAC_CG_MIXED) WD_TRY(check_ptr(clov32, "clov32"));
  if (!wd::clover_supported(ctx->d)) return fail(WDIRAC_EUNSUPPORTED, "clover term available for d_R in {2,3,4,6}");
  return cg_impl(ctx, x, b, UR64, UR32, clov64, clov32, 0.0, tol, maxit, nrhs, mode, workspace, stats, stream);
}

// ------------------------------------------------------------ multi-shift CG
int wdirac_cg_mshift_eo(const wdirac_ctx *ctx, void *x, const void *b, const void *UR64, double m0,
                        const double *shifts, int nshift, double tol, int maxit, void *workspace,
                        wdirac_cg_stats *stats, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(x, "x"));
  WD_TRY(check_ptr(b, "b"));
  WD_TRY(check_ptr(UR64, "UR64"));
  WD_TRY(check_ptr(shifts, "shifts"));
  WD_TRY(check_ptr(workspace, "workspace"));
  WD_TRY(check_ptr(stats, "stats"));
  if (ctx->nlat != 1) return fail(WDIRAC_EUNSUPPORTED, "multi-shift CG runs on a single lattice");
  if (nshift < 1 || nshift > wd::MAXSHIFT) return fail(WDIRAC_EINVAL, "nshift must be in [1, 32]");
  if (!(tol > 0.0) || maxit < 0) return fail(WDIRAC_EINVAL, "tol must be > 0 and maxit >= 0");
  int base = 0;
  for (int k = 0; k < nshift; ++k) {
    if (!(shifts[k] >= 0.0) || !std::isfinite(shifts[k])) return fail(WDIRAC_EINVAL, "shifts must be finite and >= 0");
    if (shifts[k] < shifts[base]) base = k;
  }
  const size_t hb = half_bytes(ctx, 1, WDIRAC_F64);
  {
    const char *xs = static_cast<const char *>(x), *bs = static_cast<const char *>(b);
    if (bs + hb > xs && bs < xs + (size_t)nshift * hb) return fail(WDIRAC_EINVAL, "x and b must not overlap");
  }
  const hipStream_t st = S(stream);
  WD_HIP(hipStreamSynchronize(st));   // time the solve alone
  const auto t0 = std::chrono::steady_clock::now();
  MsWork w = carve_ms(ctx, nshift, workspace);
  const wd::FieldShape f = shape(ctx, 1);
  const int nbb = wd::blas_nblocks(f);
  const double sigma0 = shifts[base];
  const long long fstride = (long long)(hb / 16);
  wd::ShiftList dl{};
  for (int k = 0; k < nshift; ++k) dl.v[k] = shifts[k] - sigma0;
  auto field = [&](void *base_ptr, int k) { return static_cast<void *>(static_cast<char *>(base_ptr) + (size_t)k * hb); };
  // x_k = 0 (padding included), p_k = b, r = b
  WD_HIP(hipMemsetAsync(x, 0, (size_t)nshift * hb, st));
  WD_HIP(wd::launch_lincomb(w.r, 1.0, b, 0.0, nullptr, f, WDIRAC_F64, st));
  for (int k = 0; k < nshift; ++k) WD_HIP(wd::launch_lincomb(field(w.p, k), 1.0, b, 0.0, nullptr, f, WDIRAC_F64, st));
  WD_HIP(wd::launch_norm2_partial(w.P2, b, f, WDIRAC_F64, st));
  // the recursion stops at half the tolerance, leaving room for the drift of
  // the recursive residuals from the true ones checked below
  WD_HIP(wd::launch_ms_init(w.sc, w.P2, nbb, dl, nshift, base, sigma0, 0.5 * tol, st));
  int hop_count = 0, rc = WDIRAC_OK;
  wd::MsScalars hs{};
  void *pb = field(w.p, base);
  for (;;) {
    WD_HIP(hipMemcpyAsync(&hs, w.sc, sizeof(hs), hipMemcpyDeviceToHost, st));
    WD_HIP(hipStreamSynchronize(st));
    if (!hs.active) break;
    if (hs.iters >= maxit) {
      rc = WDIRAC_ENOCONV;
      break;
    }
    const int nit = std::min(ctx->cg_check_every, std::max(1, maxit - hs.iters));
    for (int it = 0; it < nit; ++it) {
      wd::Counts cnt{};
      int prow = 0;
      WD_TRY(dhat(ctx, w.u, pb, UR64, m0, 0, 1, WDIRAC_F64, w.t, w.P1, st, &cnt, &prow));
      if (sigma0 != 0.0) WD_HIP(wd::launch_norm2_partial(w.P3, pb, f, WDIRAC_F64, st));
      WD_TRY(dhat(ctx, w.q, w.u, UR64, m0, 1, 1, WDIRAC_F64, w.v, nullptr, st));
      if (sigma0 != 0.0) WD_HIP(wd::launch_lincomb(w.q, 1.0, w.q, sigma0, pb, f, WDIRAC_F64, st));
      WD_HIP(wd::launch_ms_alpha(w.sc, w.P1, prow, cnt, sigma0 != 0.0 ? w.P3 : nullptr, nbb, st));
      WD_HIP(wd::launch_ms_update_r(w.r, w.q, w.sc, w.P2, f, st));
      WD_HIP(wd::launch_ms_beta(w.sc, w.P2, nbb, st));
      WD_HIP(wd::launch_ms_update_xp(x, w.p, w.r, w.sc, fstride, f, nshift, st));
      hop_count += 4;
    }
  }
  // true residuals ||b - (A + sigma_k) x_k||
  std::vector<double> res2(nshift);
  for (int k = 0; k < nshift; ++k) {
    WD_TRY(dhat(ctx, w.u, field(x, k), UR64, m0, 0, 1, WDIRAC_F64, w.t, nullptr, st));
    WD_TRY(dhat(ctx, w.q, w.u, UR64, m0, 1, 1, WDIRAC_F64, w.v, nullptr, st));
    WD_HIP(wd::launch_lincomb(w.q, 1.0, w.q, shifts[k], field(x, k), f, WDIRAC_F64, st));
    WD_HIP(wd::launch_residual(w.r, b, w.q, w.P2, f, st));
    WD_HIP(wd::launch_finalize_sum(w.P1, w.P2, nbb, wd::uniform_counts(nbb), 1, 1, st));
    WD_HIP(hipMemcpyAsync(&res2[k], w.P1, sizeof(double), hipMemcpyDeviceToHost, st));
    hop_count += 4;
  }
  WD_HIP(hipMemcpyAsync(&hs, w.sc, sizeof(hs), hipMemcpyDeviceToHost, st));
  WD_HIP(hipStreamSynchronize(st));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = WDIRAC_OK;
  for (int k = 0; k < nshift; ++k) {
    wdirac_cg_stats &sk = stats[k];
    sk.iters = hs.siters[k];
    sk.reliable_updates = 0;
    sk.hops = hop_count;
    sk.true_rel_resid = hs.b2 > 0.0 ? std::sqrt(res2[k] / hs.b2) : 0.0;
    sk.seconds = secs;
    int stk = hs.status;
    if (stk == WDIRAC_OK && hs.b2 > 0.0 && (hs.sact[k] || !(sk.true_rel_resid <= tol))) stk = WDIRAC_ENOCONV;
    sk.status = stk;
    if (stk == WDIRAC_EBREAKDOWN) worst = WDIRAC_EBREAKDOWN;
    else if (stk == WDIRAC_ENOCONV && worst == WDIRAC_OK) worst = WDIRAC_ENOCONV;
  }
  if (rc == WDIRAC_ENOCONV && worst == WDIRAC_OK) worst = WDIRAC_ENOCONV;
  if (worst == WDIRAC_ENOCONV) fail(worst, "multi-shift CG: some shift did not reach the tolerance");
  if (worst == WDIRAC_EBREAKDOWN) fail(worst, "multi-shift CG breakdown (non-finite value or <p,Ap> <= 0)");
  return worst;
}

int wdirac_axpby(const wdirac_ctx *ctx, void *out, double a, const void *x, double b, const void *y, int nrhs,
                 int prec, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(out, "out"));
  WD_TRY(check_ptr(x, "x"));
  WD_TRY(check_nrhs(ctx, nrhs));
  WD_TRY(check_prec(prec));
  WD_HIP(wd::launch_lincomb(out, a, x, b, y, shape(ctx, nrhs), prec, S(stream)));
  return WDIRAC_OK;
}

// ------------------------------------------------------------- HMC pieces
static size_t links_offset(const wdirac_ctx *c, int l) { return (size_t)c->vpre[l] * 4 * c->N * c->N * 16; }

int wdirac_gauge_force(const wdirac_ctx *ctx, void *F, const void *U, double beta, double scale, int accumulate,
                       void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(F, "F"));
  WD_TRY(check_ptr(U, "U"));
  if (accumulate != 0 && accumulate != 1) return fail(WDIRAC_EINVAL, "accumulate must be 0 or 1");
  if (F == U) return fail(WDIRAC_EINVAL, "F must not alias U");
  for (int l = 0; l < ctx->nlat; ++l)
    WD_HIP(wd::launch_gauge_force(static_cast<const char *>(U) + links_offset(ctx, l),
                                  static_cast<char *>(F) + links_offset(ctx, l), ctx->g[l], ctx->N, beta, scale,
                                  accumulate, S(stream)));
  return WDIRAC_OK;
}

// Sum of the block partials (FP64, compensated) to the host.
static int reduce_to_host(double *out, const double *partial, int nblk, double *dtmp, hipStream_t st) {
  WD_HIP(wd::launch_finalize_sum(dtmp, partial, nblk, wd::uniform_counts(nblk), 1, 1, st));
  WD_HIP(hipMemcpyAsync(out, dtmp, sizeof(double), hipMemcpyDeviceToHost, st));
  WD_HIP(hipStreamSynchronize(st));
  return WDIRAC_OK;
}

int wdirac_gauge_action(const wdirac_ctx *ctx, double *S_out, const void *U, double beta, void *workspace,
                        void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(S_out, "S"));
  WD_TRY(check_ptr(U, "U"));
  WD_TRY(check_ptr(workspace, "workspace"));
  Carver cv{static_cast<char *>(workspace)};
  int mx = 0;
  for (int l = 0; l < ctx->nlat; ++l) mx = std::max(mx, wd::kinetic_blocks(ctx->g[l]));
  double *part = static_cast<double *>(cv.take((size_t)mx * sizeof(double)));
  double *dtmp = static_cast<double *>(cv.take(sizeof(double)));
  for (int l = 0; l < ctx->nlat; ++l) {
    const int nb = wd::plaquette_blocks(ctx->g[l]);
    WD_HIP(wd::launch_plaquette_partial(static_cast<const char *>(U) + links_offset(ctx, l), part, ctx->g[l],
                                        ctx->N, S(stream)));
    double plaq = 0.0;
    WD_TRY(reduce_to_host(&plaq, part, nb, dtmp, S(stream)));
    S_out[l] = beta * (6.0 * 2.0 * ctx->g[l].Vh - plaq);
  }
  return WDIRAC_OK;
}

int wdirac_link_update(const wdirac_ctx *ctx, void *U, const void *pi, double eps, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(U, "U"));
  WD_TRY(check_ptr(pi, "pi"));
  if (U == pi) return fail(WDIRAC_EINVAL, "pi must not alias U");
  if (!std::isfinite(eps)) return fail(WDIRAC_EINVAL, "eps must be finite");
  for (int l = 0; l < ctx->nlat; ++l)
    WD_HIP(wd::launch_link_update(static_cast<char *>(U) + links_offset(ctx, l),
                                  static_cast<const char *>(pi) + links_offset(ctx, l), ctx->g[l], ctx->N, eps,
                                  S(stream)));
  return WDIRAC_OK;
}

int wdirac_kinetic(const wdirac_ctx *ctx, double *K, const void *pi, void *workspace, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(K, "K"));
  WD_TRY(check_ptr(pi, "pi"));
  WD_TRY(check_ptr(workspace, "workspace"));
  Carver cv{static_cast<char *>(workspace)};
  int mx = 0;
  for (int l = 0; l < ctx->nlat; ++l) mx = std::max(mx, wd::kinetic_blocks(ctx->g[l]));
  double *part = static_cast<double *>(cv.take((size_t)mx * sizeof(double)));
  double *dtmp = static_cast<double *>(cv.take(sizeof(double)));
  for (int l = 0; l < ctx->nlat; ++l) {
    WD_HIP(wd::launch_kinetic_partial(static_cast<const char *>(pi) + links_offset(ctx, l), part, ctx->g[l], ctx->N,
                                      S(stream)));
    WD_TRY(reduce_to_host(&K[l], part, wd::kinetic_blocks(ctx->g[l]), dtmp, S(stream)));
  }
  return WDIRAC_OK;
}

int wdirac_algebra_from_components(const wdirac_ctx *ctx, void *pi, const double *w, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(pi, "pi"));
  WD_TRY(check_ptr(w, "w"));
  const int na = ctx->N * ctx->N - 1;
  for (int l = 0; l < ctx->nlat; ++l)
    WD_HIP(wd::launch_algebra(static_cast<char *>(pi) + links_offset(ctx, l), w + (size_t)ctx->vpre[l] * 4 * na,
                              ctx->g[l], ctx->N, S(stream)));
  return WDIRAC_OK;
}

// ---------------------------------------------- twisted mass, Hasenbusch
int wdirac_gamma5(const wdirac_ctx *ctx, void *out, const void *in, int nrhs, int prec, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(out, "out"));
  WD_TRY(check_ptr(in, "in"));
  WD_TRY(check_nrhs(ctx, nrhs));
  WD_TRY(check_prec(prec));
  WD_HIP(wd::launch_gamma5_axpy(out, in, 0.0, nullptr, shape(ctx, nrhs), prec, S(stream)));
  return WDIRAC_OK;
}

int wdirac_apply_W(const wdirac_ctx *ctx, void *out, const void *in, const void *UR, double m0, double mu, int sign,
                   int nrhs, int prec, void *workspace, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(out, "out"));
  WD_TRY(check_ptr(in, "in"));
  WD_TRY(check_ptr(UR, "UR"));
  WD_TRY(check_ptr(workspace, "workspace"));
  WD_TRY(check_nrhs(ctx, nrhs));
  WD_TRY(check_prec(prec));
  if (sign != 1 && sign != -1) return fail(WDIRAC_EINVAL, "sign must be +1 or -1");
  if (!std::isfinite(mu)) return fail(WDIRAC_EINVAL, "mu must be finite");
  if (out == in) return fail(WDIRAC_EINVAL, "out must not alias in");
  const hipStream_t st = S(stream);
  WD_TRY(dhat(ctx, out, in, UR, m0, 0, nrhs, prec, workspace, nullptr, st));
  WD_HIP(wd::launch_gamma5_axpy(out, out, sign * mu, in, shape(ctx, nrhs), prec, st));
  return WDIRAC_OK;
}

int wdirac_force_bilinear_eo(const wdirac_ctx *ctx, void *P, const void *X_e, const void *X_o, const void *Y_e,
                             const void *Y_o, const void *UR64, const void *U, double scale, int accumulate,
                             void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(P, "out"));
  WD_TRY(check_ptr(X_e, "X_e"));
  WD_TRY(check_ptr(X_o, "X_o"));
  WD_TRY(check_ptr(Y_e, "Y_e"));
  WD_TRY(check_ptr(Y_o, "Y_o"));
  WD_TRY(check_ptr(UR64, "UR64"));
  if (accumulate != 0 && accumulate != 1) return fail(WDIRAC_EINVAL, "accumulate must be 0 or 1");
  const hipStream_t st = S(stream);
  const size_t el = ctx->real ? 8 : 16;
  for (int l = 0; l < ctx->nlat; ++l) {
    const size_t so = (size_t)4 * ctx->d * ctx->spre[l] * 16;
    const size_t po = (size_t)ctx->vpre[l] * 4 * ctx->N * ctx->N * 16;
    auto at = [so](const void *p) { return static_cast<const void *>(static_cast<const char *>(p) + so); };
    WD_HIP(wd::launch_force_links(static_cast<char *>(P) + po, at(X_e), at(X_o), at(Y_e), at(Y_o),
                                  static_cast<const char *>(UR64) + (size_t)8 * ctx->d * ctx->d * ctx->spre[l] * el,
                                  U ? static_cast<const char *>(U) + po : nullptr, ctx->g[l], ctx->N, ctx->rep, scale,
                                  accumulate, st));
  }
  WD_HIP(hipStreamSynchronize(st));
  return WDIRAC_OK;
}

int wdirac_force_eo(const wdirac_ctx *ctx, void *P, const void *x_e, const void *UR64, const void *U, double m0,
                    double scale, int accumulate, void *workspace, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(P, "out"));
  WD_TRY(check_ptr(x_e, "x_e"));
  WD_TRY(check_ptr(UR64, "UR64"));
  WD_TRY(check_ptr(workspace, "workspace"));
  const hipStream_t st = S(stream);
  Carver cv{static_cast<char *>(workspace)};
  const size_t h = half_bytes(ctx, 1, WDIRAC_F64);
  void *z_o = cv.take(h), *y_e = cv.take(h), *w_o = cv.take(h);
  // z_o = D_oe x;  y_e = (4+m)^2 x - D_eo z_o = D-hat x;  w_o = D_eo^+ y_e
  WD_TRY(hop(ctx, z_o, x_e, UR64, 1, 0, 1, 0.0, nullptr, 1.0, WDIRAC_F64, nullptr, st));
  WD_TRY(hop(ctx, y_e, z_o, UR64, 0, 0, 1, (4.0 + m0) * (4.0 + m0), x_e, -1.0, WDIRAC_F64, nullptr, st));
  WD_TRY(hop(ctx, w_o, y_e, UR64, 1, 1, 1, 0.0, nullptr, 1.0, WDIRAC_F64, nullptr, st));
  const size_t el = ctx->real ? 8 : 16;
  for (int l = 0; l < ctx->nlat; ++l) {
    const size_t so = (size_t)4 * ctx->d * ctx->spre[l] * 16;   // this lattice in the FP64 half fields
    const size_t po = (size_t)ctx->vpre[l] * 4 * ctx->N * ctx->N * 16;
    auto at = [so](const void *p) { return static_cast<const void *>(static_cast<const char *>(p) + so); };
    WD_HIP(wd::launch_force_links(static_cast<char *>(P) + po, at(x_e), at(z_o), at(y_e), at(w_o),
                                  static_cast<const char *>(UR64) + (size_t)8 * ctx->d * ctx->d * ctx->spre[l] * el,
                                  U ? static_cast<const char *>(U) + po : nullptr, ctx->g[l], ctx->N, ctx->rep, scale,
                                  accumulate, st));
  }
  WD_HIP(hipStreamSynchronize(st));
  return WDIRAC_OK;
}

// ------------------------------------------------------------ clover force
static size_t clover_offset(const wdirac_ctx *c, int l) {
  return (size_t)4 * c->d * (2 * c->d + 1) * c->spre[l] * 2 * 8;
}

static int clover_force_checks(const wdirac_ctx *ctx, const void *P, const void *U, const void *clov64, double m0,
                               double csw, int exponential, int gradient, int accumulate, const void *workspace) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(P, "out"));
  WD_TRY(check_ptr(U, "U"));
  WD_TRY(check_ptr(clov64, "clov64"));
  WD_TRY(check_ptr(workspace, "workspace"));
  if (!wd::clover_supported(ctx->d)) return fail(WDIRAC_EUNSUPPORTED, "clover term available for d_R in {2,3,4,6}");
  if (!std::isfinite(m0) || !std::isfinite(csw) || 4.0 + m0 == 0.0)
    return fail(WDIRAC_EINVAL, "m0 and csw must be finite and 4 + m0 != 0");
  if (exponential != 0 && exponential != 1) return fail(WDIRAC_EINVAL, "exponential must be 0 or 1");
  if (gradient != 0 && gradient != 1) return fail(WDIRAC_EINVAL, "gradient must be 0 or 1");
  if (accumulate != 0 && accumulate != 1) return fail(WDIRAC_EINVAL, "accumulate must be 0 or 1");
  return WDIRAC_OK;
}

int wdirac_force_eo_clover(const wdirac_ctx *ctx, void *P, const void *x_e, const void *UR64, const void *U,
                           const void *clov64, double m0, double csw, int exponential, double scale, int gradient,
                           int accumulate, void *workspace, void *stream) {
  WD_TRY(clover_force_checks(ctx, P, U, clov64, m0, csw, exponential, gradient, accumulate, workspace));
  WD_TRY(check_ptr(x_e, "x_e"));
  WD_TRY(check_ptr(UR64, "UR64"));
  const hipStream_t st = S(stream);
  const CloverForceWs w = carve_clover_force(ctx, workspace);
  // z_o = D_oo^{-1} D_oe x;  y_e = D_ee x - D_eo z_o = D-hat x;  w_o = D_oo^{-1} D_eo^+ y_e
  WD_TRY(hop(ctx, w.z_o, x_e, UR64, 1, 0, 1, 0.0, nullptr, 1.0, WDIRAC_F64, nullptr, st));
  WD_TRY(clover_apply(ctx, w.z_o, w.z_o, clov64, 1, 1, WDIRAC_F64, st));
  WD_TRY(clover_apply(ctx, w.y_e, x_e, clov64, 0, 1, WDIRAC_F64, st));
  WD_TRY(hop(ctx, w.y_e, w.z_o, UR64, 0, 0, 1, 1.0, w.y_e, -1.0, WDIRAC_F64, nullptr, st));
  WD_TRY(hop(ctx, w.w_o, w.y_e, UR64, 1, 1, 1, 0.0, nullptr, 1.0, WDIRAC_F64, nullptr, st));
  WD_TRY(clover_apply(ctx, w.w_o, w.w_o, clov64, 1, 1, WDIRAC_F64, st));
  const size_t el = ctx->real ? 8 : 16;
  for (int l = 0; l < ctx->nlat; ++l) {
    const size_t so = (size_t)4 * ctx->d * ctx->spre[l] * 16;
    const size_t po = links_offset(ctx, l);
    auto at = [so](const void *p) { return static_cast<const void *>(static_cast<const char *>(p) + so); };
    const char *Ul = static_cast<const char *>(U) + po;
    WD_HIP(wd::launch_force_links(static_cast<char *>(P) + po, at(x_e), at(w.z_o), at(w.y_e), at(w.w_o),
                                  static_cast<const char *>(UR64) + (size_t)8 * ctx->d * ctx->d * ctx->spre[l] * el,
                                  gradient ? Ul : nullptr, ctx->g[l], ctx->N, ctx->rep, scale, accumulate, st));
    WD_HIP(wd::launch_clover_force(static_cast<char *>(P) + po, at(x_e), at(w.z_o), at(w.y_e), at(w.w_o), Ul,
                                   static_cast<const char *>(clov64) + clover_offset(ctx, l), w.F, w.K, w.G, w.Us,
                                   ctx->g[l], ctx->N, ctx->rep, m0, csw, exponential, 0.0, csw / 8.0 * scale,
                                   gradient, 1, st));
  }
  WD_HIP(hipStreamSynchronize(st));
  return WDIRAC_OK;
}

int wdirac_force_clover_logdet(const wdirac_ctx *ctx, void *P, const void *U, const void *clov64, double m0,
                               double csw, int exponential, double scale, int gradient, int accumulate,
                               void *workspace, void *stream) {
  WD_TRY(clover_force_checks(ctx, P, U, clov64, m0, csw, exponential, gradient, accumulate, workspace));
  const hipStream_t st = S(stream);
  const CloverForceWs w = carve_clover_force(ctx, workspace);
  for (int l = 0; l < ctx->nlat; ++l) {
    const size_t po = links_offset(ctx, l);
    WD_HIP(wd::launch_clover_force(static_cast<char *>(P) + po, nullptr, nullptr, nullptr, nullptr,
                                   static_cast<const char *>(U) + po,
                                   static_cast<const char *>(clov64) + clover_offset(ctx, l), w.F, w.K, w.G, w.Us,
                                   ctx->g[l], ctx->N, ctx->rep, m0, csw, exponential, 1.0, csw / 8.0 * scale,
                                   gradient, accumulate, st));
  }
  WD_HIP(hipStreamSynchronize(st));
  return WDIRAC_OK;
}

int wdirac_clover_logdet(const wdirac_ctx *ctx, double *logdet, const void *clov64, void *workspace, void *stream) {
  WD_TRY(check_ctx(ctx));
  WD_TRY(check_ptr(logdet, "logdet"));
  WD_TRY(check_ptr(clov64, "clov64"));
  WD_TRY(check_ptr(workspace, "workspace"));
  if (!wd::clover_supported(ctx->d)) return fail(WDIRAC_EUNSUPPORTED, "clover term available for d_R in {2,3,4,6}");
  const hipStream_t st = S(stream);
  const CloverForceWs w = carve_clover_force(ctx, workspace);
  for (int l = 0; l < ctx->nlat; ++l) {
    WD_HIP(wd::launch_clover_logdet(static_cast<const char *>(clov64) + clover_offset(ctx, l), w.part, ctx->g[l],
                                    ctx->d, st));
    WD_TRY(reduce_to_host(&logdet[l], w.part, wd::clover_logdet_blocks(ctx->g[l]), w.dtmp, st));
  }
  return WDIRAC_OK;
}

}  // extern "C"
