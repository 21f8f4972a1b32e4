"""C-ABI checks that need no GPU: the library loads, exports every function
include/wdirac.h declares, and rejects bad arguments on the host before any
device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, 'include', 'wdirac.h')
LIB = os.path.join(ROOT, 'paper_2503_06721_amd', 'libwdirac.so')


@pytest.fixture(scope='module')
def W():
    if not os.path.exists(LIB):
        from paper_2503_06721_amd import build
        build.build()
    from paper_2503_06721_amd import wdirac
    return wdirac


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r'/\*.*?\*/', '', text, flags=re.S)
    return sorted(set(re.findall(r'\b(wdirac_\w+)\s*\(', text)))


def test_every_declared_symbol_is_exported(W):
    names = declared_functions()
    assert len(names) >= 18
    lib = ctypes.CDLL(W.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def geom(W, dims=(4, 4, 4, 4), bc=(-1, 1, 1, 1)):
    return W.Geom((ctypes.c_int32 * 4)(*dims), (ctypes.c_int32 * 4)(*bc))


def create(W, N, rep, dims=(4, 4, 4, 4), bc=(-1, 1, 1, 1)):
    h = ctypes.c_void_p()
    g = geom(W, dims, bc)
    rc = W._lib.wdirac_create(ctypes.byref(h), N, rep, ctypes.byref(g))
    return rc, h


@pytest.mark.parametrize('N,rep,d,real', [(2, 0, 2, 0), (2, 1, 3, 1), (2, 2, 3, 0), (3, 0, 3, 0), (3, 1, 8, 1),
                                          (3, 2, 6, 0), (3, 3, 3, 0), (4, 0, 4, 0), (4, 1, 15, 1), (4, 2, 10, 0),
                                          (4, 3, 6, 0)])
def test_create_and_rep_info(W, N, rep, d, real):
    rc, h = create(W, N, rep)
    assert rc == W.OK
    dd, rr = ctypes.c_int(), ctypes.c_int()
    assert W._lib.wdirac_rep_info(h, ctypes.byref(dd), ctypes.byref(rr)) == W.OK
    assert (dd.value, rr.value) == (d, real)
    Vh, stride = 128, 256
    assert W._lib.wdirac_field_bytes(h, W.FIELD_HALF_SPINOR, 1, W.F64) == 4 * d * stride * 16
    assert W._lib.wdirac_field_bytes(h, W.FIELD_HALF_SPINOR, 3, W.F32) == 3 * 4 * d * stride * 8
    # two-index representations with compact hop forms also hold the fundamental links
    compact = (rep == 2 and N >= 2) or (rep == 3 and N == 4)
    assert W._lib.wdirac_field_bytes(h, W.FIELD_LINKS, 1, W.F64) == (8 * d * d * stride * 8 * (1 if real else 2)
                                                                     + (8 * N * N * stride * 16 if compact else 0))
    assert W._lib.wdirac_workspace_bytes(h, W.OP_CG, 2, W.CG_MIXED) > W._lib.wdirac_workspace_bytes(h, W.OP_CG, 2,
                                                                                                     W.CG_F64)
    assert Vh * 2 == 256
    assert W._lib.wdirac_destroy(h) == W.OK


@pytest.mark.parametrize('N,rep,dims,bc,code', [
    (2, 3, (4, 4, 4, 4), (1, 1, 1, 1), -2),     # SU(2) 2AS: d_R = 1
    (5, 0, (4, 4, 4, 4), (1, 1, 1, 1), -2),     # N not built
    (3, 7, (4, 4, 4, 4), (1, 1, 1, 1), -1),     # unknown rep
    (3, 0, (4, 3, 4, 4), (1, 1, 1, 1), -1),     # odd extent
    (3, 0, (0, 4, 4, 4), (1, 1, 1, 1), -1),     # empty lattice
    (3, 0, (4, 4, 4, 4), (1, 0, 1, 1), -1),     # bc not +-1
])
def test_create_rejects(W, N, rep, dims, bc, code):
    rc, h = create(W, N, rep, dims, bc)
    assert rc == code
    assert not h.value
    assert len(W.last_error()) > 0


def test_null_and_range_checks(W):
    rc, h = create(W, 3, 0)
    assert rc == W.OK
    L = W._lib
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first
    assert L.wdirac_dslash_eo(h, None, dummy, dummy, 0, 0, 1, 0.0, None, 1.0, 0, None) == W.EINVAL
    assert L.wdirac_dslash_eo(h, dummy, dummy, dummy, 2, 0, 1, 0.0, None, 1.0, 0, None) == W.EINVAL
    assert L.wdirac_dslash_eo(h, dummy, dummy, dummy, 0, 0, 13, 0.0, None, 1.0, 0, None) == W.EINVAL
    assert L.wdirac_dslash_eo(h, dummy, dummy, dummy, 0, 0, 0, 0.0, None, 1.0, 0, None) == W.EINVAL
    assert L.wdirac_dslash_eo(h, dummy, dummy, dummy, 0, 2, 1, 0.0, None, 1.0, 0, None) == W.EINVAL
    assert L.wdirac_dslash_eo(h, dummy, dummy, dummy, 0, 0, 1, 0.0, None, 1.0, 5, None) == W.EINVAL
    assert L.wdirac_dslash_eo(h, dummy, dummy, dummy, 0, 0, 1, 0.0, None, 1.0, 0, None) == W.EINVAL  # in == out
    assert L.wdirac_dslash_eo(None, dummy, dummy, dummy, 0, 0, 1, 0.0, None, 1.0, 0, None) == W.EINVAL
    assert L.wdirac_apply_Mee(h, dummy, dummy, -4.0, 1, 1, 0, None) == W.EINVAL
    assert L.wdirac_eo_reconstruct(h, dummy, ctypes.c_void_p(0x2000), dummy, dummy, -4.0, 1, None) == W.EINVAL
    st = (W.CgStats * 1)()
    assert L.wdirac_cg_eo(h, dummy, dummy, dummy, None, -0.2, 0.0, 10, 1, 0, dummy, st, None) == W.EINVAL
    assert L.wdirac_cg_eo(h, dummy, dummy, dummy, None, -0.2, 1e-10, 10, 1, 1, dummy, st, None) == W.EINVAL
    assert L.wdirac_cg_eo(h, dummy, dummy, dummy, None, -0.2, 1e-10, 10, 1, 7, dummy, st, None) == W.EINVAL
    assert L.wdirac_set_option(h, W.OPT_CG_CHECK_EVERY, 0.0) == W.EINVAL
    assert L.wdirac_set_option(h, W.OPT_MIXED_DELTA, 1.5) == W.EINVAL
    assert L.wdirac_set_option(h, 99, 1.0) == W.EINVAL
    assert L.wdirac_set_option(h, W.OPT_TILE_TBLOCK, -100.0) == W.EINVAL
    assert L.wdirac_set_option(h, W.OPT_TILE_TBLOCK, 65.0) == W.EINVAL
    for tb in (-99.0, -33.0, 64.0, 0.0):
        assert L.wdirac_set_option(h, W.OPT_TILE_TBLOCK, tb) == W.OK
    assert L.wdirac_set_option(h, W.OPT_HOP_VARIANT_F64, W.HOP_SITE) == W.OK
    assert L.wdirac_field_bytes(h, 9, 1, 0) == 0
    assert L.wdirac_workspace_bytes(h, 10, 1, 0) == 0
    assert L.wdirac_destroy(h) == W.OK


def test_site_variant_unavailable_for_large_rep(W):
    rc, h = create(W, 4, 1)   # SU(4) ADJ, d = 15
    assert rc == W.OK
    assert W._lib.wdirac_set_option(h, W.OPT_HOP_VARIANT_F64, W.HOP_SITE) == W.EUNSUPPORTED
    assert W._lib.wdirac_set_option(h, W.OPT_HOP_VARIANT_F64, W.HOP_COLOUR_QUAD) == W.EUNSUPPORTED
    assert W._lib.wdirac_destroy(h) == W.OK
    rc, h6 = create(W, 3, 2)   # SU(3) SYM, d = 6: four hops per phase available
    assert rc == W.OK
    assert W._lib.wdirac_set_option(h6, W.OPT_HOP_VARIANT_F64, W.HOP_COLOUR_QUAD) == W.OK
    assert W._lib.wdirac_destroy(h6) == W.OK
    rc, h = create(W, 4, 1)
    assert rc == W.OK
    # the multi-rhs staged-link form is built for d_R = 3 and 6 only
    assert W._lib.wdirac_set_option(h, W.OPT_HOP_VARIANT_F64, W.HOP_MULTI) == W.EUNSUPPORTED
    assert W._lib.wdirac_set_option(h, W.OPT_HOP_VARIANT_F64, 7) == W.EINVAL
    assert W._lib.wdirac_set_option(h, W.OPT_HOP_NR_F64, 13) == W.EINVAL
    assert W._lib.wdirac_set_option(h, W.OPT_TUNE_COMPACT, 2) == W.EINVAL
    assert W._lib.wdirac_set_option(h, W.OPT_TUNE_COMPACT, 0) == W.OK
    W._lib.wdirac_destroy(h)


def create_batch(W, N, rep, shapes, bc=(-1, 1, 1, 1)):
    h = ctypes.c_void_p()
    gs = (W.Geom * len(shapes))(*[geom(W, dd, bc) for dd in shapes]) if shapes else None
    rc = W._lib.wdirac_create_batch(ctypes.byref(h), N, rep, gs, len(shapes))
    return rc, h


def test_batch_sizes_and_rejects(W):
    shapes = [(4, 6, 4, 6), (2, 2, 2, 2), (8, 8, 8, 8)]
    rc, h = create_batch(W, 3, 2, shapes)            # SU(3) SYM, d = 6
    assert rc == W.OK
    rows = [((dd[0] * dd[1] * dd[2] * dd[3] // 2 + 255) // 256) * 256 for dd in shapes]
    # pitches that are a multiple of 1024 entries are padded by 256
    strides = [r + 256 if r % 1024 == 0 else r for r in rows]
    assert W._lib.wdirac_field_bytes(h, W.FIELD_HALF_SPINOR, 1, W.F64) == 4 * 6 * sum(strides) * 16
    assert W._lib.wdirac_field_bytes(h, W.FIELD_LINKS, 1, W.F32) == (8 * 36 + 8 * 9) * sum(strides) * 8
    dummy = ctypes.c_void_p(0x1000)
    # a batch carries one right-hand side per lattice
    assert W._lib.wdirac_dslash_eo(h, dummy, ctypes.c_void_p(0x2000), dummy, 0, 0, 2, 0.0, None, 1.0, 0,
                                   None) == W.EINVAL
    assert 'one right-hand side' in W.last_error()
    assert W._lib.wdirac_destroy(h) == W.OK
    assert create_batch(W, 3, 0, [(4, 4, 4, 4)] * 9)[0] == W.EINVAL        # more than 8 lattices
    assert create_batch(W, 3, 0, [])[0] == W.EINVAL                         # none
    assert create_batch(W, 3, 0, [(4, 4, 4, 4), (4, 3, 4, 4)])[0] == W.EINVAL  # an odd extent in a later lattice


def test_mshift_argument_checks(W):
    rc, h = create(W, 3, 0)
    assert rc == W.OK
    L = W._lib
    dummy = ctypes.c_void_p(0x1000)
    st = (W.CgStats * 33)()
    sh = (ctypes.c_double * 33)(*([0.1] * 33))
    hb = L.wdirac_field_bytes(h, W.FIELD_HALF_SPINOR, 1, W.F64)
    x, b = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x100000 + 2 * hb)
    assert L.wdirac_cg_mshift_eo(h, x, b, dummy, -0.2, sh, 0, 1e-10, 10, dummy, st, None) == W.EINVAL
    assert L.wdirac_cg_mshift_eo(h, x, b, dummy, -0.2, sh, 33, 1e-10, 10, dummy, st, None) == W.EINVAL
    neg = (ctypes.c_double * 2)(0.1, -1.0)
    assert L.wdirac_cg_mshift_eo(h, x, b, dummy, -0.2, neg, 2, 1e-10, 10, dummy, st, None) == W.EINVAL
    # b inside the output fields
    assert L.wdirac_cg_mshift_eo(h, x, b, dummy, -0.2, sh, 3, 1e-10, 10, dummy, st, None) == W.EINVAL
    assert 'overlap' in W.last_error()
    assert L.wdirac_workspace_bytes(h, W.OP_MSHIFT, 32, W.F64) > L.wdirac_workspace_bytes(h, W.OP_MSHIFT, 1, W.F64)
    assert L.wdirac_workspace_bytes(h, W.OP_MSHIFT, 33, W.F64) == 0
    assert L.wdirac_workspace_bytes(h, W.OP_MSHIFT, 2, W.F32) == 0
    assert L.wdirac_destroy(h) == W.OK
    rc, hb2 = create_batch(W, 3, 0, [(4, 4, 4, 4), (2, 2, 2, 2)])
    assert rc == W.OK
    assert L.wdirac_cg_mshift_eo(hb2, x, ctypes.c_void_p(0x900000), dummy, -0.2, sh, 2, 1e-10, 10, dummy, st,
                                 None) == W.EUNSUPPORTED
    assert L.wdirac_workspace_bytes(hb2, W.OP_MSHIFT, 2, W.F64) == 0
    L.wdirac_destroy(hb2)


def test_stream_probe_argument_checks(W):
    L = W._lib
    out = ctypes.c_double()
    dummy = ctypes.c_void_p(0x1000)
    assert L.wdirac_stream_probe(None, 1024, 7, 1, ctypes.byref(out), None) == W.EINVAL
    assert L.wdirac_stream_probe(dummy, 1024, 0, 1, ctypes.byref(out), None) == W.EINVAL
    assert L.wdirac_stream_probe(dummy, 1024, 9, 1, ctypes.byref(out), None) == W.EINVAL
    assert L.wdirac_stream_probe(dummy, 0, 7, 1, ctypes.byref(out), None) == W.EINVAL
    assert L.wdirac_stream_probe(dummy, 1024, 7, 0, ctypes.byref(out), None) == W.EINVAL
    assert L.wdirac_stream_probe(dummy, 1024, 7, 1, None, None) == W.EINVAL


def test_clover_argument_checks(W):
    rc, h = create(W, 3, 2)   # SU(3) SYM, d = 6
    assert rc == W.OK
    L = W._lib
    dummy = ctypes.c_void_p(0x1000)
    stride = 256
    # two chirality blocks per site and parity, upper triangles of 12 x 12
    assert L.wdirac_field_bytes(h, W.FIELD_CLOVER, 1, W.F64) == 4 * 78 * stride * 16
    assert L.wdirac_workspace_bytes(h, W.OP_CLOVER, 1, W.F64) >= 6 * 36 * 256 * 16
    assert L.wdirac_clover_field(h, dummy, dummy, -4.0, 1.0, 0, 0, dummy, None) == W.EINVAL     # 4 + m0 = 0
    assert L.wdirac_clover_field(h, dummy, dummy, -0.1, 1.0, 2, 0, dummy, None) == W.EINVAL     # exponential flag
    assert L.wdirac_clover_field(h, None, dummy, -0.1, 1.0, 0, 0, dummy, None) == W.EINVAL
    assert L.wdirac_apply_clover(h, dummy, dummy, dummy, 2, 1, 0, None) == W.EINVAL             # parity
    assert L.wdirac_apply_dhat_clover(h, dummy, dummy, dummy, dummy, 0, 1, 0, dummy, None) == W.EINVAL  # alias
    st = (W.CgStats * 1)()
    assert L.wdirac_cg_eo_clover(h, dummy, ctypes.c_void_p(0x2000), dummy, None, None, None, 1e-10, 10, 1, 0, dummy,
                                 st, None) == W.EINVAL                                          # clov64 NULL
    # clover force: workspace holds three half fields and the leaf scratch
    V = 4 * 4 * 4 * 4
    assert L.wdirac_workspace_bytes(h, W.OP_CLOVER_FORCE, 1, W.F64) >= (18 * 36 + 24 * 9) * V * 16
    assert L.wdirac_force_eo_clover(h, dummy, dummy, dummy, dummy, dummy, -4.0, 1.0, 0, 1.0, 0, 0, dummy,
                                    None) == W.EINVAL                                          # 4 + m0 = 0
    assert L.wdirac_force_eo_clover(h, dummy, dummy, dummy, dummy, dummy, 0.1, 1.0, 0, 1.0, 2, 0, dummy,
                                    None) == W.EINVAL                                          # gradient flag
    assert L.wdirac_force_eo_clover(h, dummy, None, dummy, dummy, dummy, 0.1, 1.0, 0, 1.0, 0, 0, dummy,
                                    None) == W.EINVAL                                          # x_e NULL
    assert L.wdirac_force_clover_logdet(h, dummy, None, dummy, 0.1, 1.0, 0, 1.0, 0, 0, dummy, None) == W.EINVAL
    assert L.wdirac_force_clover_logdet(h, dummy, dummy, dummy, 0.1, 1.0, 0, 1.0, 0, 3, dummy, None) == W.EINVAL
    ld = (ctypes.c_double * 1)()
    assert L.wdirac_clover_logdet(h, ld, None, dummy, None) == W.EINVAL
    L.wdirac_destroy(h)
    rc, h = create(W, 4, 1)   # SU(4) ADJ, d = 15: no clover
    assert L.wdirac_field_bytes(h, W.FIELD_CLOVER, 1, W.F64) == 0
    assert L.wdirac_workspace_bytes(h, W.OP_CLOVER_FORCE, 1, W.F64) == 0
    assert L.wdirac_clover_field(h, dummy, dummy, -0.1, 1.0, 0, 0, dummy, None) == W.EUNSUPPORTED
    assert L.wdirac_force_clover_logdet(h, dummy, dummy, dummy, 0.1, 1.0, 0, 1.0, 0, 0, dummy, None) == W.EUNSUPPORTED
    assert L.wdirac_clover_logdet(h, ld, dummy, dummy, None) == W.EUNSUPPORTED
    L.wdirac_destroy(h)
