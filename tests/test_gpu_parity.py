"""GPU path (through the C ABI) against the CPU oracle, element by element on
the same seeded inputs: represented links, packing, the hopping blocks in
both parities and their adjoints, the diagonal blocks, D-hat, source
preparation and reconstruction, norms, CG and the force.

Tolerances: relative 2-norm 1e-13 in FP64, 1e-6 in FP32 (FP32 runs consume
FP32-rounded inputs and are compared with the FP64 oracle on FP64 inputs);
integer/byte work (packing) bit-exact."""
import numpy as np
import pytest

from gpu_common import APBC, TOL, Setup, log, rel, wdirac
from oracle import cg as OCG
from oracle import dirac as D
from oracle import force as OF
from oracle import lattice as L
from oracle.reductions import norm2

pytestmark = pytest.mark.gpu

PAIRS = [(2, 'FUND'), (2, 'ADJ'), (2, 'SYM'), (3, 'FUND'), (3, 'ADJ'), (3, 'SYM'), (3, '2AS'),
         (4, 'FUND'), (4, 'ADJ'), (4, 'SYM'), (4, '2AS')]
# extents: a lattice spanning several 64-site tiles with a ragged tail, and
# the 2^4 lattice on which x+mu and x-mu coincide
DIMS = [(4, 6, 4, 6), (2, 2, 2, 2)]


@pytest.fixture(scope='module')
def W():
    import torch
    assert torch.cuda.is_available(), 'GPU tests need a GPU'
    return wdirac()


@pytest.mark.parametrize('dims', DIMS)
@pytest.mark.parametrize('N,rep', PAIRS)
def test_rep_links(W, N, rep, dims):
    log(f'rep_links N={N} rep={rep} dims={dims}')
    s = Setup(N, rep, dims, seed=100 + N, bc=(-1, 1, -1, 1))
    expect = D.links_with_boundary_phase(s.UR, s.bc)
    for prec in (0, 1):
        got = s.lat.links_canonical(s.URg[prec], prec).cpu().numpy()
        assert got.dtype == (np.float64 if rep == 'ADJ' else np.complex128)
        assert rel(got, expect) < TOL[prec], (prec, rel(got, expect))


@pytest.mark.parametrize('prec', [0, 1])
def test_pack_roundtrip_exact(W, prec):
    import torch
    s = Setup(3, 'SYM', (4, 6, 4, 6), seed=7, precs=(0,))
    full = s.spinor(8, nrhs=3).astype(np.complex128 if prec == 0 else np.complex64)
    t = torch.from_numpy(full).cuda()
    for p in (0, 1):
        packed = s.lat.pack_half(t, p, 3, prec)
        back = s.lat.unpack_half(packed, p, 3, prec).cpu().numpy()
        mask = (L.parity_field(s.dims) == p)[None, ..., None, None]
        assert np.array_equal(np.where(mask, full, 0), back)


def hop_expect(s, psi_full, p, dagger, alpha, beta, xadd_full):
    out = []
    for r in range(psi_full.shape[0]):
        h = D.hop_block(L.to_half(psi_full[r], s.dims, 1 - p), s.UR, s.bc, s.dims, p, dagger=bool(dagger))
        v = beta * h
        if xadd_full is not None:
            v = v + alpha * L.to_half(xadd_full[r], s.dims, p)
        out.append(v)
    return np.stack(out)


@pytest.mark.parametrize('dims', DIMS)
@pytest.mark.parametrize('N,rep', PAIRS)
def test_dslash_eo(W, N, rep, dims):
    s = Setup(N, rep, dims, seed=200 + N)
    variants = ([W.HOP_COLOUR] + ([W.HOP_SITE] if s.d <= 6 else []) + ([W.HOP_COLOUR_QUAD] if s.d <= 6 else [])
                + ([W.HOP_COMPACT, W.HOP_COMPACT_PAIR] if s.lat.compact else []))
    nrhs = 2
    psi = s.spinor(201, nrhs)
    xadd = s.spinor(202, nrhs)
    for variant in variants:
        for prec in (0, 1):
            s.lat.set_option(W.OPT_HOP_VARIANT_F64 if prec == 0 else W.OPT_HOP_VARIANT_F32, variant)
            for p in (0, 1):
                for dagger in (0, 1):
                    for (alpha, beta, use_x) in ((0.0, 1.0, False), (0.7, -1.3, True)):
                        log(f'dslash N={N} rep={rep} dims={dims} var={variant} prec={prec} p={p} dag={dagger}')
                        inp = s.to_gpu_half(psi, 1 - p, prec)
                        xg = s.to_gpu_half(xadd, p, prec) if use_x else None
                        out = s.lat.new_half(nrhs, prec)
                        s.lat.dslash_eo(out, inp, s.URg[prec], p, dagger, nrhs, alpha, xg, beta, prec)
                        got = s.from_gpu_half(out, p, nrhs, prec)
                        exp = hop_expect(s, psi, p, dagger, alpha, beta, xadd if use_x else None)
                        err = rel(got, exp)
                        assert err < TOL[prec], (variant, prec, p, dagger, alpha, err)


@pytest.mark.parametrize('N,rep', [(3, 'FUND'), (3, 'SYM'), (2, 'ADJ'), (4, 'FUND'), (4, '2AS')])
def test_dslash_rhs_groups(W, N, rep):
    """Several right-hand sides sharing each link load (1..4 per block in the
    colour-split forms, 6 in the unpaired form for d_R <= 4, 4 across the
    lanes of a wavefront in the site-parallel form), with a ragged tile tail;
    every rhs must equal its own single-rhs hop."""
    s = Setup(N, rep, (4, 6, 4, 6), seed=250 + N)
    for nrhs in (4, 6, 12):
        psi = s.spinor(251 + nrhs, nrhs)
        exp = {(p, dagger): hop_expect(s, psi, p, dagger, 0.0, 1.0, None) for p, dagger in ((0, 0), (1, 1))}
        for prec in (0, 1):
            for variant in (W.HOP_COLOUR, W.HOP_COLOUR_PAIR, W.HOP_SITE) + (
                    (W.HOP_COMPACT, W.HOP_COMPACT_PAIR) if s.lat.compact else ()) + (
                    (W.HOP_COLOUR_QUAD,) if s.d <= 6 else ()):
                s.lat.set_option(W.OPT_HOP_VARIANT_F64 if prec == 0 else W.OPT_HOP_VARIANT_F32, variant)
                for nr in (1, 2, 3, 4, 6):
                    s.lat.set_option(W.OPT_HOP_NR_F64 if prec == 0 else W.OPT_HOP_NR_F32, nr)
                    log(f'rhs groups N={N} rep={rep} nrhs={nrhs} prec={prec} variant={variant} nr={nr}')
                    for p, dagger in ((0, 0), (1, 1)):
                        inp = s.to_gpu_half(psi, 1 - p, prec)
                        out = s.lat.new_half(nrhs, prec)
                        s.lat.dslash_eo(out, inp, s.URg[prec], p, dagger, nrhs, 0.0, None, 1.0, prec)
                        got = s.from_gpu_half(out, p, nrhs, prec)
                        assert rel(got, exp[(p, dagger)]) < TOL[prec], (nrhs, prec, variant, nr, p)


MULTI_PAIRS = [(3, 'FUND'), (3, 'SYM'), (4, '2AS'), (2, 'ADJ')]


@pytest.mark.parametrize('dims', [(4, 6, 4, 6), (2, 6, 2, 6), (2, 2, 2, 2)])
@pytest.mark.parametrize('N,rep', MULTI_PAIRS)
def test_dslash_multi_rhs_staged_links(W, N, rep, dims):
    """The multi-rhs form with links staged in LDS (one wavefront per rhs, two
    lanes per site for d_R = 6): every rhs group size, both parities, the
    dagger form, the x_add epilogue, both precisions, both XCD mappings;
    (2, 6, 2, 6) leaves a ragged tile tail (36 sites per parity) and 2^4 has
    x+mu = x-mu."""
    s = Setup(N, rep, dims, seed=280 + N)
    for nrhs, nrs in ((12, (1, 2, 3, 4, 6, 12)), (4, (1, 2, 4))):
        psi = s.spinor(281 + nrhs, nrhs)
        xadd = s.spinor(282 + nrhs, nrhs)
        exp = {(p, dagger, use_x): hop_expect(s, psi, p, dagger, 0.6 if use_x else 0.0, -1.1 if use_x else 1.0,
                                              xadd if use_x else None)
               for p in (0, 1) for dagger in (0, 1) for use_x in (False, True)}
        for prec, nr, remap in [(pr, n, m) for pr in (0, 1) for n in nrs for m in (0, 1)]:
            s.lat.set_option(W.OPT_HOP_VARIANT_F64 if prec == 0 else W.OPT_HOP_VARIANT_F32, W.HOP_MULTI)
            s.lat.set_option(W.OPT_XCD_REMAP, remap)
            s.lat.set_option(W.OPT_HOP_NR_F64 if prec == 0 else W.OPT_HOP_NR_F32, nr)
            log(f'multi-rhs N={N} rep={rep} dims={dims} nrhs={nrhs} prec={prec} nr={nr} remap={remap}')
            for (p, dagger, use_x), e in exp.items():
                inp = s.to_gpu_half(psi, 1 - p, prec)
                xg = s.to_gpu_half(xadd, p, prec) if use_x else None
                out = s.lat.new_half(nrhs, prec)
                s.lat.dslash_eo(out, inp, s.URg[prec], p, dagger, nrhs, 0.6 if use_x else 0.0, xg,
                                -1.1 if use_x else 1.0, prec)
                err = rel(s.from_gpu_half(out, p, nrhs, prec), e)
                assert err < TOL[prec], (nrhs, prec, nr, remap, p, dagger, use_x, err)


@pytest.mark.parametrize('mode', [0, 1])
def test_cg_multi_rhs_staged_links(W, mode):
    """Batched CG with the multi-rhs form (its per-tile |D-hat p|^2 partial
    sums feed <p, A p>): every rhs reaches the oracle's true residual."""
    m = -0.3
    s = Setup(3, 'SYM', (4, 6, 4, 6), seed=290, links='expH')
    for prec in (0, 1):
        s.lat.set_option(W.OPT_HOP_VARIANT_F64 if prec == 0 else W.OPT_HOP_VARIANT_F32, W.HOP_MULTI)
        s.lat.set_option(W.OPT_HOP_NR_F64 if prec == 0 else W.OPT_HOP_NR_F32, 3)
    nrhs = 6
    full = s.spinor(291, nrhs)
    b = s.half(full, 0)
    x = s.lat.new_half(nrhs)
    rc, st = s.lat.cg_eo(x, s.to_gpu_half(full, 0), s.URg[0], m, tol=1e-10, maxit=5000, nrhs=nrhs, mode=mode,
                         UR32=s.URg[1])
    assert rc == W.OK, st
    xs = s.from_gpu_half(x, 0, nrhs)
    for r in range(nrhs):
        res = np.sqrt(norm2(b[r] - D.normal_op(xs[r], s.UR, m, s.bc, s.dims)) / norm2(b[r]))
        assert res <= 1.001e-10, (r, res, st[r])
        _, it_or, _ = OCG.cg_eo(b[r], s.UR, m, s.bc, s.dims, tol=1e-10, maxit=5000)
        if mode == 0:
            assert abs(st[r]['iters'] - it_or) <= 2, (r, st[r]['iters'], it_or)


@pytest.mark.parametrize('variant', [1, 2, 0])
def test_dslash_tile_orders(W, variant):
    """t-blocked and sub-lattice tile orders permute the work, never the
    result (codes -(10 bx + by) with bx | X = 6 and by | 1 tile per row; -22
    does not fit and falls back to lexicographic order)."""
    s = Setup(3, 'FUND', (8, 6, 8, 16), seed=270)   # Y*Z = 128: whole tiles per (t, x) row
    psi = s.spinor(271, 2)
    for tb in (0, 2, 4, 8, -11, -21, -31, -61, -22):
        s.lat.set_option(W.OPT_TILE_TBLOCK, tb)
        for prec in (0, 1):
            s.lat.set_option(W.OPT_HOP_VARIANT_F64 if prec == 0 else W.OPT_HOP_VARIANT_F32, variant)
            for p, dagger in ((0, 0), (1, 1)):
                inp = s.to_gpu_half(psi, 1 - p, prec)
                out = s.lat.new_half(2, prec)
                s.lat.dslash_eo(out, inp, s.URg[prec], p, dagger, 2, 0.0, None, 1.0, prec)
                got = s.from_gpu_half(out, p, 2, prec)
                assert rel(got, hop_expect(s, psi, p, dagger, 0.0, 1.0, None)) < TOL[prec], (tb, prec, p)


@pytest.mark.parametrize('N,rep', [(3, 'SYM'), (3, 'FUND')])
def test_multi_rhs_tile_orders(W, N, rep):
    """The multi-rhs form (12 rhs, 4 per block, 3 groups) under the
    sub-lattice sweeps and t-blocks: with d_R = 6 a tile is 32 sites, so a
    (t, x) row of Y*Z = 128 sites holds 2 tiles and by may be 1 or 2."""
    s = Setup(N, rep, (4, 4, 8, 16), seed=275, precs=(0,))
    nrhs = 12
    psi = s.spinor(276, nrhs)
    exp = hop_expect(s, psi, 0, 0, 0.0, 1.0, None)
    s.lat.set_option(W.OPT_HOP_VARIANT_F64, W.HOP_MULTI)
    s.lat.set_option(W.OPT_HOP_NR_F64, 4)
    for tb in (0, 2, -11, -21, -41, -12, -22, -42):
        s.lat.set_option(W.OPT_TILE_TBLOCK, tb)
        inp = s.to_gpu_half(psi, 1, 0)
        out = s.lat.new_half(nrhs, 0)
        s.lat.dslash_eo(out, inp, s.URg[0], 0, 0, nrhs, 0.0, None, 1.0, 0)
        assert rel(s.from_gpu_half(out, 0, nrhs, 0), exp) < TOL[0], tb


def test_autotune_keeps_results(W):
    s = Setup(3, 'SYM', (4, 6, 4, 6), seed=260)
    for prec in (0, 1):
        for nrhs in (1, 4):
            best = s.lat.autotune(s.URg[prec], prec, nrhs)
            log(f'autotune prec={prec} nrhs={nrhs}: {best}')
            assert best['candidates'] >= 2 and best['us'] > 0
            psi = s.spinor(261, nrhs)
            inp = s.to_gpu_half(psi, 1, prec)
            out = s.lat.new_half(nrhs, prec)
            s.lat.dslash_eo(out, inp, s.URg[prec], 0, 0, nrhs, 0.0, None, 1.0, prec)
            assert rel(s.from_gpu_half(out, 0, nrhs, prec), hop_expect(s, psi, 0, 0, 0.0, 1.0, None)) < TOL[prec]


def test_dslash_in_place_xadd(W):
    """x_add may alias out (documented)."""
    s = Setup(3, 'FUND', (4, 6, 4, 6), seed=300, precs=(0,))
    psi = s.spinor(301)
    x = s.spinor(302)
    inp = s.to_gpu_half(psi, 1, 0)
    out = s.to_gpu_half(x, 0, 0)
    s.lat.dslash_eo(out, inp, s.URg[0], 0, 0, 1, 2.0, out, 0.5, 0)
    exp = hop_expect(s, psi, 0, 0, 2.0, 0.5, x)
    assert rel(s.from_gpu_half(out, 0), exp) < TOL[0]


@pytest.mark.parametrize('N,rep', [(2, 'FUND'), (3, 'SYM'), (4, '2AS'), (2, 'ADJ')])
def test_diag_dhat_source_reconstruct(W, N, rep):
    log(f'dhat N={N} rep={rep}')
    s = Setup(N, rep, (4, 6, 4, 6), seed=400 + N, precs=(0, 1))
    m = -0.3
    eta = s.spinor(401)
    eta_e, eta_o = s.half(eta, 0)[0], s.half(eta, 1)[0]
    ge, go = s.to_gpu_half(eta, 0), s.to_gpu_half(eta, 1)
    out = s.lat.new_half()
    # diagonal blocks and their inverses
    s.lat.apply_Mee(out, ge, m)
    assert rel(s.from_gpu_half(out, 0)[0], (4 + m) * eta_e) < TOL[0]
    s.lat.apply_Moo(out, go, m, inverse=1)
    assert rel(s.from_gpu_half(out, 1)[0], eta_o / (4 + m)) < TOL[0]
    # D-hat and its adjoint
    for prec in (0, 1):
        gin = s.to_gpu_half(eta, 0, prec)
        o = s.lat.new_half(1, prec)
        for dagger in (0, 1):
            s.lat.apply_dhat(o, gin, s.URg[prec], m, dagger, 1, prec)
            f = D.Dhat_dag if dagger else D.Dhat
            exp = f(eta_e, s.UR, m, s.bc, s.dims)
            assert rel(s.from_gpu_half(o, 0, 1, prec)[0], exp) < TOL[prec], (prec, dagger)
    # source preparation and reconstruction (FP64)
    b = s.lat.new_half()
    s.lat.eo_source(b, ge, go, s.URg[0], m)
    assert rel(s.from_gpu_half(b, 0)[0], D.eo_source(eta[0], s.UR, m, s.bc, s.dims)) < TOL[0]
    psi_e = s.spinor(402)
    pe = s.to_gpu_half(psi_e, 0)
    po = s.lat.new_half()
    s.lat.eo_reconstruct(po, pe, go, s.URg[0], m)
    exp_o = (eta_o - D.D_oe(s.half(psi_e, 0)[0], s.UR, s.bc, s.dims)) / (4 + m)
    assert rel(s.from_gpu_half(po, 1)[0], exp_o) < TOL[0]


def test_norm2(W):
    s = Setup(3, 'FUND', (4, 6, 4, 6), seed=500, precs=(0,))
    psi = s.spinor(501, nrhs=3)
    g = s.to_gpu_half(psi, 1)
    got = s.lat.norm2(g, nrhs=3)
    exp = [norm2(h) for h in s.half(psi, 1)]
    assert np.allclose(got, exp, rtol=1e-14, atol=0)


def test_dot(W):
    from oracle.reductions import inner
    s = Setup(2, 'SYM', (4, 6, 4, 6), seed=510, precs=(0,))
    a, b = s.spinor(511, nrhs=2), s.spinor(512, nrhs=2)
    ga, gb = s.to_gpu_half(a, 0), s.to_gpu_half(b, 0)
    got = s.lat.dot(ga, gb, nrhs=2)
    for k in range(2):
        exp = inner(s.half(a, 0)[k], s.half(b, 0)[k])
        assert abs(got[k] - exp) <= 1e-14 * abs(exp)
    # norms of FP32 fields are accumulated in FP64
    g32 = s.to_gpu_half(a, 0, prec=1)
    n32 = s.lat.norm2(g32, nrhs=2, prec=1)
    exp32 = [norm2(h) for h in s.half(a.astype(np.complex64).astype(np.complex128), 0)]
    assert np.allclose(n32, exp32, rtol=1e-13, atol=0)


def solve_problem(s, m, seed):
    eta = s.spinor(seed)
    bprime = D.eo_source(eta[0], s.UR, m, s.bc, s.dims)
    rhs = D.Dhat_dag(bprime, s.UR, m, s.bc, s.dims)
    return rhs


def oracle_true_residual(s, x, b, m):
    r = b - D.normal_op(x, s.UR, m, s.bc, s.dims)
    return np.sqrt(norm2(r) / norm2(b))


def test_cg_f64_su2_fund_4x4x4x4(W):
    """Haar-random SU(2) fundamental 4^4, m0 = -0.2, antiperiodic in time."""
    log('cg f64 su2 fund 4^4')
    s = Setup(2, 'FUND', (4, 4, 4, 4), seed=1000, precs=(0,))
    m = -0.2
    b = solve_problem(s, m, 2000)
    x_or, it_or, res_or = OCG.cg(lambda v: D.normal_op(v, s.UR, m, s.bc, s.dims), b, 1e-10, 5000)
    bg = s.to_gpu_half(_embed(s, b), 0)
    xg = s.lat.new_half()
    rc, st = s.lat.cg_eo(xg, bg, s.URg[0], m, tol=1e-10, maxit=5000)
    assert rc == W.OK, st
    x = s.from_gpu_half(xg, 0)[0]
    res = oracle_true_residual(s, x, b, m)
    log(f'  gpu iters {st[0]["iters"]} oracle iters {it_or} res {res:.3e} lib res {st[0]["true_rel_resid"]:.3e}')
    assert res <= 1.05e-10
    assert abs(st[0]['true_rel_resid'] - res) <= 1e-12
    assert abs(st[0]['iters'] - it_or) <= 2


def _embed(s, half_e):
    """Full field (nrhs = 1) holding half_e on the even sites."""
    return L.from_half(half_e, s.dims, 0)[None]


@pytest.mark.parametrize('N,rep,m', [(3, 'FUND', -0.4), (2, 'ADJ', -1.1), (3, 'SYM', -0.4)])
def test_cg_modes_and_multi_rhs(W, N, rep, m):
    log(f'cg modes N={N} rep={rep}')
    s = Setup(N, rep, (4, 6, 4, 6), seed=600 + N, links='expH')
    nrhs = 3
    bs = [solve_problem(s, m, 610 + k) for k in range(nrhs)]
    full = np.concatenate([_embed(s, b) for b in bs])
    for mode in (W.CG_F64, W.CG_MIXED):
        bg = s.to_gpu_half(full, 0)
        xg = s.lat.new_half(nrhs)
        rc, st = s.lat.cg_eo(xg, bg, s.URg[0], m, tol=1e-10, maxit=20000, nrhs=nrhs, mode=mode, UR32=s.URg[1])
        assert rc == W.OK, st
        xs = s.from_gpu_half(xg, 0, nrhs)
        for k in range(nrhs):
            res = oracle_true_residual(s, xs[k], bs[k], m)
            log(f'  mode {mode} rhs {k}: iters {st[k]["iters"]} updates {st[k]["reliable_updates"]} res {res:.3e}')
            assert res <= 1.05e-10, (mode, k, res)
        if mode == W.CG_F64:
            # each right-hand side follows its own single-rhs recurrence
            for k in range(nrhs):
                _, it_or, _ = OCG.cg(lambda v: D.normal_op(v, s.UR, m, s.bc, s.dims), bs[k], 1e-10, 20000)
                assert abs(st[k]['iters'] - it_or) <= 2, (k, st[k]['iters'], it_or)


@pytest.mark.parametrize('N,rep,m', [(3, 'SYM', -0.4), (4, '2AS', -0.3), (2, 'SYM', -0.2)])
def test_cg_compact_links(W, N, rep, m):
    """CG with the compact hop forms (U_R rebuilt from the fundamental links
    in registers) in FP64 and mixed precision, two right-hand sides."""
    log(f'cg compact N={N} rep={rep}')
    s = Setup(N, rep, (4, 6, 4, 6), seed=640 + N, links='expH')
    assert s.lat.compact
    bs = [solve_problem(s, m, 650 + k) for k in range(2)]
    full = np.concatenate([_embed(s, b) for b in bs])
    for pair in (0, 1):
        for prec in (0, 1):
            s.lat.set_option(W.OPT_HOP_VARIANT_F64 if prec == 0 else W.OPT_HOP_VARIANT_F32,
                             W.HOP_COMPACT_PAIR if pair else W.HOP_COMPACT)
        for mode in (W.CG_F64, W.CG_MIXED):
            xg = s.lat.new_half(2)
            rc, st = s.lat.cg_eo(xg, s.to_gpu_half(full, 0), s.URg[0], m, tol=1e-10, maxit=20000, nrhs=2, mode=mode,
                                 UR32=s.URg[1])
            assert rc == W.OK, st
            xs = s.from_gpu_half(xg, 0, 2)
            for k in range(2):
                res = oracle_true_residual(s, xs[k], bs[k], m)
                log(f'  pair {pair} mode {mode} rhs {k}: iters {st[k]["iters"]} res {res:.3e}')
                assert res <= 1.05e-10, (pair, mode, k, res)


def test_cg_zero_rhs_and_maxit(W):
    s = Setup(2, 'FUND', (4, 4, 4, 4), seed=700, precs=(0,))
    m = -0.2
    zero = s.lat.new_half()
    x = s.to_gpu_half(s.spinor(701), 0)       # nonzero initial guess
    rc, st = s.lat.cg_eo(x, zero, s.URg[0], m)
    assert rc == W.OK and st[0]['iters'] == 0
    assert not s.from_gpu_half(x, 0).any()
    b = s.to_gpu_half(_embed(s, solve_problem(s, m, 702)), 0)
    x = s.lat.new_half()
    rc, st = s.lat.cg_eo(x, b, s.URg[0], m, maxit=3)
    assert rc == W.ENOCONV and st[0]['status'] == W.ENOCONV and st[0]['iters'] == 3


@pytest.mark.parametrize('N,rep,m', [(2, 'ADJ', -1.1), (3, 'FUND', -0.1), (3, 'SYM', 0.2), (4, '2AS', 0.3),
                                     (2, 'FUND', 0.0), (4, 'FUND', 0.1)])
def test_force(W, N, rep, m):
    import torch
    log(f'force N={N} rep={rep}')
    s = Setup(N, rep, (4, 6, 4, 6), seed=800 + N, links='expH', precs=(0,))
    phi = solve_problem(s, m, 801)
    x, _, _ = OCG.cg(lambda v: D.normal_op(v, s.UR, m, s.bc, s.dims), phi, 1e-12, 20000)
    exp = OF.force(x, s.UR, m, s.bc, s.dims, N, rep)
    xg = s.to_gpu_half(_embed(s, x), 0)
    P = torch.zeros(s.dims + (4, N, N), dtype=torch.complex128, device='cuda')
    s.lat.force_eo(P, xg, s.URg[0], m, scale=1.0, accumulate=0)
    got = P.cpu().numpy()
    assert rel(got, exp) < TOL[0], rel(got, exp)
    s.lat.force_eo(P, xg, s.URg[0], m, scale=-0.5, accumulate=1)
    assert rel(P.cpu().numpy(), 0.5 * exp) < TOL[0]
    # gradient form G = 2i P U (dS = Re tr(G^+ dU) for dU = i w T U)
    G = torch.zeros_like(P)
    s.lat.force_eo(G, xg, s.URg[0], m, U=s.Ug, scale=1.0)
    expG = 2j * np.einsum('...ij,...jk->...ik', exp, s.U)
    assert rel(G.cpu().numpy(), expG) < TOL[0]


def test_stream_probe_runs(W):
    """The roofline's streaming probe returns a finite positive bandwidth and
    writes the sum of its input streams."""
    import torch
    elems, nread = 1 << 16, 3
    bufs = torch.zeros((nread + 1) * elems * 2, dtype=torch.float64, device='cuda')
    for s in range(nread):
        bufs[s * elems * 2:(s + 1) * elems * 2] = float(s + 1)
    import ctypes
    out = ctypes.c_double()
    assert W._lib.wdirac_stream_probe(bufs.data_ptr(), elems, nread, 3, ctypes.byref(out), None) == W.OK
    assert out.value > 0 and np.isfinite(out.value)
    assert torch.all(bufs[nread * elems * 2:] == 6.0)


@pytest.mark.parametrize('mode', [0, 1])
def test_cg_graph_replay_matches_direct_launches(W, mode):
    """CG iterations replayed from a captured HIP graph (many replays per
    solve, host checks in between) give bit-identical solutions to direct
    launches: the same kernels in the same order."""
    import torch
    s = Setup(3, 'FUND', (8, 6, 8, 6), seed=290, links='expH')
    psi = s.spinor(291, 2)
    b = s.to_gpu_half(psi, 0)
    out = {}
    for graph in (0, 1):
        s.lat.set_option(W.OPT_CG_GRAPH, graph)
        x = s.lat.new_half(2)
        rc, st = s.lat.cg_eo(x, b, s.URg[0], -0.3, tol=1e-10, maxit=5000, nrhs=2, mode=mode, UR32=s.URg[1])
        assert rc == W.OK
        out[graph] = (x.clone(), [r['iters'] for r in st])
    assert out[0][1] == out[1][1]
    assert torch.equal(out[0][0], out[1][0])
