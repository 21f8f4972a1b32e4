"""Batches of lattices of different shapes processed in one launch per kernel,
checked lattice by lattice against the oracle: represented links, hops in
both parities and their adjoints (both kernel forms, FP64 and FP32), norms
and inner products, CG (FP64 and mixed) and the force.  Includes the SU(3)
SYM batch of 8^4, 12^4 and 16^3x32 lattices."""
import numpy as np
import pytest
import torch

from gpu_common import TOL, log, rel, wdirac
from oracle import cg as OCG
from oracle import dirac as D
from oracle import force as OF
from oracle import lattice as L
from oracle import reps as R
from oracle.reductions import inner, norm2
from paper_2503_06721_amd import synth

pytestmark = pytest.mark.gpu
APBC = (-1, 1, 1, 1)


class Batch:
    def __init__(self, W, N, rep, shapes, seed, precs=(0, 1)):
        self.W, self.N, self.rep, self.shapes = W, N, rep, [tuple(s) for s in shapes]
        self.U = [synth.expH_links(dd, N, 0.3, seed + k) for k, dd in enumerate(self.shapes)]
        self.UR = [R.represent(U, rep) for U in self.U]
        self.d = self.UR[0].shape[-1]
        self.lat = W.Lattice(N, rep, self.shapes, APBC)
        self.Ug = torch.cat([torch.from_numpy(U.reshape(-1, 4, N, N)) for U in self.U]).cuda()
        self.URg = {}
        for p in precs:
            self.URg[p] = self.lat.new_links(p)
            self.lat.rep_links(self.URg[p], self.Ug, p)

    def spinors(self, seed):
        return [synth.gaussian_spinor(dd + (4, self.d), seed + k) for k, dd in enumerate(self.shapes)]

    def to_gpu(self, fields, parity, prec=0):
        dt = np.complex128 if prec == 0 else np.complex64
        flat = np.concatenate([f.reshape(-1, 4, self.d) for f in fields]).astype(dt)
        return self.lat.pack_half(torch.from_numpy(flat).cuda(), parity, 1, prec)

    def from_gpu(self, packed, parity, prec=0):
        flat = self.lat.unpack_half(packed, parity, 1, prec).cpu().numpy().astype(np.complex128)
        out, o = [], 0
        for dd in self.shapes:
            v = int(np.prod(dd))
            out.append(L.to_half(flat[o:o + v].reshape(dd + (4, self.d)), dd, parity))
            o += v
        return out

    def embed_even(self, halves):
        return [L.from_half(h, dd, 0) for h, dd in zip(halves, self.shapes)]


@pytest.fixture(scope='module')
def W():
    assert torch.cuda.is_available()
    return wdirac()


SHAPES = [(4, 6, 4, 6), (2, 2, 2, 2), (4, 4, 2, 4)]


@pytest.mark.parametrize('N,rep', [(3, 'SYM'), (2, 'FUND'), (2, 'ADJ')])
def test_batch_links_and_hops(W, N, rep):
    b = Batch(W, N, rep, SHAPES, seed=900)
    for prec in (0, 1):
        got = b.lat.links_canonical(b.URg[prec], prec).cpu().numpy()
        o = 0
        for k, dd in enumerate(b.shapes):
            v = int(np.prod(dd))
            exp = D.links_with_boundary_phase(b.UR[k], APBC)
            assert rel(got[o:o + v].reshape(exp.shape), exp) < TOL[prec]
            o += v
    psi = b.spinors(901)
    for variant in (W.HOP_COLOUR, W.HOP_COLOUR_PAIR, W.HOP_SITE) + (
            (W.HOP_COMPACT, W.HOP_COMPACT_PAIR) if b.lat.compact else ()) + (
            (W.HOP_COLOUR_QUAD,) if b.lat.d <= 6 else ()):
        for prec in (0, 1):
            b.lat.set_option(W.OPT_HOP_VARIANT_F64 if prec == 0 else W.OPT_HOP_VARIANT_F32, variant)
            for p, dagger in ((0, 0), (1, 1), (0, 1)):
                log(f'batch hop N={N} rep={rep} variant={variant} prec={prec} p={p} dag={dagger}')
                out = b.lat.new_half(1, prec)
                b.lat.dslash_eo(out, b.to_gpu(psi, 1 - p, prec), b.URg[prec], p, dagger, 1, 0.0, None, 1.0, prec)
                got = b.from_gpu(out, p, prec)
                for k, dd in enumerate(b.shapes):
                    exp = D.hop_block(L.to_half(psi[k], dd, 1 - p), b.UR[k], APBC, dd, p, dagger=bool(dagger))
                    assert rel(got[k], exp) < TOL[prec], (variant, prec, p, dagger, k)


def test_batch_norm_dot(W):
    b = Batch(W, 3, 'FUND', SHAPES, seed=910, precs=(0,))
    x, y = b.spinors(911), b.spinors(912)
    gx, gy = b.to_gpu(x, 0), b.to_gpu(y, 0)
    n = b.lat.norm2(gx)
    dt = b.lat.dot(gx, gy)
    assert len(n) == len(SHAPES) and len(dt) == len(SHAPES)
    for k, dd in enumerate(b.shapes):
        hx, hy = L.to_half(x[k], dd, 0), L.to_half(y[k], dd, 0)
        assert abs(n[k] - norm2(hx)) <= 1e-14 * norm2(hx)
        assert abs(dt[k] - inner(hx, hy)) <= 1e-14 * abs(inner(hx, hy))


@pytest.mark.parametrize('N,rep,m', [(3, 'FUND', -0.2), (2, 'ADJ', -0.6)])
def test_batch_cg(W, N, rep, m):
    b = Batch(W, N, rep, SHAPES, seed=920)
    eta = b.spinors(921)
    rhs = [D.Dhat_dag(D.eo_source(e, UR, m, APBC, dd), UR, m, APBC, dd)
           for e, UR, dd in zip(eta, b.UR, b.shapes)]
    for mode in (W.CG_F64, W.CG_MIXED):
        x = b.lat.new_half()
        rc, st = b.lat.cg_eo(x, b.to_gpu(b.embed_even(rhs), 0), b.URg[0], m, tol=1e-10, maxit=10000, mode=mode,
                             UR32=b.URg[1])
        assert rc == W.OK, st
        assert len(st) == len(SHAPES)
        xs = b.from_gpu(x, 0)
        for k, dd in enumerate(b.shapes):
            r = rhs[k] - D.normal_op(xs[k], b.UR[k], m, APBC, dd)
            res = np.sqrt(norm2(r) / norm2(rhs[k]))
            log(f'  batch cg mode {mode} lattice {dd}: iters {st[k]["iters"]} residual {res:.2e}')
            assert res <= 1.05e-10
            if mode == W.CG_F64:
                _, it_or, _ = OCG.cg(lambda v: D.normal_op(v, b.UR[k], m, APBC, dd), rhs[k], 1e-10, 10000)
                assert abs(st[k]['iters'] - it_or) <= 2


def test_batch_force(W):
    b = Batch(W, 3, 'SYM', SHAPES, seed=930, precs=(0,))
    m = 0.1
    xs = [L.to_half(f, dd, 0) for f, dd in zip(b.spinors(931), b.shapes)]
    P = torch.zeros((sum(int(np.prod(dd)) for dd in b.shapes), 4, 3, 3), dtype=torch.complex128, device='cuda')
    b.lat.force_eo(P, b.to_gpu(b.embed_even(xs), 0), b.URg[0], m)
    got, o = P.cpu().numpy(), 0
    for k, dd in enumerate(b.shapes):
        v = int(np.prod(dd))
        exp = OF.force(xs[k], b.UR[k], m, APBC, dd, 3, 'SYM')
        assert rel(got[o:o + v].reshape(exp.shape), exp) < TOL[0]
        o += v


def test_su3_sym_batch_8_12_16x32(W):
    """SU(3) SYM, lattices 8^4, 12^4 and 16^3x32 in one launch, FP64 and FP32,
    against the oracle on every site; batched CG against separate solves."""
    shapes = [(8, 8, 8, 8), (12, 12, 12, 12), (32, 16, 16, 16)]
    b = Batch(W, 3, 'SYM', shapes, seed=940)
    psi = b.spinors(941)
    for prec in (0, 1):
        b.lat.autotune(b.URg[prec], prec, 1)
        out = b.lat.new_half(1, prec)
        b.lat.dslash_eo(out, b.to_gpu(psi, 1, prec), b.URg[prec], 0, 0, 1, 0.0, None, 1.0, prec)
        got = b.from_gpu(out, 0, prec)
        for k, dd in enumerate(shapes):
            exp = D.hop_block(L.to_half(psi[k], dd, 1), b.UR[k], APBC, dd, 0)
            err = rel(got[k], exp)
            log(f'  {dd} prec {prec}: relative error {err:.2e}')
            assert err < TOL[prec]
    m = -0.4
    eta = [L.to_half(f, dd, 0) for f, dd in zip(b.spinors(942), shapes)]
    bb = b.to_gpu(b.embed_even(eta), 0)
    x = b.lat.new_half()
    rc, st = b.lat.cg_eo(x, bb, b.URg[0], m, tol=1e-10, maxit=20000)
    assert rc == W.OK
    t_batch = st[0]['seconds']
    t_sep = 0.0
    for k, dd in enumerate(shapes):
        lat1 = W.Lattice(3, 'SYM', dd, APBC)
        UR1 = lat1.new_links(0)
        lat1.rep_links(UR1, torch.from_numpy(b.U[k]).cuda())
        x1 = lat1.new_half()
        b1 = lat1.pack_half(torch.from_numpy(L.from_half(eta[k], dd, 0)[None]).cuda(), 0)
        rc1, st1 = lat1.cg_eo(x1, b1, UR1, m, tol=1e-10, maxit=20000)
        assert rc1 == W.OK and abs(st1[0]['iters'] - st[k]['iters']) <= 2
        t_sep += st1[0]['seconds']
        log(f'  {dd}: batched {st[k]["iters"]} it, separate {st1[0]["iters"]} it')
    log(f'  batched CG {t_batch:.4f} s vs three separate solves {t_sep:.4f} s')
