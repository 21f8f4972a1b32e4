"""Clover-improved operator (Sec. 6.1.2, and the exponential form of Sec. 6.1.3) against the
oracle: the diagonal blocks D_ee and D_oo^{-1} built on the device from the
fundamental links, the even-odd D-hat = D_ee - D_eo D_oo^{-1} D_oe and its
adjoint, and the CG on D-hat^+ D-hat in FP64 and mixed precision."""
import numpy as np
import pytest
import torch

from gpu_common import APBC, TOL, Setup, log, rel, wdirac
from oracle import clover as CL
from oracle import lattice as L
from oracle.reductions import norm2

pytestmark = pytest.mark.gpu

PAIRS = [(2, 'FUND'), (3, 'FUND'), (3, 'SYM'), (2, 'ADJ'), (4, '2AS'), (4, 'FUND')]
DIMS = (4, 6, 4, 6)


@pytest.fixture(scope='module')
def W():
    assert torch.cuda.is_available()
    return wdirac()


def clover_gpu(s, m, csw, expo, prec):
    c = s.lat.new_clover(prec)
    s.lat.clover_field(c, s.Ug, m, csw, expo, prec)
    return c


@pytest.mark.parametrize('N,rep', PAIRS)
def test_clover_blocks(W, N, rep):
    s = Setup(N, rep, DIMS, seed=600 + N, links='expH', eps=0.5, precs=(0,))
    m, csw = -0.3, 1.7
    psi = s.spinor(601)
    for expo in (0, 1):
        M = CL.diagonal_blocks(s.UR, m, csw, bool(expo))
        Me, Mo = CL.half_blocks(M, DIMS, 0), CL.half_blocks(M, DIMS, 1)
        exp_e = CL.apply_sitewise(Me, s.half(psi, 0)[0])
        exp_o = CL.apply_sitewise(np.linalg.inv(Mo), s.half(psi, 1)[0])
        for prec in (0, 1):
            c = clover_gpu(s, m, csw, expo, prec)
            for parity, exp in ((0, exp_e), (1, exp_o)):
                inp = s.to_gpu_half(psi, parity, prec)
                out = s.lat.new_half(1, prec)
                s.lat.apply_clover(out, inp, c, parity, 1, prec)
                got = s.from_gpu_half(out, parity, 1, prec)[0]
                err = rel(got, exp)
                log(f'  N={N} {rep} expo={expo} prec={prec} parity={parity}: {err:.2e}')
                assert err < TOL[prec], (expo, prec, parity)
                # in place
                s.lat.apply_clover(inp, inp, c, parity, 1, prec)
                assert rel(s.from_gpu_half(inp, parity, 1, prec)[0], exp) < TOL[prec]


@pytest.mark.parametrize('N,rep', PAIRS)
def test_dhat_clover(W, N, rep):
    s = Setup(N, rep, DIMS, seed=610 + N, links='expH', eps=0.5)
    m, csw = 0.1, 1.3
    psi = s.spinor(611)
    x_e = s.half(psi, 0)[0]
    for expo in (0, 1):
        for dagger in (0, 1):
            exp = CL.Dhat_clover(x_e, s.UR, m, csw, APBC, DIMS, bool(expo), dagger=bool(dagger))
            for prec in (0, 1):
                c = clover_gpu(s, m, csw, expo, prec)
                out = s.lat.new_half(1, prec)
                s.lat.apply_dhat_clover(out, s.to_gpu_half(psi, 0, prec), s.URg[prec], c, dagger, 1, prec)
                err = rel(s.from_gpu_half(out, 0, 1, prec)[0], exp)
                log(f'  N={N} {rep} expo={expo} dagger={dagger} prec={prec}: {err:.2e}')
                assert err < TOL[prec]


@pytest.mark.parametrize('N,rep,m,csw,expo', [(3, 'FUND', -0.2, 1.5, 0), (2, 'ADJ', -0.6, 1.2, 1),
                                              (3, 'SYM', -0.1, 1.0, 0)])
def test_cg_clover(W, N, rep, m, csw, expo):
    s = Setup(N, rep, DIMS, seed=620 + N, links='expH')
    psi = s.spinor(621, 2)
    b = s.half(psi, 0)
    c64, c32 = clover_gpu(s, m, csw, expo, 0), clover_gpu(s, m, csw, expo, 1)
    for mode in (W.CG_F64, W.CG_MIXED):
        x = s.lat.new_half(2)
        rc, st = s.lat.cg_eo_clover(x, s.to_gpu_half(psi, 0), s.URg[0], c64, tol=1e-10, maxit=5000, nrhs=2,
                                    mode=mode, UR32=s.URg[1], clov32=c32)
        assert rc == W.OK, st
        xs = s.from_gpu_half(x, 0, 2)
        for k in range(2):
            r = b[k] - CL.normal_op_clover(xs[k], s.UR, m, csw, APBC, DIMS, bool(expo))
            res = np.sqrt(norm2(r) / norm2(b[k]))
            log(f'  mode {mode} rhs {k}: iters {st[k]["iters"]}, oracle residual {res:.2e} '
                f'(reported {st[k]["true_rel_resid"]:.2e})')
            assert res <= 1.05e-10


def test_clover_zero_csw_is_plain_operator(W):
    """csw = 0: D-hat_clover = D-hat / (4 + m) exactly (up to rounding)."""
    s = Setup(3, 'SYM', DIMS, seed=630, precs=(0,))
    m = -0.25
    psi = s.spinor(631)
    c = clover_gpu(s, m, 0.0, 0, 0)
    inp = s.to_gpu_half(psi, 0)
    a, b = s.lat.new_half(), s.lat.new_half()
    s.lat.apply_dhat_clover(a, inp, s.URg[0], c, 0)
    s.lat.apply_dhat(b, inp, s.URg[0], m)
    ga, gb = s.from_gpu_half(a, 0)[0], s.from_gpu_half(b, 0)[0]
    assert rel(ga * (4.0 + m), gb) < 1e-14
