"""Clover force on the GPU against the oracle: the pseudofermion force with the
clover D-hat (regular clover of Sec. 6.1.2 and the exponential form of
Sec. 6.1.3, hopping part plus the clover-leaf part), the force of the odd-block
determinant term and its action, on every link of lattices with ragged tile
tails, in both output forms (P and the gradient 2i P U) and with
accumulation; a three-lattice batch."""
import numpy as np
import pytest
import torch

from gpu_common import APBC, TOL, Setup, log, rel, wdirac
from oracle import clover_force as CF
from oracle import lattice as L
from paper_2503_06721_amd import synth

pytestmark = pytest.mark.gpu

DIMS = (4, 6, 4, 6)
CASES = [(3, 'FUND', 0.1, 1.7, 0), (2, 'ADJ', -0.2, 1.3, 1), (3, 'SYM', 0.3, 1.1, 0), (4, '2AS', 0.2, 1.2, 1),
         (2, 'FUND', 0.0, 2.0, 1), (4, 'FUND', -0.1, 1.5, 0), (2, 'SYM', 0.1, 1.4, 1), (3, '2AS', 0.2, 1.6, 0)]


@pytest.fixture(scope='module')
def W():
    assert torch.cuda.is_available()
    return wdirac()


def components_to_P(g, N):
    from oracle import reps as R
    return R.algebra_to_matrix(g, N)


@pytest.mark.parametrize('N,rep,m,csw,expo', CASES)
def test_force_eo_clover(W, N, rep, m, csw, expo):
    s = Setup(N, rep, DIMS, seed=960 + N, links='expH', eps=0.5, precs=(0,))
    x_e = s.half(s.spinor(961), 0)[0]
    exp = components_to_P(CF.pseudofermion_force_components(x_e, s.U, rep, m, csw, APBC, DIMS, bool(expo)), N)
    clov = s.lat.new_clover(0)
    s.lat.clover_field(clov, s.Ug, m, csw, expo, 0)
    xg = s.to_gpu_half(L.from_half(x_e, DIMS, 0)[None], 0)
    P = torch.zeros(DIMS + (4, N, N), dtype=torch.complex128, device='cuda')
    s.lat.force_eo_clover(P, xg, s.URg[0], s.Ug, clov, m, csw, expo)
    err = rel(P.cpu().numpy(), exp)
    log(f'  N={N} {rep} expo={expo}: force error {err:.2e}')
    assert err < TOL[0]
    s.lat.force_eo_clover(P, xg, s.URg[0], s.Ug, clov, m, csw, expo, scale=-0.5, accumulate=1)
    assert rel(P.cpu().numpy(), 0.5 * exp) < TOL[0]
    G = torch.zeros_like(P)
    s.lat.force_eo_clover(G, xg, s.URg[0], s.Ug, clov, m, csw, expo, gradient=1)
    assert rel(G.cpu().numpy(), 2j * np.einsum('...ij,...jk->...ik', exp, s.U)) < TOL[0]


@pytest.mark.parametrize('N,rep,m,csw,expo', [c for c in CASES if c[4] == 0][:3] + [(2, 'ADJ', -0.2, 1.3, 1)])
def test_clover_logdet_and_force(W, N, rep, m, csw, expo):
    s = Setup(N, rep, DIMS, seed=970 + N, links='expH', eps=0.5, precs=(0,))
    clov = s.lat.new_clover(0)
    s.lat.clover_field(clov, s.Ug, m, csw, expo, 0)
    ld = s.lat.clover_logdet(clov)
    ld_or = CF.logdet_odd(s.U, rep, m, csw, DIMS, bool(expo))
    log(f'  N={N} {rep} expo={expo}: logdet {ld:.12f} (oracle {ld_or:.12f})')
    assert abs(ld - ld_or) <= 1e-12 * abs(ld_or)
    exp = components_to_P(CF.det_force_components(s.U, rep, m, csw, DIMS, bool(expo)), N)
    P = torch.zeros(DIMS + (4, N, N), dtype=torch.complex128, device='cuda')
    s.lat.force_clover_logdet(P, s.Ug, clov, m, csw, expo)
    got = P.cpu().numpy()
    if expo:
        # constant determinant: the force vanishes up to rounding
        assert np.abs(got).max() < 1e-12
    else:
        err = rel(got, exp)
        log(f'  det force error {err:.2e}')
        assert err < TOL[0]


def test_clover_force_batch(W):
    """Three lattices of different shapes in one context: every lattice's
    force equals its own oracle force."""
    from test_gpu_batch import Batch
    shapes = [(4, 4, 4, 4), (6, 4, 2, 4), (2, 4, 6, 2)]
    b = Batch(W, 3, 'FUND', shapes, seed=980, precs=(0,))
    m, csw = 0.05, 1.5
    xs = [L.to_half(f, dd, 0) for f, dd in zip(b.spinors(981), b.shapes)]
    clov = b.lat.new_clover(0)
    b.lat.clover_field(clov, b.Ug, m, csw, 0, 0)
    vt = sum(int(np.prod(dd)) for dd in b.shapes)
    P = torch.zeros((vt, 4, 3, 3), dtype=torch.complex128, device='cuda')
    b.lat.force_eo_clover(P, b.to_gpu(b.embed_even(xs), 0), b.URg[0], b.Ug, clov, m, csw, 0)
    b.lat.force_clover_logdet(P, b.Ug, clov, m, csw, 0, accumulate=1)
    lds = b.lat.clover_logdet(clov)
    got, o = P.cpu().numpy(), 0
    for k, dd in enumerate(b.shapes):
        v = int(np.prod(dd))
        g = (CF.pseudofermion_force_components(xs[k], b.U[k], 'FUND', m, csw, APBC, dd)
             + CF.det_force_components(b.U[k], 'FUND', m, csw, dd))
        exp = components_to_P(g, 3)
        assert rel(got[o:o + v].reshape(exp.shape), exp) < TOL[0], k
        assert abs(lds[k] - CF.logdet_odd(b.U[k], 'FUND', m, csw, dd)) <= 1e-12 * abs(lds[k])
        o += v


@pytest.mark.parametrize('dims', [(2, 6, 2, 2), (4, 2, 6, 2), (6, 2, 2, 6)])
@pytest.mark.parametrize('N,rep,m,csw,expo', [(3, 'FUND', 0.1, 1.7, 0), (2, 'ADJ', -0.2, 1.3, 1)])
def test_clover_force_ragged_volume(W, dims, N, rep, m, csw, expo):
    """Volumes that are not a multiple of the 64-site chunks the clover field,
    leaf and gather kernels assign to one wavefront per plane or direction:
    the clover field (through log det D_oo), the pseudofermion force and the
    determinant force on every link."""
    s = Setup(N, rep, dims, seed=990 + N, links='expH', eps=0.5, precs=(0,))
    x_e = s.half(s.spinor(991), 0)[0]
    clov = s.lat.new_clover(0)
    s.lat.clover_field(clov, s.Ug, m, csw, expo, 0)
    ld, ld_or = s.lat.clover_logdet(clov), CF.logdet_odd(s.U, rep, m, csw, dims, bool(expo))
    assert abs(ld - ld_or) <= 1e-12 * max(abs(ld_or), 1.0), (ld, ld_or)
    xg = s.to_gpu_half(L.from_half(x_e, dims, 0)[None], 0)
    P = torch.zeros(tuple(dims) + (4, N, N), dtype=torch.complex128, device='cuda')
    s.lat.force_eo_clover(P, xg, s.URg[0], s.Ug, clov, m, csw, expo)
    s.lat.force_clover_logdet(P, s.Ug, clov, m, csw, expo, accumulate=1)
    g = (CF.pseudofermion_force_components(x_e, s.U, rep, m, csw, APBC, dims, bool(expo))
         + CF.det_force_components(s.U, rep, m, csw, dims, bool(expo)))
    err = rel(P.cpu().numpy(), components_to_P(g, N))
    log(f'  {dims} N={N} {rep} expo={expo}: force error {err:.2e}')
    assert err < TOL[0]
