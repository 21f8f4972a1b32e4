"""HMC molecular dynamics (Sec. 5.2, 5.3) on the GPU against the oracle: gauge
action, gauge force, link update, kinetic term, momentum construction; a
whole Omelyan trajectory with fermions against the oracle's trajectory from
the same inputs; and, on an 8^4 lattice, reversibility and the O(eps^2)
energy-error scaling of both integrators (the paper's table of integrators);
the same with a clover term (regular and exponential), against the oracle's
clover trajectory and, on 8^4, in its energy-error scaling; and the
algorithmic tests of Sec. 8 (Creutz equality, acceptance rate) on a
thermalised SU(2) adjoint ensemble."""
import numpy as np
import pytest
import torch

from gpu_common import APBC, log, rel, wdirac
from oracle import clover as CL
from oracle import dirac as D
from oracle import hmc as OH
from oracle import lattice as L
from oracle import reps as R
from paper_2503_06721_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope='module')
def W():
    assert torch.cuda.is_available()
    return wdirac()


def components(dims, N, seed):
    return np.random.default_rng(seed).normal(size=tuple(dims) + (4, N * N - 1))


@pytest.mark.parametrize('N', [2, 3, 4])
def test_gauge_pieces(W, N):
    dims = (4, 6, 4, 2)
    U = synth.expH_links(dims, N, 0.5, 800 + N)
    lat = W.Lattice(N, 'FUND', dims, APBC)
    Ug = torch.from_numpy(U).cuda()
    beta = 2.7
    S = lat.gauge_action(Ug, beta)
    assert abs(S - OH.gauge_action(U, beta)) <= 1e-12 * abs(S)
    Fg = torch.zeros_like(Ug)
    lat.gauge_force(Fg, Ug, beta, scale=0.5)
    lat.gauge_force(Fg, Ug, beta, scale=0.5, accumulate=1)
    assert rel(Fg.cpu().numpy(), OH.gauge_force(U, beta)) < 1e-13
    w = components(dims, N, 801)
    pi = torch.empty_like(Ug)
    lat.algebra_from_components(pi, torch.from_numpy(w).cuda())
    pi_or = R.algebra_to_matrix(w, N)
    assert rel(pi.cpu().numpy(), pi_or) < 1e-15
    K = lat.kinetic(pi)
    assert abs(K - OH.kinetic(pi_or)) <= 1e-12 * K
    U2 = Ug.clone()
    lat.link_update(U2, pi, 0.37)
    exp = OH.exp_i(0.37 * pi_or) @ U
    err = rel(U2.cpu().numpy(), exp)
    log(f'  N={N}: link update error {err:.2e}')
    assert err < 1e-14


def test_trajectory_matches_oracle(W):
    from paper_2503_06721_amd.hmc import HMC
    dims, N, rep, beta, m = (4, 4, 2, 2), 2, 'ADJ', 2.0, 0.2
    U = synth.expH_links(dims, N, 0.4, 810)
    UR = R.represent(U, rep)
    d = UR.shape[-1]
    eta = synth.gaussian_spinor((int(np.prod(dims)) // 2, 4, d), 811)
    w = components(dims, N, 812)
    # oracle
    phi_or = D.Dhat_dag(eta, UR, m, APBC, dims)
    act = OH.Action(beta, m, rep, APBC, phi_or, tol=1e-14)
    U1_or, pi1_or, H0_or, H1_or = OH.trajectory(U, R.algebra_to_matrix(w, N), act, 0.1, 4, 'omelyan2')
    # GPU
    lat = W.Lattice(N, rep, dims, APBC)
    hmc = HMC(lat, beta, m, tol=1e-13)
    Ug = torch.from_numpy(U).cuda()
    eta_g = lat.pack_half(torch.from_numpy(L.from_half(eta, dims, 0)[None]).cuda(), 0)
    pi, phi = hmc.refresh(Ug, torch.from_numpy(w).cuda(), eta_g)
    H0, H1 = hmc.trajectory(Ug, pi, phi, 0.1, 4, 'omelyan2')
    errU = rel(Ug.cpu().numpy(), U1_or)
    errP = rel(pi.cpu().numpy(), pi1_or)
    log(f'  H0 {H0:.10f} (oracle {H0_or:.10f}); dH {H1 - H0:.3e} (oracle {H1_or - H0_or:.3e}); '
        f'U error {errU:.2e}, pi error {errP:.2e}')
    assert abs(H0 - H0_or) <= 1e-11 * abs(H0_or)
    assert abs((H1 - H0) - (H1_or - H0_or)) <= 1e-8
    assert errU < 1e-10 and errP < 1e-9


@pytest.mark.parametrize('expo', [0, 1])
def test_clover_trajectory_matches_oracle(W, expo):
    from paper_2503_06721_amd.hmc import HMC
    dims, N, rep, beta, m, csw = (4, 2, 2, 4), 2, 'FUND', 2.0, 0.2, 1.8
    U = synth.expH_links(dims, N, 0.4, 840 + expo)
    UR = R.represent(U, rep)
    eta = synth.gaussian_spinor((int(np.prod(dims)) // 2, 4, 2), 842)
    w = components(dims, N, 843)
    phi_or = CL.Dhat_clover(eta, UR, m, csw, APBC, dims, bool(expo), dagger=True)
    act = OH.Action(beta, m, rep, APBC, phi_or, tol=1e-14, csw=csw, exponential=bool(expo))
    U1_or, pi1_or, H0_or, H1_or = OH.trajectory(U, R.algebra_to_matrix(w, N), act, 0.1, 3, 'omelyan2')
    lat = W.Lattice(N, rep, dims, APBC)
    hmc = HMC(lat, beta, m, tol=1e-13, csw=csw, exponential=expo)
    Ug = torch.from_numpy(U).cuda()
    eta_g = lat.pack_half(torch.from_numpy(L.from_half(eta, dims, 0)[None]).cuda(), 0)
    pi, phi = hmc.refresh(Ug, torch.from_numpy(w).cuda(), eta_g)
    H0, H1 = hmc.trajectory(Ug, pi, phi, 0.1, 3, 'omelyan2')
    errU = rel(Ug.cpu().numpy(), U1_or)
    errP = rel(pi.cpu().numpy(), pi1_or)
    log(f'  expo={expo}: H0 {H0:.10f} (oracle {H0_or:.10f}); dH {H1 - H0:.3e} (oracle {H1_or - H0_or:.3e}); '
        f'U error {errU:.2e}, pi error {errP:.2e}')
    assert abs(H0 - H0_or) <= 1e-11 * abs(H0_or)
    assert abs((H1 - H0) - (H1_or - H0_or)) <= 1e-8
    assert errU < 1e-10 and errP < 1e-9


def hmc_setup(W, seed, N=3, rep='FUND', dims=(8, 8, 8, 8), beta=5.6, m=0.1, csw=None, expo=0):
    from paper_2503_06721_amd.hmc import HMC
    lat = W.Lattice(N, rep, dims, APBC)
    hmc = HMC(lat, beta, m, tol=1e-12, csw=csw, exponential=expo)
    Ug = torch.from_numpy(synth.expH_links(dims, N, 0.3, seed)).cuda()
    g = torch.Generator(device='cuda')
    g.manual_seed(seed)
    w = torch.randn(tuple(dims) + (4, N * N - 1), dtype=torch.float64, device='cuda', generator=g)
    eta = torch.randn((1,) + tuple(dims) + (4, lat.d), dtype=torch.complex128, device='cuda', generator=g)
    pi, phi = hmc.refresh(Ug, w, lat.pack_half(eta, 0))
    return hmc, Ug, pi, phi


def test_reversibility_8x8x8x8(W):
    hmc, U, pi, phi = hmc_setup(W, 820)
    U0, pi0 = U.clone(), pi.clone()
    H0, H1 = hmc.trajectory(U, pi, phi, 0.05, 10, 'omelyan2')
    pi.neg_()
    H2, H3 = hmc.trajectory(U, pi, phi, 0.05, 10, 'omelyan2')
    dU = (torch.linalg.vector_norm(U - U0) / torch.linalg.vector_norm(U0)).item()
    dpi = (torch.linalg.vector_norm(pi + pi0) / torch.linalg.vector_norm(pi0)).item()
    log(f'  dH forward {H1 - H0:.3e}; back to start: |dU| {dU:.2e}, |dpi| {dpi:.2e}, H {H3 - H0:.2e}')
    assert dU < 1e-10 and dpi < 1e-9 and abs(H3 - H0) < 1e-7


@pytest.mark.parametrize('integrator', ['leapfrog', 'omelyan2'])
def test_energy_error_scaling_8x8x8x8(W, integrator):
    dH = []
    for n in (5, 10, 20):
        hmc, U, pi, phi = hmc_setup(W, 830)
        H0, H1 = hmc.trajectory(U, pi, phi, 0.5 / n, n, integrator)
        dH.append(abs(H1 - H0))
    log(f'  {integrator}: |dH| {dH}')
    assert 3.3 < dH[0] / dH[1] < 4.8 and 3.6 < dH[1] / dH[2] < 4.4


@pytest.mark.parametrize('expo', [0, 1])
def test_clover_energy_error_scaling_8x8x8x8(W, expo):
    """Omelyan with the clover force and (regular form) the determinant force:
    |dH| ~ eps^2 only if both are the exact gradients of their actions."""
    dH = []
    for n in (5, 10, 20):
        hmc, U, pi, phi = hmc_setup(W, 850, m=0.2, csw=1.5, expo=expo)
        H0, H1 = hmc.trajectory(U, pi, phi, 0.5 / n, n, 'omelyan2')
        dH.append(abs(H1 - H0))
    log(f'  clover expo={expo}: |dH| {dH}')
    assert 3.3 < dH[0] / dH[1] < 4.8 and 3.6 < dH[1] / dH[2] < 4.4


def test_creutz_equality_and_acceptance(W):
    """The algorithmic tests of Sec. 8 on SU(2) with two adjoint flavours
    (4^4, beta = 2.2): after thermalisation, the Creutz equality
    <exp(-dH)> = 1, a positive <dH>, and the acceptance rate against
    erfc(sqrt(<dH^2>/8)), each within four standard errors."""
    from paper_2503_06721_amd.hmc import HMC
    dims, N, rep = (4, 4, 4, 4), 2, 'ADJ'
    lat = W.Lattice(N, rep, dims, APBC)
    hmc = HMC(lat, 2.2, -0.5, tol=1e-12)
    U = torch.from_numpy(synth.expH_links(dims, N, 0.3, 860)).cuda()
    g = torch.Generator(device='cuda')
    g.manual_seed(861)
    # step size for an acceptance near 85%: dH is large enough for the tests
    # to bite, and exp(-dH) has no heavy tail that a finite sample misses
    for _ in range(60):
        hmc.update(U, 0.25, 4, g)
    dH, acc = [], []
    for _ in range(300):
        d, a = hmc.update(U, 0.25, 4, g)
        dH.append(d)
        acc.append(a)
    dH = np.array(dH)
    n = len(dH)
    e = np.exp(-dH)
    creutz, se = e.mean(), e.std(ddof=1) / np.sqrt(n)
    p_obs = float(np.mean(acc))
    from scipy.special import erfc
    p_exp = float(erfc(np.sqrt(np.mean(dH ** 2) / 8.0)))
    sp = np.sqrt(p_exp * (1 - p_exp) / n)
    log(f'  <exp(-dH)> = {creutz:.4f} +- {se:.4f}; <dH> = {dH.mean():.4f} +- {dH.std(ddof=1) / np.sqrt(n):.4f}; '
        f'acceptance {p_obs:.3f} (erfc prediction {p_exp:.3f} +- {sp:.3f}); CG iterations {hmc.cg_iters}')
    assert 0.6 < p_obs < 0.97, 'step size outside the range the test is meant for'
    assert abs(creutz - 1.0) < 4 * se
    assert dH.mean() > -4 * dH.std(ddof=1) / np.sqrt(n)
    assert abs(p_obs - p_exp) < 4 * sp + 1.0 / n
