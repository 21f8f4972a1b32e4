"""Pins of the oracle's Wilson-Dirac operator, even-odd blocks and CG against
closed forms, invariants and brute force (no GPU)."""
import itertools
import math

import numpy as np
import pytest

from oracle import cg as CG
from oracle import dense
from oracle import dirac as D
from oracle import lattice as L
from oracle import reps as R
from oracle.gamma import GAMMA, GAMMA5
from oracle.reductions import inner
from paper_2503_06721_amd import synth

APBC = (-1, 1, 1, 1)
PBC = (1, 1, 1, 1)


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def momenta(dims, bc):
    axes = []
    for mu in range(4):
        n = np.arange(dims[mu])
        axes.append((2 * n + (1 if bc[mu] == -1 else 0)) * np.pi / dims[mu])
    return axes


def plane_wave(dims, p, u):
    c = L.coordinates(dims)
    phase = np.exp(1j * (c @ np.asarray(p))).reshape(tuple(dims))
    return phase[..., None, None] * u


def free_symbol(p, m):
    """m + sum_mu (1 - cos p_mu) + i sum_mu gamma_mu sin p_mu  (4x4)."""
    return (m + sum(1 - math.cos(q) for q in p)) * np.eye(4) + 1j * sum(
        GAMMA[mu] * math.sin(p[mu]) for mu in range(4))


# ----------------------------------------------------------------- free field
@pytest.mark.parametrize('bc', [APBC, PBC, (1, -1, 1, -1)])
@pytest.mark.parametrize('N,rep', [(2, 'FUND'), (3, 'SYM'), (2, 'ADJ')])
def test_free_field_plane_waves(bc, N, rep):
    dims = (4, 2, 6, 4)
    m = -0.37
    UR = R.represent(synth.unit_links(dims, N), rep)
    d = UR.shape[-1]
    rng = np.random.default_rng(1)
    ks = momenta(dims, bc)
    for _ in range(6):
        p = [ks[mu][rng.integers(dims[mu])] for mu in range(4)]
        u = rng.normal(size=(4, d)) + 1j * rng.normal(size=(4, d))
        psi = plane_wave(dims, p, u)
        expect = plane_wave(dims, p, free_symbol(p, m) @ u)
        assert rel(D.dirac(psi, UR, m, bc), expect) < 1e-14


def test_free_field_spectrum_dense():
    dims = (2, 2, 2, 2)
    m = 0.13
    UR = R.represent(synth.unit_links(dims, 2), 'FUND')
    shape = dims + (4, 2)
    M = dense.dense_matrix(lambda v: D.dirac(v, UR, m, APBC), shape)
    ev = np.linalg.eigvals(M)
    expect = []
    for p in itertools.product(*momenta(dims, APBC)):
        s = math.sqrt(sum(math.sin(q) ** 2 for q in p))
        base = m + sum(1 - math.cos(q) for q in p)
        expect += [base + 1j * s] * 4 + [base - 1j * s] * 4
    key = lambda z: (round(z.real, 9), round(z.imag, 9))
    assert np.allclose(sorted(ev, key=key), sorted(expect, key=key), atol=1e-12)


def test_free_field_dhat_spectrum():
    dims = (4, 2, 2, 2)
    m = -0.21
    UR = R.represent(synth.unit_links(dims, 2), 'FUND')
    shape = (L.volume(dims) // 2, 4, 2)
    M = dense.dense_matrix(lambda v: D.Dhat(v, UR, m, APBC, dims), shape)
    ev = np.linalg.eigvals(M)
    expect = []
    for p in itertools.product(*momenta(dims, APBC)):
        s = math.sqrt(sum(math.sin(q) ** 2 for q in p))
        c = sum(math.cos(q) for q in p)
        for sg in (1, -1):
            lam_p = 4 + m - c + sg * 1j * s        # lambda_+-(p)
            lam_q = 4 + m + c - sg * 1j * s        # lambda_-+(p + pi-hat)
            expect += [lam_p * lam_q] * 2          # colour multiplicity d = 2
    key = lambda z: (round(z.real, 8), round(z.imag, 8))
    assert np.allclose(sorted(ev, key=key), sorted(expect, key=key), atol=1e-11)


# ------------------------------------------------------------- invariants
def random_setup(dims, N, rep, seed, haar=True):
    U = synth.haar_links(dims, N, seed) if haar else synth.expH_links(dims, N, 0.3, seed)
    UR = R.represent(U, rep)
    d = UR.shape[-1]
    return U, UR, d


@pytest.mark.parametrize('N,rep', [(2, 'FUND'), (2, 'ADJ'), (3, 'SYM'), (4, '2AS'), (3, 'FUND')])
def test_adjoint_and_gamma5_hermiticity(N, rep):
    dims = (4, 2, 2, 4)
    _, UR, d = random_setup(dims, N, rep, 3)
    psi = synth.gaussian_spinor(dims + (4, d), 4)
    chi = synth.gaussian_spinor(dims + (4, d), 5)
    Hpsi = D.hopping(psi, UR, APBC)
    Hdchi = D.hopping(chi, UR, APBC, dagger=True)
    a, b = inner(chi, Hpsi), inner(Hdchi, psi)
    assert abs(a - b) < 1e-13 * abs(a)
    # H^dagger = gamma_5 H gamma_5
    assert rel(Hdchi, D.gamma5(D.hopping(D.gamma5(chi), UR, APBC))) < 1e-14


@pytest.mark.parametrize('N,rep', [(2, 'FUND'), (2, 'ADJ'), (3, 'SYM'), (3, '2AS'), (4, 'FUND')])
def test_gauge_covariance(N, rep):
    dims = (2, 4, 2, 4)
    U, UR, d = random_setup(dims, N, rep, 8)
    g = synth.gauge_transform(dims, N, 9)
    Ug = np.empty_like(U)
    for mu in range(4):
        g_fwd = np.roll(g, -1, axis=mu)
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(g_fwd, -1, -2))
    Rg = R.represent(g, rep)
    psi = synth.gaussian_spinor(dims + (4, d), 10)
    lhs = D.dirac(np.einsum('...ab,...sb->...sa', Rg, psi), R.represent(Ug, rep), 0.1, APBC)
    rhs = np.einsum('...ab,...sb->...sa', Rg, D.dirac(psi, UR, 0.1, APBC))
    assert rel(lhs, rhs) < 1e-13


def test_bc_as_link_sign():
    """Antiperiodic fermion BC == periodic hopping on U_R with -1 on the
    links that cross the boundary (Sec. 6.3.1: one time slice of U_R negated)."""
    dims = (4, 2, 4, 2)
    _, UR, d = random_setup(dims, 3, 'FUND', 12)
    psi = synth.gaussian_spinor(dims + (4, d), 13)
    URs = UR.copy()
    URs[-1, :, :, :, 0] *= -1.0
    assert rel(D.hopping(psi, URs, PBC), D.hopping(psi, UR, APBC)) < 1e-15
    assert np.array_equal(D.links_with_boundary_phase(UR, APBC), URs)
    bc2 = (1, -1, 1, -1)
    assert rel(D.hopping(psi, D.links_with_boundary_phase(UR, bc2), PBC), D.hopping(psi, UR, bc2)) < 1e-15


@pytest.mark.parametrize('N,rep', [(2, 'FUND'), (2, 'ADJ')])
def test_det_identity(N, rep):
    dims = (2, 2, 2, 2)
    _, UR, d = random_setup(dims, N, rep, 21)
    m = -0.3
    full = dense.dense_matrix(lambda v: D.dirac(v, UR, m, APBC), dims + (4, d))
    hat = dense.dense_matrix(lambda v: D.Dhat(v, UR, m, APBC, dims), (8, 4, d))
    s1, l1 = np.linalg.slogdet(full)
    s2, l2 = np.linalg.slogdet(hat)
    assert abs(l1 - l2) < 1e-10 and abs(s1 - s2) < 1e-10


def test_eo_blocks_of_dense_matrix():
    dims = (2, 2, 2, 4)
    _, UR, d = random_setup(dims, 2, 'FUND', 22)
    H = dense.dense_matrix(lambda v: D.hopping(v, UR, APBC), dims + (4, d))
    n = 4 * d
    ev = L.parity_sites(dims, 0)
    od = L.parity_sites(dims, 1)
    rows = lambda sites: (sites[:, None] * n + np.arange(n)).ravel()
    Deo = dense.dense_matrix(lambda v: D.D_eo(v, UR, APBC, dims), (len(od), 4, d))
    Doe = dense.dense_matrix(lambda v: D.D_oe(v, UR, APBC, dims), (len(ev), 4, d))
    assert np.array_equal(Deo, H[np.ix_(rows(ev), rows(od))])
    assert np.array_equal(Doe, H[np.ix_(rows(od), rows(ev))])
    assert np.abs(H[np.ix_(rows(ev), rows(ev))]).max() == 0.0


def test_dhat_dagger_is_adjoint():
    dims = (4, 2, 2, 2)
    _, UR, d = random_setup(dims, 3, 'FUND', 23)
    m = -0.4
    Mh = dense.dense_matrix(lambda v: D.Dhat(v, UR, m, APBC, dims), (16, 4, d))
    Md = dense.dense_matrix(lambda v: D.Dhat_dag(v, UR, m, APBC, dims), (16, 4, d))
    assert np.abs(Md - Mh.conj().T).max() < 1e-14
    G5 = np.kron(np.eye(16), np.kron(GAMMA5, np.eye(d)))
    assert np.abs(G5 @ Mh @ G5 - Md).max() < 1e-14


def test_qhat_hermitian_and_squares_to_normal_op():
    """Q-hat = gamma_5 D-hat (Sec. 5.3.3) is Hermitian, and Q-hat^2 is the
    normal operator D-hat^+ D-hat that CG inverts (dense, 4x2^3)."""
    dims = (4, 2, 2, 2)
    _, UR, d = random_setup(dims, 2, 'SYM', 26)
    m = -0.3
    Q = dense.dense_matrix(lambda v: D.Qhat(v, UR, m, APBC, dims), (16, 4, d))
    A = dense.dense_matrix(lambda v: D.normal_op(v, UR, m, APBC, dims), (16, 4, d))
    scale = np.abs(Q).max()
    assert np.abs(Q - Q.conj().T).max() < 1e-14 * scale
    assert np.abs(Q @ Q - A).max() < 1e-13 * np.abs(A).max()
    # not trivially Hermitian: D-hat itself is not
    Mh = dense.dense_matrix(lambda v: D.Dhat(v, UR, m, APBC, dims), (16, 4, d))
    assert np.abs(Mh - Mh.conj().T).max() > 1e-2


def test_hop_at_sites_matches_field():
    dims = (4, 2, 4, 2)
    _, UR, d = random_setup(dims, 2, 'SYM', 24)
    psi = synth.gaussian_spinor(dims + (4, d), 25)
    full = {False: D.hopping(psi, UR, APBC), True: D.hopping(psi, UR, APBC, dagger=True)}
    coords = L.coordinates(dims)[::3]
    shp = tuple(dims)
    n = len(coords)
    Uf = np.empty((n, 4, d, d), complex)
    Ub = np.empty((n, 4, d, d), complex)
    pf = np.empty((n, 4, 4, d), complex)
    pb = np.empty((n, 4, 4, d), complex)
    wf = np.empty((n, 4), bool)
    wb = np.empty((n, 4), bool)
    for mu in range(4):
        cf, wf[:, mu] = L.neighbour(coords, mu, +1, dims)
        cb, wb[:, mu] = L.neighbour(coords, mu, -1, dims)
        Uf[:, mu] = UR[tuple(coords.T)][:, mu]
        Ub[:, mu] = UR[tuple(cb.T)][:, mu]
        pf[:, mu] = psi[tuple(cf.T)]
        pb[:, mu] = psi[tuple(cb.T)]
    for dag in (False, True):
        got = D.hop_at_sites(coords, Uf, Ub, pf, pb, wf, wb, APBC, dagger=dag)
        assert rel(got, full[dag][tuple(coords.T)]) < 1e-15
    assert shp == dims


# ---------------------------------------------------------------- solvers
def test_cg_matches_dense_solve():
    dims = (2, 2, 2, 2)
    _, UR, d = random_setup(dims, 2, 'FUND', 31)
    m = -0.2
    b = synth.gaussian_spinor((8, 4, d), 32)
    x, it, res = CG.cg_eo(b, UR, m, APBC, dims, tol=1e-12, maxit=1000)
    A = dense.dense_matrix(lambda v: D.normal_op(v, UR, m, APBC, dims), (8, 4, d))
    xs = np.linalg.solve(A, b.ravel()).reshape(b.shape)
    assert res <= 1e-12
    assert rel(x, xs) < 1e-11
    assert 0 < it <= 8 * 4 * d + 5


def test_cg_zero_rhs():
    dims = (2, 2, 2, 2)
    _, UR, d = random_setup(dims, 2, 'FUND', 33)
    x, it, res = CG.cg_eo(np.zeros((8, 4, d), complex), UR, -0.2, APBC, dims)
    assert it == 0 and res == 0.0 and not x.any()


def test_eo_solve_matches_full_solve():
    dims = (2, 2, 4, 2)
    _, UR, d = random_setup(dims, 2, 'ADJ', 34)
    m = 0.05
    eta = synth.gaussian_spinor(dims + (4, d), 35)
    psi, it = CG.solve_dirac_eo(eta, UR, m, APBC, dims, tol=1e-12)
    M = dense.dense_matrix(lambda v: D.dirac(v, UR, m, APBC), dims + (4, d))
    ref = np.linalg.solve(M, eta.ravel()).reshape(eta.shape)
    assert rel(psi, ref) < 1e-10
