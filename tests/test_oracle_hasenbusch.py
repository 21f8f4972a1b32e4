"""Pins of the oracle's twisted-mass and Hasenbusch monomials (Sec. 6.2,
Sec. 6.2.1): the algebra of W_pm, central finite differences of both actions
and of the bilinear derivative along random algebra directions (no GPU)."""
import numpy as np
import pytest

from oracle import dense
from oracle import dirac as D
from oracle import force as F
from oracle import hasenbusch as HB
from oracle import reps as R
from oracle.reductions import inner
from paper_2503_06721_amd import synth

APBC = (-1, 1, 1, 1)


def exp_i(H):
    w, V = np.linalg.eigh(H)
    return np.einsum('...ij,...j,...kj->...ik', V, np.exp(1j * w), np.conj(V))


def fd_check(action, U, N, rep, g, h=1e-5, ndir=3, tol=1e-6, seed=3100):
    dims = U.shape[:4]
    for k in range(ndir):
        w = synth.algebra_directions(dims, N, seed + k)
        w /= np.linalg.norm(w)
        X = R.algebra_to_matrix(w, N)
        Sp = action(R.represent(exp_i(h * X) @ U, rep))
        Sm = action(R.represent(exp_i(-h * X) @ U, rep))
        fd = (Sp - Sm) / (2 * h)
        an = float(np.sum(w * g))
        # rounding of S(U +- h X) (|S| can be far above the derivative)
        roundoff = 64 * np.finfo(float).eps * max(abs(Sp), abs(Sm)) / h
        assert abs(fd - an) <= tol * abs(an) + roundoff, (k, fd, an)


def test_w_algebra():
    """W_- = W_+^dagger and W_+ W_- = A + mu^2 (dense, 2^4)."""
    dims = (2, 2, 2, 2)
    UR = R.represent(synth.haar_links(dims, 2, 71), 'FUND')
    m, mu = -0.2, 0.37
    shp = (8, 4, 2)
    Wp = dense.dense_matrix(lambda v: HB.W(v, UR, m, APBC, dims, mu, +1), shp)
    Wm = dense.dense_matrix(lambda v: HB.W(v, UR, m, APBC, dims, mu, -1), shp)
    A = dense.dense_matrix(lambda v: D.normal_op(v, UR, m, APBC, dims), shp)
    assert np.allclose(Wm, Wp.conj().T, atol=1e-12)
    assert np.allclose(Wp @ Wm, A + mu * mu * np.eye(A.shape[0]), atol=1e-10)


@pytest.mark.parametrize('N,rep,m', [(2, 'ADJ', -0.3), (3, 'FUND', 0.1), (3, 'SYM', 0.2)])
def test_hasenbusch_force_finite_differences(N, rep, m):
    dims = (4, 2, 2, 2)
    U = synth.expH_links(dims, N, 0.3, 72)
    UR = R.represent(U, rep)
    d = UR.shape[-1]
    phi = synth.gaussian_spinor((16, 4, d), 73)
    mu1, mu2 = 0.15, 0.6
    g = HB.hasenbusch_force_components(phi, UR, m, APBC, dims, N, rep, mu1, mu2)
    fd_check(lambda URx: HB.action_hasenbusch(phi, URx, m, APBC, dims, mu1, mu2), U, N, rep, g)


def test_tm_force_finite_differences():
    dims = (2, 4, 2, 2)
    N, rep, m, mu = 2, 'FUND', -0.1, 0.3
    U = synth.expH_links(dims, N, 0.3, 74)
    UR = R.represent(U, rep)
    phi = synth.gaussian_spinor((16, 4, 2), 75)
    g = HB.tm_force_components(phi, UR, m, APBC, dims, N, rep, mu)
    fd_check(lambda URx: HB.action_tm(phi, URx, m, APBC, dims, mu), U, N, rep, g)


def test_bilinear_force_finite_differences():
    """d/dw of 2 Re(Y^dagger H(U) X) for fixed random X, Y."""
    dims = (2, 2, 4, 2)
    N, rep = 3, '2AS'
    U = synth.expH_links(dims, N, 0.3, 76)
    UR = R.represent(U, rep)
    d = UR.shape[-1]
    X = synth.gaussian_spinor(dims + (4, d), 77)
    Y = synth.gaussian_spinor(dims + (4, d), 78)
    g = HB.bilinear_force_components(X, Y, UR, APBC, N, rep)
    fd_check(lambda URx: 2.0 * inner(Y, D.hopping(X, URx, APBC)).real, U, N, rep, g, tol=1e-8)


def test_zero_mu_reduces_to_plain_monomial():
    """mu1 = mu2 = 0: S_H = phi^dagger Q-hat A^{-1} Q-hat phi = |phi|^2 (A = Q-hat^2),
    and its force vanishes; mu = 0 twisted mass = the plain action."""
    dims = (2, 2, 2, 4)
    N, rep, m = 2, 'FUND', 0.05
    UR = R.represent(synth.haar_links(dims, N, 79), rep)
    phi = synth.gaussian_spinor((16, 4, 2), 80)
    assert abs(HB.action_hasenbusch(phi, UR, m, APBC, dims, 0.0, 0.0) - inner(phi, phi).real) < 1e-10
    g = HB.hasenbusch_force_components(phi, UR, m, APBC, dims, N, rep, 0.0, 0.0)
    assert np.abs(g).max() < 1e-9
    S_plain, _ = F.action(phi, UR, m, APBC, dims)
    assert abs(HB.action_tm(phi, UR, m, APBC, dims, 0.0) - S_plain) < 1e-10 * abs(S_plain)
