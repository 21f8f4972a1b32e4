"""Pins of the oracle's clover force (no GPU): the leaf table against the
operator's leaves, the exponential's adjoint derivative against the block
exponential, central finite differences of the pseudofermion and determinant
actions along random algebra directions (regular and exponential clover), the
closed-form determinant of the exponential form, and the c_sw = 0 limit that
reduces to the pinned Wilson force."""
import numpy as np
import pytest
import scipy.linalg

from oracle import cg as CG
from oracle import clover as CL
from oracle import clover_force as CF
from oracle import force as F
from oracle import reps as R
from oracle.reductions import inner
from paper_2503_06721_amd import synth

APBC = (-1, 1, 1, 1)


def exp_i(H):
    w, V = np.linalg.eigh(H)
    return np.einsum('...ij,...j,...kj->...ik', V, np.exp(1j * w), np.conj(V))


def test_leaf_steps_are_the_operator_leaves():
    U = synth.expH_links((4, 3, 2, 4), 3, 0.6, 900)
    UR = R.represent(U, 'SYM')
    for mu in range(4):
        for nu in range(4):
            if mu != nu:
                Q = sum(CF.leaf_product(UR, mu, nu, k) for k in range(4))
                assert np.abs(Q - CL.leaves(UR, mu, nu)).max() < 1e-13


def test_exp_adjoint_is_the_block_exponential():
    """int exp((1-s)A) W exp(sA) ds is the upper-right block of
    exp([[A, W], [0, A]]) (Van Loan), and tr[dE W] = tr[dA W'] for E = exp(A)."""
    rng = np.random.default_rng(901)
    n = 6
    G = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    A = 0.7 * (G + G.conj().T)
    W = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    Wp = CF.exp_adjoint(A, W)
    big = np.zeros((2 * n, 2 * n), dtype=complex)
    big[:n, :n] = A
    big[n:, n:] = A
    big[:n, n:] = W
    assert np.abs(Wp - scipy.linalg.expm(big)[:n, n:]).max() < 1e-12 * np.abs(Wp).max()
    dA = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    h = 1e-6
    fd = np.trace((scipy.linalg.expm(A + h * dA) - scipy.linalg.expm(A - h * dA)) @ W) / (2 * h)
    assert abs(fd - np.trace(dA @ Wp)) < 1e-7 * abs(fd)
    # degenerate spectrum: A = a 1 gives exp(a) W
    assert np.abs(CF.exp_adjoint(0.3 * np.eye(n), W) - np.exp(0.3) * W).max() < 1e-14


def normal_op(UR, m, csw, dims, expo):
    M = CL.diagonal_blocks(UR, m, csw, expo)
    return lambda v: CL.normal_op_clover(v, UR, m, csw, APBC, dims, expo, blocks=M)


def pf_action(U, phi, rep, m, csw, dims, expo):
    """Variational estimate 2 Re<phi, x> - <x, A x> (error quadratic in the CG error)."""
    UR = R.represent(U, rep)
    A = normal_op(UR, m, csw, dims, expo)
    x, _, _ = CG.cg(A, phi, 1e-14, 20000)
    return 2.0 * inner(phi, x).real - inner(x, A(x)).real


@pytest.mark.parametrize('N,rep,m,csw,expo', [(3, 'FUND', 0.1, 1.7, False), (2, 'ADJ', -0.2, 1.3, True),
                                              (3, 'SYM', 0.3, 1.1, False), (2, 'FUND', 0.0, 2.0, True)])
def test_pseudofermion_force_finite_differences(N, rep, m, csw, expo):
    dims = (4, 2, 2, 2)
    U = synth.expH_links(dims, N, 0.5, 910 + N)
    UR = R.represent(U, rep)
    d = UR.shape[-1]
    eta = synth.gaussian_spinor((16, 4, d), 911)
    phi = CL.Dhat_clover(eta, UR, m, csw, APBC, dims, expo, dagger=True)
    x, _, _ = CG.cg(normal_op(UR, m, csw, dims, expo), phi, 1e-14, 20000)
    g = CF.pseudofermion_force_components(x, U, rep, m, csw, APBC, dims, expo)
    h = 1e-5
    for k in range(3):
        w = synth.algebra_directions(dims, N, 3100 + k)
        w /= np.linalg.norm(w)
        X = R.algebra_to_matrix(w, N)
        fd = (pf_action(exp_i(h * X) @ U, phi, rep, m, csw, dims, expo)
              - pf_action(exp_i(-h * X) @ U, phi, rep, m, csw, dims, expo)) / (2 * h)
        an = float(np.sum(w * g))
        assert abs(fd - an) <= 1e-6 * abs(an), (k, fd, an)


def test_pseudofermion_force_single_links():
    """Locality: directions on one link at a time, including links of the
    time boundary (the phase must cancel in every leaf)."""
    dims = (4, 2, 2, 2)
    N, rep, m, csw = 2, 'FUND', 0.2, 1.9
    U = synth.expH_links(dims, N, 0.6, 920)
    UR = R.represent(U, rep)
    phi = synth.gaussian_spinor((16, 4, 2), 921)
    x, _, _ = CG.cg(normal_op(UR, m, csw, dims, False), phi, 1e-14, 20000)
    g = CF.pseudofermion_force_components(x, U, rep, m, csw, APBC, dims, False)
    rng = np.random.default_rng(922)
    h = 1e-5
    for site, mu in [((3, 1, 0, 1), 0), ((0, 0, 1, 1), 0), ((2, 1, 1, 0), 2), ((1, 0, 0, 0), 3)]:
        w = rng.normal(size=N * N - 1)
        Up, Um = U.copy(), U.copy()
        Up[site + (mu,)] = exp_i(h * R.algebra_to_matrix(w, N)) @ U[site + (mu,)]
        Um[site + (mu,)] = exp_i(-h * R.algebra_to_matrix(w, N)) @ U[site + (mu,)]
        fd = (pf_action(Up, phi, rep, m, csw, dims, False) - pf_action(Um, phi, rep, m, csw, dims, False)) / (2 * h)
        an = float(w @ g[site + (mu,)])
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-2), (site, mu, fd, an)


@pytest.mark.parametrize('N,rep', [(3, 'FUND'), (2, 'ADJ'), (4, '2AS')])
def test_det_force_finite_differences(N, rep):
    dims = (4, 2, 2, 4)
    m, csw = -0.1, 1.6
    U = synth.expH_links(dims, N, 0.5, 930 + N)
    g = CF.det_force_components(U, rep, m, csw, dims)
    assert np.abs(g).max() > 1e-3
    # fourth-order central stencil: |S_det| ~ 10^3 makes the two-point
    # difference at small h roundoff-limited
    h = 1e-3
    for k in range(3):
        w = synth.algebra_directions(dims, N, 3200 + k)
        w /= np.linalg.norm(w)
        X = R.algebra_to_matrix(w, N)
        S = [CF.det_action(exp_i(j * h * X) @ U, rep, m, csw, dims) for j in (-2, -1, 1, 2)]
        fd = (S[0] - 8.0 * S[1] + 8.0 * S[2] - S[3]) / (12.0 * h)
        an = float(np.sum(w * g))
        assert abs(fd - an) <= 1e-7 * abs(an), (k, fd, an)


def test_exponential_determinant_is_constant():
    """log det((4+m) exp(A)) = 4 d log(4+m) + tr A and the clover term is
    traceless: S_det is a closed-form constant and its force vanishes."""
    dims = (2, 2, 2, 4)
    N, rep, m, csw = 3, 'FUND', -0.3, 1.8
    U = synth.expH_links(dims, N, 0.7, 940)
    n_odd = int(np.prod(dims)) // 2
    assert abs(CF.logdet_odd(U, rep, m, csw, dims, True) - n_odd * 12 * np.log(4.0 + m)) < 1e-10
    g = CF.det_force_components(U, rep, m, csw, dims, True)
    assert np.abs(g).max() < 1e-12


def test_csw_zero_is_the_wilson_force():
    """c_sw = 0: D-hat = D-hat_Wilson / (4 + m), so S = (4+m)^2 S_Wilson and the
    force scales the same way (at x = (4+m)^2 x_Wilson)."""
    dims = (4, 2, 2, 2)
    N, rep, m = 2, 'SYM', 0.15
    U = synth.expH_links(dims, N, 0.5, 950)
    UR = R.represent(U, rep)
    phi = synth.gaussian_spinor((16, 4, 3), 951)
    xw, _, _ = CG.cg_eo(phi, UR, m, APBC, dims, tol=1e-14)
    gw = F.force_components(xw, UR, m, APBC, dims, N, rep)
    g = CF.pseudofermion_force_components((4.0 + m) ** 2 * xw, U, rep, m, 0.0, APBC, dims, False)
    assert np.abs(g - (4.0 + m) ** 2 * gw).max() < 1e-12 * np.abs(gw).max()
