"""Pins of the oracle's shifted solves and rational functions of
A = D-hat^dagger D-hat (Sec. 5.3.2) against dense linear algebra and exact
partial-fraction identities (no GPU)."""
import numpy as np

from oracle import cg as CG
from oracle import dense
from oracle import dirac as D
from oracle import rational as RA
from oracle import reps as R
from paper_2503_06721_amd import synth

APBC = (-1, 1, 1, 1)


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def setup(dims, N, rep, seed):
    U = synth.haar_links(dims, N, seed)
    UR = R.represent(U, rep)
    return UR, UR.shape[-1]


def test_shifted_solves_match_dense():
    dims = (2, 2, 2, 2)
    UR, d = setup(dims, 2, 'FUND', 41)
    m = -0.3
    b = synth.gaussian_spinor((8, 4, d), 42)
    shifts = [0.0, 0.01, 0.3, 2.5]
    A = dense.dense_matrix(lambda v: D.normal_op(v, UR, m, APBC, dims), (8, 4, d))
    sols = RA.shifted_solves(b, UR, m, APBC, dims, shifts, tol=1e-13)
    for s, (x, it, res) in zip(shifts, sols):
        ref = np.linalg.solve(A + s * np.eye(A.shape[0]), b.ravel()).reshape(b.shape)
        assert res <= 1e-13
        assert rel(x, ref) < 1e-11, s


def test_rational_apply_matches_spectral_evaluation():
    dims = (2, 2, 2, 2)
    UR, d = setup(dims, 2, 'ADJ', 43)
    m = 0.1
    b = synth.gaussian_spinor((8, 4, d), 44)
    gammas, betas, g0 = [0.4, 1.3, 0.05], [0.02, 0.7, 4.0], 0.25
    A = dense.dense_matrix(lambda v: D.normal_op(v, UR, m, APBC, dims), (8, 4, d))
    lam, V = np.linalg.eigh(A)
    assert lam.min() > 0
    rl = g0 + sum(g / (lam + bk) for g, bk in zip(gammas, betas))
    ref = (V @ (rl * (V.conj().T @ b.ravel()))).reshape(b.shape)
    got = RA.rational_apply(b, UR, m, APBC, dims, gammas, betas, gamma0=g0, tol=1e-13)
    assert rel(got, ref) < 1e-11


def test_partial_fraction_identity():
    """1/((x+1)(x+2)) = 1/(x+1) - 1/(x+2): (A+1)(A+2) r(A) b = b exactly."""
    dims = (4, 4, 2, 2)
    UR, d = setup(dims, 3, 'FUND', 45)
    m = -0.2
    b = synth.gaussian_spinor((32, 4, d), 46)
    y = RA.rational_apply(b, UR, m, APBC, dims, [1.0, -1.0], [1.0, 2.0], tol=1e-13)

    def A(v):
        return D.normal_op(v, UR, m, APBC, dims)
    back = A(A(y) + 2.0 * y) + (A(y) + 2.0 * y)
    assert rel(back, b) < 1e-11


def test_zero_shift_is_the_plain_solve():
    dims = (2, 2, 4, 2)
    UR, d = setup(dims, 2, 'FUND', 47)
    m = -0.1
    b = synth.gaussian_spinor((16, 4, d), 48)
    (x, it, res), = RA.shifted_solves(b, UR, m, APBC, dims, [0.0], tol=1e-12)
    x2, it2, res2 = CG.cg_eo(b, UR, m, APBC, dims, tol=1e-12)
    assert it == it2 and np.array_equal(x, x2)
