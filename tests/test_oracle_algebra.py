"""Pins of the oracle's gamma basis, representations and compensated sums
against facts fixed by the paper and by mathematics (no GPU)."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

from oracle import gamma as G
from oracle import reductions as RD
from oracle import reps as R
from paper_2503_06721_amd import synth

HERE = os.path.dirname(__file__)
PAIRS = [(N, rep) for N in (2, 3, 4) for rep in R.REPS if not (N == 2 and rep == R.ASYM)]


# ---------------------------------------------------------------- gamma basis
def test_clifford_algebra():
    for mu in range(4):
        for nu in range(4):
            ac = G.GAMMA[mu] @ G.GAMMA[nu] + G.GAMMA[nu] @ G.GAMMA[mu]
            assert np.array_equal(ac, 2.0 * (mu == nu) * G.I4)


def test_gamma_hermitian_and_gamma5():
    for mu in range(4):
        assert np.array_equal(G.GAMMA[mu], G.GAMMA[mu].conj().T)
        assert np.array_equal(G.GAMMA5 @ G.GAMMA[mu] + G.GAMMA[mu] @ G.GAMMA5, np.zeros((4, 4)))
    # gamma_0 gamma_1 gamma_2 gamma_3 in the chiral basis of Sec. 2.2
    assert np.array_equal(G.GAMMA5, np.diag([1, 1, -1, -1]).astype(complex))
    assert np.array_equal(G.GAMMA5 @ G.GAMMA5, G.I4)


def test_spin_projectors():
    # (1 -+ gamma_mu)/2 are complementary rank-2 projectors
    for mu in range(4):
        for s in (1, -1):
            P = 0.5 * (G.I4 - s * G.GAMMA[mu])
            assert np.allclose(P @ P, P, atol=0)
            assert np.linalg.matrix_rank(P) == 2


# --------------------------------------------------------- representations
def test_generators_normalised():
    for N in (2, 3, 4, 5):
        T = R.fund_generators(N)
        assert T.shape == (N * N - 1, N, N)
        gram = np.einsum('aij,bji->ab', T, T)
        assert np.allclose(gram, 0.5 * np.eye(N * N - 1), atol=1e-15)
        assert np.allclose(T, np.conj(np.swapaxes(T, 1, 2)), atol=0)
        assert np.allclose(np.trace(T, axis1=1, axis2=2), 0, atol=1e-15)
    # SU(2): T^a = sigma_a / 2 in this ordering
    assert np.allclose(R.fund_generators(2), G.SIGMA / 2, atol=0)


def test_rep_table_matches_paper():
    with open(os.path.join(HERE, 'golden', 'rep_table.json')) as f:
        table = json.load(f)
    for row in table['values']:
        N, rep = row['N'], row['rep']
        assert R.dim(N, rep) == row['dim']
        assert Fraction(R.T_R(N, rep)).limit_denominator(100) == Fraction(*row['T_R'])
        assert Fraction(R.casimir(N, rep)).limit_denominator(100) == Fraction(*row['C2'])


@pytest.mark.parametrize('N,rep', PAIRS)
def test_index_identity(N, rep):
    # T_R (N^2 - 1) = C_2(R) d_R: fixes the 2AS normalisation to (N-2)/2
    assert math.isclose(R.T_R(N, rep) * (N * N - 1), R.casimir(N, rep) * R.dim(N, rep),
                        rel_tol=1e-14, abs_tol=1e-14)


@pytest.mark.parametrize('N,rep', PAIRS)
def test_rep_group_properties(N, rep):
    rng = np.random.default_rng(7)
    U = synth.haar_su_n(20, N, rng)
    V = synth.haar_su_n(20, N, rng)
    RU, RV, RUV = R.represent(U, rep), R.represent(V, rep), R.represent(U @ V, rep)
    d = R.dim(N, rep)
    assert RU.shape == (20, d, d)
    eye = np.eye(d)
    assert np.abs(RU @ np.conj(np.swapaxes(RU, 1, 2)) - eye).max() < 1e-13   # unitary
    assert np.abs(np.linalg.det(RU) - 1).max() < 1e-13                        # special
    assert np.abs(RUV - RU @ RV).max() < 1e-13                                # homomorphism
    tr = np.trace(U, axis1=1, axis2=2)
    tr2 = np.trace(U @ U, axis1=1, axis2=2)
    chi = np.trace(RU, axis1=1, axis2=2)
    expected = {R.FUND: tr, R.ADJ: np.abs(tr) ** 2 - 1,
                R.SYM: (tr ** 2 + tr2) / 2, R.ASYM: (tr ** 2 - tr2) / 2}[rep]
    assert np.abs(chi - expected).max() < 1e-13                               # character
    if rep == R.ADJ:
        assert RU.dtype == np.float64                                         # real rep
    if rep == R.FUND:
        assert np.array_equal(RU, U)


@pytest.mark.parametrize('N,rep', PAIRS)
def test_rep_generators(N, rep):
    TR = R.rep_generators(N, rep)
    d = R.dim(N, rep)
    n = N * N - 1
    assert TR.shape == (n, d, d)
    assert np.abs(TR - np.conj(np.swapaxes(TR, 1, 2))).max() < 1e-14        # Hermitian
    gram = np.einsum('aij,bji->ab', TR, TR)
    assert np.abs(gram - R.T_R(N, rep) * np.eye(n)).max() < 1e-13
    cas = np.einsum('aij,ajk->ik', TR, TR)
    assert np.abs(cas - R.casimir(N, rep) * np.eye(d)).max() < 1e-13
    # the defining relation U^R = exp(i w^a T^a_R) for U = exp(i w^a T^a_F)
    rng = np.random.default_rng(11)
    for _ in range(3):
        w = rng.normal(0, 0.7, n)
        U = scipy.linalg.expm(1j * np.einsum('a,aij->ij', w, R.fund_generators(N)))
        UR = scipy.linalg.expm(1j * np.einsum('a,aij->ij', w, TR))
        assert np.abs(R.represent(U[None], rep)[0] - UR).max() < 1e-12


def test_algebra_roundtrip():
    rng = np.random.default_rng(3)
    for N in (2, 3, 4):
        w = rng.normal(size=(5, N * N - 1))
        assert np.allclose(R.matrix_to_algebra(R.algebra_to_matrix(w, N)), w, atol=1e-14)


# ------------------------------------------------------------ reductions
def test_fast_two_sum_exact():
    rng = np.random.default_rng(5)
    for _ in range(200):
        a, b = rng.normal() * 10.0 ** rng.integers(-20, 20), rng.normal() * 10.0 ** rng.integers(-20, 20)
        s, c = RD.fast_two_sum(a, b)
        assert s == a + b
        assert Fraction(s) + Fraction(c) == Fraction(a) + Fraction(b)


def test_compensated_sums():
    vals = [1e16, 1.0, -1e16]
    assert sum(vals) == 0.0                       # naive sum loses the 1
    assert RD.neumaier_sum(vals) == 1.0
    assert RD.second_order_neumaier_sum(vals) == 1.0
    assert RD.double_double_sum(vals) == 1.0
    rng = np.random.default_rng(9)
    x = rng.normal(size=20000) * 10.0 ** rng.integers(-8, 8, size=20000)
    x = np.concatenate([x, -x[:10000] * (1 + 1e-12)])
    exact = math.fsum(x.tolist())
    naive = float(np.sum(x))
    for f in (RD.neumaier_sum, RD.second_order_neumaier_sum, RD.double_double_sum):
        assert abs(f(x) - exact) <= abs(naive - exact) + 1e-300
        assert abs(f(x) - exact) <= 4 * np.finfo(float).eps * abs(exact) + 1e-300


def test_inner_and_norms():
    a = np.array([1 + 2j, 3 - 1j])
    b = np.array([2 - 1j, 1j])
    assert RD.inner(a, b) == (1 - 2j) * (2 - 1j) + (3 + 1j) * 1j
    assert RD.norm2(a) == 15.0
    assert RD.max_norm(np.array([1 - 5j, 4 + 0j])) == 5.0
