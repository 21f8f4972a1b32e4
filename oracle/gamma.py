"""Dirac matrices in the basis of Sec. 2.2 of the paper.

sigma_1..3 are the Pauli matrices, e_0 = -1 (2x2), e_i = -i sigma_i, and
gamma_mu = [[0, e_mu], [e_mu^dagger, 0]] in 2x2 spin blocks.

gamma_5 is not written in the paper.  The reading used here is
gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3, which in this basis equals
diag(1, 1, -1, -1): Hermitian, squares to one, anticommutes with every
gamma_mu.
"""
import numpy as np

I2 = np.eye(2, dtype=np.complex128)
I4 = np.eye(4, dtype=np.complex128)

SIGMA = np.array([
    [[0, 1], [1, 0]],
    [[0, -1j], [1j, 0]],
    [[1, 0], [0, -1]],
], dtype=np.complex128)

E = np.array([-I2, -1j * SIGMA[0], -1j * SIGMA[1], -1j * SIGMA[2]])


def _gamma(mu):
    g = np.zeros((4, 4), dtype=np.complex128)
    g[0:2, 2:4] = E[mu]
    g[2:4, 0:2] = E[mu].conj().T
    return g


GAMMA = np.array([_gamma(mu) for mu in range(4)])
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]


def apply_spin(M, psi):
    """(M psi)_s = sum_t M_st psi_t for psi with spin on axis -2 (colour last)."""
    return np.einsum('st,...ta->...sa', M, psi)
