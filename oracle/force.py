"""Pseudofermion action on the even sites and its derivative with respect to
the gauge links.

Action (Sec. 5.3.1; the exponent printed there lacks the minus sign of
e^{-S}, read here as S = phi^dagger (Q^2)^{-1} phi >= 0), in even-odd form:

    S_f = phi_e^dagger (D-hat^dagger D-hat)^{-1} phi_e.

Link derivative.  A link is varied as U(x,mu) -> exp(i w^a T^a_F) U(x,mu)
(left multiplication, the form of the molecular-dynamics equation
dU/dtau = pi U of Sec. 2.5); a representation is a homomorphism, so
U_R -> exp(i w^a T^a_R) U_R.  With x = A^{-1} phi_e, y = D-hat x,
z_o = D_oe x and w_o = D_eo^dagger y, the full-lattice fields
X = (x, z_o) and Y = (y, w_o) give

    dS/dw^a_mu(x) = Im tr[ T^a_R U_R(x,mu) Sigma_mu(x) ],
    Sigma_mu(x) = tr_spin[ (1 - g_mu) X(x+mu) Y(x)^dagger
                           + (1 + g_mu) Y(x+mu) X(x)^dagger ],

derived from dS = -x^dagger dA x = 2 Re(Y^dagger dH X).  This is the even-odd
analogue of the paper's spin-traced force of Sec. 2.5, whose printed
projection omits the factor i T^a_R and the direction index.

The returned force is the Hermitian traceless matrix
P_mu(x) = sum_a (dS/dw^a_mu(x)) T^a_F.
"""
import numpy as np

from . import dirac
from . import lattice as L
from . import reps
from .cg import cg_eo
from .gamma import GAMMA, I4
from .reductions import inner


def action(phi_e, UR, m, bc, dims, tol=1e-13, maxit=20000):
    """S_f = <phi, A^{-1} phi>.  Returns (S, x)."""
    x, _, _ = cg_eo(phi_e, UR, m, bc, dims, tol, maxit)
    return inner(phi_e, x).real, x


def action_variational(phi_e, x_e, UR, m, bc, dims):
    """S~ = 2 Re<phi, x> - <x, A x>: equals S at x = A^{-1} phi, with an error
    quadratic in the solver error (useful for finite differences)."""
    Ax = dirac.normal_op(x_e, UR, m, bc, dims)
    return 2.0 * inner(phi_e, x_e).real - inner(x_e, Ax).real


def sigma_fields(x_e, UR, m, bc, dims):
    """X, Y (full lattice) built from the CG solution x = A^{-1} phi."""
    z_o = dirac.D_oe(x_e, UR, bc, dims)
    y_e = dirac.Dhat(x_e, UR, m, bc, dims)
    w_o = dirac.hop_block(y_e, UR, bc, dims, 1, dagger=True)
    X = L.from_half(x_e, dims, 0) + L.from_half(z_o, dims, 1)
    Y = L.from_half(y_e, dims, 0) + L.from_half(w_o, dims, 1)
    return X, Y


def sigma(X, Y, bc):
    """Sigma_mu(x) for all x, mu: array (T, X, Y, Z, 4, d, d)."""
    d = X.shape[-1]
    out = np.zeros(X.shape[:4] + (4, d, d), dtype=np.complex128)
    for mu in range(4):
        Xf = L.shift_fwd(X, mu, bc)
        Yf = L.shift_fwd(Y, mu, bc)
        # tr_spin[M A B^dagger]_{ab} = sum_{s,t} M_st A_{t a} conj(B_{s b})
        out[..., mu, :, :] = (np.einsum('st,...ta,...sb->...ab', I4 - GAMMA[mu], Xf, np.conj(Y))
                              + np.einsum('st,...ta,...sb->...ab', I4 + GAMMA[mu], Yf, np.conj(X)))
    return out


def force_components(x_e, UR, m, bc, dims, N, rep):
    """dS/dw^a_mu(x), array (T, X, Y, Z, 4, N^2-1)."""
    X, Y = sigma_fields(x_e, UR, m, bc, dims)
    S = sigma(X, Y, bc)
    TR = reps.rep_generators(N, rep)
    US = np.einsum('...ab,...bc->...ac', UR, S)
    return np.einsum('kab,...ba->...k', TR, US).imag


def force(x_e, UR, m, bc, dims, N, rep):
    """P_mu(x) = sum_a (dS/dw^a_mu(x)) T^a_F, array (T, X, Y, Z, 4, N, N)."""
    g = force_components(x_e, UR, m, bc, dims, N, rep)
    return reps.algebra_to_matrix(g, N)
