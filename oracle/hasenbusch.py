"""Twisted-mass and Hasenbusch monomials of the even-odd operator
(Sec. 6.2 and Sec. 6.2.1).

With Q-hat = gamma_5 D-hat (D-hat the even-odd Wilson operator of Sec. 5.3.3,
one factor of 4+m absorbed) and W_pm(mu) = Q-hat +- i mu, Q-hat is Hermitian,
W_-(mu) = W_+(mu)^dagger and W_+ W_- = Q-hat^2 + mu^2 = A + mu^2 with
A = D-hat^dagger D-hat.

* twisted-mass monomial, det(W_+ W_-):  S_tm = phi^dagger (A + mu^2)^{-1} phi;
* Hasenbusch monomial, det[W_-(mu1) (W_+(mu2) W_-(mu2))^{-1} W_+(mu1)]:
      S_H = psi^dagger (A + mu2^2)^{-1} psi,   psi = W_+(mu1) phi.

Derivative (variation of the links as in oracle.force): with
y = (A + mu2^2)^{-1} psi,
      dS_H = 2 Re(y^dagger dW_+ phi) - y^dagger dA y,
and dW_+ = gamma_5 dD-hat = -gamma_5 (dD_eo D_oe + D_eo dD_oe), so
      2 Re(y^dagger dW_+ phi) = -2 Re(Y'^dagger dH X'),
      X' = (phi, D_oe phi),  Y' = (gamma_5 y, D_eo^dagger gamma_5 y).
Both pieces are the bilinear derivative d[2 Re(Y^dagger H X)] of oracle.force
(with X, Y from y for the first).
"""
import numpy as np

from . import dirac
from . import force as F
from . import lattice as L
from . import reps
from .cg import cg
from .reductions import inner


def W(x_e, UR, m, bc, dims, mu, sign=1):
    """W_pm(mu) x = gamma_5 D-hat x + i sign mu x."""
    return dirac.gamma5(dirac.Dhat(x_e, UR, m, bc, dims)) + 1j * sign * mu * x_e


def shifted_solve(b_e, UR, m, bc, dims, shift, tol=1e-13, maxit=20000):
    def A(v):
        return dirac.normal_op(v, UR, m, bc, dims) + shift * v
    x, _, _ = cg(A, b_e, tol, maxit)
    return x


def action_tm(phi_e, UR, m, bc, dims, mu, tol=1e-13):
    return inner(phi_e, shifted_solve(phi_e, UR, m, bc, dims, mu * mu, tol)).real


def action_hasenbusch(phi_e, UR, m, bc, dims, mu1, mu2, tol=1e-13):
    psi = W(phi_e, UR, m, bc, dims, mu1, +1)
    return inner(psi, shifted_solve(psi, UR, m, bc, dims, mu2 * mu2, tol)).real


def bilinear_force_components(X, Y, UR, bc, N, rep):
    """d/dw^a_mu(x) of 2 Re(Y^dagger H X) for fixed full-lattice fields X, Y."""
    S = F.sigma(X, Y, bc)
    TR = reps.rep_generators(N, rep)
    US = np.einsum('...ab,...bc->...ac', UR, S)
    return np.einsum('kab,...ba->...k', TR, US).imag


def hasenbusch_force_components(phi_e, UR, m, bc, dims, N, rep, mu1, mu2, tol=1e-13):
    psi = W(phi_e, UR, m, bc, dims, mu1, +1)
    y = shifted_solve(psi, UR, m, bc, dims, mu2 * mu2, tol)
    g1 = F.force_components(y, UR, m, bc, dims, N, rep)
    g5y = dirac.gamma5(y)
    Xp = L.from_half(phi_e, dims, 0) + L.from_half(dirac.D_oe(phi_e, UR, bc, dims), dims, 1)
    Yp = L.from_half(g5y, dims, 0) + L.from_half(dirac.hop_block(g5y, UR, bc, dims, 1, dagger=True), dims, 1)
    return g1 - bilinear_force_components(Xp, Yp, UR, bc, N, rep)


def tm_force_components(phi_e, UR, m, bc, dims, N, rep, mu, tol=1e-13):
    """S_tm: the plain force formula at x = (A + mu^2)^{-1} phi."""
    return F.force_components(shifted_solve(phi_e, UR, m, bc, dims, mu * mu, tol), UR, m, bc, dims, N, rep)
