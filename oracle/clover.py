"""Clover-improved Wilson-Dirac operator (Sec. 6.1.2) and its even-odd form.

The clover term adds to the diagonal blocks
    D_ee,m + D_oo,m = (4 + m) + c_sw (i/4) sum_{mu,nu} sigma_mu,nu F_mu,nu(x),
with the field strength built from the four plaquettes of the (mu, nu) plane
that have a corner at x (the "clover leaves").

Readings (the section leaves these open or prints them garbled):
* sigma_mu,nu = (i/2) [gamma_mu, gamma_nu] in the gamma basis of Sec. 2.2.
* Q_mu,nu(x) is the sum of the four leaves, each a closed loop that starts and
  ends at x and turns from mu to nu in the same sense:
      U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
    + U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu)
    + U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
    + U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^+,
  and F_mu,nu = (Q_mu,nu - Q_mu,nu^+) / 8 (the printed prefactor; the
  expression printed after it is garbled).  Links are the represented links
  U_R; a boundary phase folded into the links cancels in every closed loop.
* With the clover term the diagonal blocks are no longer multiples of one, so
  the even-odd operator is the Schur complement
      D-hat = D_ee - D_eo D_oo^{-1} D_oe
  (Sec. 5.3.3 writes this general form before specialising it); for
  c_sw = 0 it equals the plain D-hat divided by (4 + m).
* The exponential variant (Sec. 6.1.3) replaces the diagonal blocks by
  (4 + m) exp(c_sw / (4 + m) (i/4) sum sigma F).
"""
import numpy as np
import scipy.linalg

from . import dirac
from . import lattice as L
from .gamma import GAMMA, I4

SIGMA_MUNU = np.array([[0.5j * (GAMMA[m] @ GAMMA[n] - GAMMA[n] @ GAMMA[m]) for n in range(4)] for m in range(4)])


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def _mm(*Ms):
    out = Ms[0]
    for M in Ms[1:]:
        out = np.einsum('...ab,...bc->...ac', out, M)
    return out


def _sh(f, mu, step):
    """f(x + step * mu) with periodic wrap (no phase)."""
    return np.roll(f, -step, axis=mu)


def leaves(UR, mu, nu):
    """Q_mu,nu(x): sum of the four clover leaves at every site, (T,X,Y,Z,d,d)."""
    Um, Un = UR[..., mu, :, :], UR[..., nu, :, :]
    l1 = _mm(Um, _sh(Un, mu, 1), _dag(_sh(Um, nu, 1)), _dag(Un))
    Um_m = _sh(Um, mu, -1)                       # U_mu(x - mu)
    Un_m = _sh(Un, mu, -1)                       # U_nu(x - mu)
    l2 = _mm(Un, _dag(_sh(Um_m, nu, 1)), _dag(Un_m), Um_m)
    Um_mn = _sh(Um_m, nu, -1)                    # U_mu(x - mu - nu)
    Un_mn = _sh(Un_m, nu, -1)                    # U_nu(x - mu - nu)
    Un_n = _sh(Un, nu, -1)                       # U_nu(x - nu)
    l3 = _mm(_dag(Um_m), _dag(Un_mn), Um_mn, Un_n)
    Um_n = _sh(Um, nu, -1)                       # U_mu(x - nu)
    l4 = _mm(_dag(Un_n), Um_n, _sh(Un_n, mu, 1), _dag(Um))
    return l1 + l2 + l3 + l4


def field_strength(UR):
    """F[mu, nu] = (Q - Q^+) / 8, array (4, 4, T, X, Y, Z, d, d)."""
    d = UR.shape[-1]
    F = np.zeros((4, 4) + UR.shape[:4] + (d, d), dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            if mu != nu:
                Q = leaves(UR, mu, nu)
                F[mu, nu] = (Q - _dag(Q)) / 8.0
    return F


def clover_term(UR, csw):
    """(i/4) c_sw sum_{mu,nu} sigma_mu,nu (x) F_mu,nu as per-site (4d x 4d)
    matrices with row index spin * d + colour, array (T, X, Y, Z, 4d, 4d)."""
    F = field_strength(UR)
    d = UR.shape[-1]
    out = np.zeros(UR.shape[:4] + (4 * d, 4 * d), dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            if mu != nu:
                out += np.einsum('st,...ab->...satb', SIGMA_MUNU[mu, nu], F[mu, nu]).reshape(out.shape)
    return 0.25j * csw * out


def diagonal_blocks(UR, m, csw, exponential=False):
    """The site-diagonal part of the operator, (T, X, Y, Z, 4d, 4d)."""
    C = clover_term(UR, csw)
    n = C.shape[-1]
    if not exponential:
        return (4.0 + m) * np.eye(n) + C
    A = C / (4.0 + m)
    E = np.stack([scipy.linalg.expm(a) for a in A.reshape(-1, n, n)]).reshape(A.shape)
    return (4.0 + m) * E


def apply_sitewise(M, psi):
    """(M psi)(x) for per-site matrices M (...,4d,4d) and a field (..., 4, d)."""
    sh = psi.shape
    v = psi.reshape(sh[:-2] + (sh[-2] * sh[-1],))
    return np.einsum('...ij,...j->...i', M, v).reshape(sh)


def dirac_clover(psi, UR, m, csw, bc, exponential=False, blocks=None):
    """Full-lattice clover operator: diagonal blocks + hopping term (blocks:
    as in Dhat_clover)."""
    M = diagonal_blocks(UR, m, csw, exponential) if blocks is None else blocks
    return apply_sitewise(M, psi) + dirac.hopping(psi, UR, bc)


def half_blocks(M, dims, p):
    """Per-site matrices of the sites of parity p, (V/2, 4d, 4d)."""
    return L.to_half(M, dims, p)


def Dhat_clover(x_e, UR, m, csw, bc, dims, exponential=False, dagger=False, blocks=None):
    """D-hat = D_ee - D_eo D_oo^{-1} D_oe on an even half field (dagger: its adjoint).
    blocks: diagonal_blocks(UR, m, csw, exponential) when the caller already
    holds them (a solver applying the operator many times)."""
    M = diagonal_blocks(UR, m, csw, exponential) if blocks is None else blocks
    Me, Mo = half_blocks(M, dims, 0), half_blocks(M, dims, 1)
    if dagger:
        Me, Mo = _dag(Me), _dag(Mo)
    Moi = np.linalg.inv(Mo)
    t = dirac.hop_block(x_e, UR, bc, dims, 1, dagger=dagger)
    t = apply_sitewise(Moi, t)
    return apply_sitewise(Me, x_e) - dirac.hop_block(t, UR, bc, dims, 0, dagger=dagger)


def normal_op_clover(x_e, UR, m, csw, bc, dims, exponential=False, blocks=None):
    """A = D-hat^dagger D-hat with the clover term (blocks: as in Dhat_clover)."""
    y = Dhat_clover(x_e, UR, m, csw, bc, dims, exponential, blocks=blocks)
    return Dhat_clover(y, UR, m, csw, bc, dims, exponential, dagger=True, blocks=blocks)
