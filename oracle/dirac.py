"""The Wilson-Dirac operator in representation R and its even-odd blocks.

Definitions followed (paper Sec. 2.3, lattice spacing a = 1):

  D_m psi(x) = (4 + m) psi(x)
               - 1/2 sum_mu [ (1 - gamma_mu) U_R(x,mu) psi(x+mu)
                              + (1 + gamma_mu) U_R(x-mu,mu)^dagger psi(x-mu) ]

The hopping term H is D_m without its diagonal (4 + m).  The fermion boundary
condition enters through psi(x + L_mu e_mu) = bc[mu] psi(x) (Sec. 6.3.1).

Even-odd blocks (Sec. 5.3.3): D_eo is H from odd to even sites, D_oe from even
to odd; D_ee = D_oo = (4 + m) for unimproved Wilson fermions; the
preconditioned operator is D-hat = (4+m)^2 - D_eo D_oe (the paper's form that
absorbs one factor of (4+m) into the Schur complement), and the Hermitian form
is Q-hat = gamma_5 D-hat.

Fields: spinors have shape (T, X, Y, Z, 4, d) (spin then colour), represented
links (T, X, Y, Z, 4, d, d) with the direction on axis 4; half fields
(V/2, 4, d) list the sites of one parity in lexicographic order.
"""
import numpy as np

from . import lattice as L
from .gamma import GAMMA, GAMMA5, I4, apply_spin


def _colour(Umat, psi):
    """(U psi)_sa = sum_b U_ab psi_sb, site by site."""
    return np.einsum('...ab,...sb->...sa', Umat, psi)


def _colour_dag(Umat, psi):
    """(U^dagger psi)_sa = sum_b conj(U_ba) psi_sb, site by site."""
    return np.einsum('...ba,...sb->...sa', np.conj(Umat), psi)


def hopping(psi, UR, bc, dagger=False):
    """(H psi)(x) = -1/2 sum_mu [(1-g_mu) U(x,mu) psi(x+mu) + (1+g_mu) U(x-mu,mu)^+ psi(x-mu)].

    With dagger=True this is the adjoint H^dagger, written out from the
    definition of the adjoint of a shift: the adjoint of A(x) psi(x+mu) is
    A(x-mu)^dagger chi(x-mu), so the two spin projectors trade places,
        (H^+ chi)(x) = -1/2 sum_mu [(1+g_mu) U(x,mu) chi(x+mu)
                                    + (1-g_mu) U(x-mu,mu)^+ chi(x-mu)]
    (gamma_mu is Hermitian; the boundary phases are real)."""
    s = -1.0 if dagger else 1.0
    out = np.zeros(psi.shape, dtype=np.complex128)
    for mu in range(4):
        fwd = _colour(UR[..., mu, :, :], L.shift_fwd(psi, mu, bc))
        out += apply_spin(I4 - s * GAMMA[mu], fwd)
        bwd = _colour_dag(L.link_bwd(UR, mu), L.shift_bwd(psi, mu, bc))
        out += apply_spin(I4 + s * GAMMA[mu], bwd)
    return -0.5 * out


def links_with_boundary_phase(UR, bc):
    """U_R with the fermion boundary phase bc[mu] multiplied into the links
    U_R(x, mu) with x_mu = L_mu - 1, the hops that cross the boundary (Sec.
    6.3.1 implements antiperiodic conditions as a sign on one slice of the
    represented field).  Periodic hopping on these links equals hopping with
    the boundary condition on the fermion field."""
    out = np.array(UR, copy=True)
    for mu in range(4):
        if bc[mu] != 1:
            idx = [slice(None)] * 4 + [mu]
            idx[mu] = -1
            out[tuple(idx)] *= bc[mu]
    return out


def dirac(psi, UR, m, bc):
    """D_m psi = (4 + m) psi + H psi."""
    return (4.0 + m) * psi + hopping(psi, UR, bc)


def gamma5(psi):
    return apply_spin(GAMMA5, psi)


def hop_block(half_in, UR, bc, dims, out_parity, dagger=False):
    """H restricted to (out parity p, in parity 1-p): D_eo for p = 0, D_oe for p = 1.

    With dagger=True: the (p, 1-p) block of H^dagger, which is the adjoint of
    the block H_{1-p,p} (so D_oe^dagger for p = 0, D_eo^dagger for p = 1)."""
    full = L.from_half(half_in, dims, 1 - out_parity)
    return L.to_half(hopping(full, UR, bc, dagger), dims, out_parity)


def D_eo(psi_o, UR, bc, dims):
    return hop_block(psi_o, UR, bc, dims, 0)


def D_oe(psi_e, UR, bc, dims):
    return hop_block(psi_e, UR, bc, dims, 1)


def Dhat(x_e, UR, m, bc, dims):
    """D-hat x = (4+m)^2 x - D_eo D_oe x (Sec. 5.3.3)."""
    return (4.0 + m) ** 2 * x_e - D_eo(D_oe(x_e, UR, bc, dims), UR, bc, dims)


def Dhat_dag(x_e, UR, m, bc, dims):
    """D-hat^dagger = (4+m)^2 - D_oe^dagger D_eo^dagger (adjoint of each factor)."""
    t_o = hop_block(x_e, UR, bc, dims, 1, dagger=True)     # D_eo^dagger x
    return (4.0 + m) ** 2 * x_e - hop_block(t_o, UR, bc, dims, 0, dagger=True)


def Qhat(x_e, UR, m, bc, dims):
    """Q-hat = gamma_5 D-hat."""
    return gamma5(Dhat(x_e, UR, m, bc, dims))


def normal_op(x_e, UR, m, bc, dims):
    """A = D-hat^dagger D-hat, the Hermitian positive operator inverted by CG."""
    return Dhat_dag(Dhat(x_e, UR, m, bc, dims), UR, m, bc, dims)


def eo_source(eta, UR, m, bc, dims):
    """Even-odd right-hand side: D-hat psi_e = (4+m) eta_e - D_eo eta_o.

    Follows from eliminating psi_o = (eta_o - D_oe psi_e)/(4+m) in the block
    form of D_m psi = eta (Sec. 5.3.3)."""
    eta_e = L.to_half(eta, dims, 0)
    eta_o = L.to_half(eta, dims, 1)
    return (4.0 + m) * eta_e - D_eo(eta_o, UR, bc, dims)


def eo_reconstruct(psi_e, eta, UR, m, bc, dims):
    """Full solution of D_m psi = eta from its even part: psi_o = (eta_o - D_oe psi_e)/(4+m)."""
    eta_o = L.to_half(eta, dims, 1)
    psi_o = (eta_o - D_oe(psi_e, UR, bc, dims)) / (4.0 + m)
    return L.from_half(psi_e, dims, 0) + L.from_half(psi_o, dims, 1)


def hop_at_sites(coords, UR_fwd, UR_bwd, psi_fwd, psi_bwd, wrap_fwd, wrap_bwd, bc,
                 dagger=False):
    """(H psi)(x) at a list of n sites, from their gathered neighbourhood.

    coords    (n, 4) sites x
    UR_fwd    (n, 4, d, d)   U_R(x, mu)
    UR_bwd    (n, 4, d, d)   U_R(x - mu, mu)
    psi_fwd   (n, 4, 4, d)   psi(x + mu) as stored (direction first)
    psi_bwd   (n, 4, 4, d)   psi(x - mu) as stored
    wrap_*    (n, 4) bool    whether the hop in direction mu crosses the boundary
    Same formula as `hopping` (including its dagger form), written per site
    for sampled checks of large lattices."""
    s = -1.0 if dagger else 1.0
    n = coords.shape[0]
    d = psi_fwd.shape[-1]
    out = np.zeros((n, 4, d), dtype=np.complex128)
    for mu in range(4):
        sf = np.where(wrap_fwd[:, mu], bc[mu], 1.0)[:, None, None]
        sb = np.where(wrap_bwd[:, mu], bc[mu], 1.0)[:, None, None]
        fwd = _colour(UR_fwd[:, mu], sf * psi_fwd[:, mu])
        out += apply_spin(I4 - s * GAMMA[mu], fwd)
        bwd = _colour_dag(UR_bwd[:, mu], sb * psi_bwd[:, mu])
        out += apply_spin(I4 + s * GAMMA[mu], bwd)
    return -0.5 * out
