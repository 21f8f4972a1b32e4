"""Hybrid Monte Carlo molecular dynamics (Sec. 5.2 integrators, Sec. 5.3 HMC)
for the Wilson plaquette gauge action and the even-odd pseudofermion action.

Conventions (written out here; the paper gives the integrators' step schemes
and error scaling in its table of integrators but not the equations):
* momenta pi_mu(x) = pi^a T^a_F are Hermitian traceless N x N matrices;
  H = sum_{x,mu} tr(pi^2) + S_g + S_f, and tr(pi^2) = (1/2) sum_a (pi^a)^2;
* dU/dtau = i pi U and dpi/dtau = -F with F = sum_a (dS/dw^a) T^a_F the force
  matrix of the variation U -> exp(i w^a T^a_F) U (the convention of
  oracle.force), which conserves H;
* gauge action S_g = beta sum_x sum_{mu<nu} (1 - Re tr P_mu,nu(x) / N) with
  P_mu,nu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ (fundamental links,
  periodic); with the staple sum A_mu(x), sum over the plaquettes containing
  U_mu(x) of Re tr P = Re tr(U_mu(x) A_mu(x)), so
  dS_g/dw^a_mu(x) = (beta / N) Im tr(T^a U_mu(x) A_mu(x));
* pseudofermion S_f = phi^+ (D-hat^+ D-hat)^{-1} phi with its force from
  oracle.force; phi = D-hat^+ eta for Gaussian eta at the start;
* with a clover term (c_sw given): the clover D-hat of oracle.clover, and
  S_det = -2 sum_{x odd} log det D_oo added to the action, both with their
  forces from oracle.clover_force;
* integrators: leapfrog (PQP) and second-order Omelyan (PQPQP, lambda =
  0.1931833275037836), nsteps steps of size eps over the trajectory.
"""
import numpy as np

from . import clover as CL
from . import clover_force as CF
from . import force as F
from . import reps
from .cg import cg, cg_eo
from .reductions import inner


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def _mm(*Ms):
    out = Ms[0]
    for M in Ms[1:]:
        out = np.einsum('...ab,...bc->...ac', out, M)
    return out


def _sh(f, mu, step):
    return np.roll(f, -step, axis=mu)


def exp_i(H):
    """exp(i H) for Hermitian H (..., N, N), by eigendecomposition."""
    w, V = np.linalg.eigh(H)
    return np.einsum('...ij,...j,...kj->...ik', V, np.exp(1j * w), np.conj(V))


def plaquettes(U):
    """Re tr P_mu,nu(x) / N for mu < nu, array (T, X, Y, Z, 6)."""
    N = U.shape[-1]
    out = []
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Um, Un = U[..., mu, :, :], U[..., nu, :, :]
            P = _mm(Um, _sh(Un, mu, 1), _dag(_sh(Um, nu, 1)), _dag(Un))
            out.append(np.trace(P, axis1=-2, axis2=-1).real / N)
    return np.stack(out, axis=-1)


def gauge_action(U, beta):
    return beta * float(np.sum(1.0 - plaquettes(U)))


def staples(U, mu):
    """A_mu(x) with Re tr(U_mu(x) A_mu(x)) = sum of Re tr P over the six
    plaquettes that contain U_mu(x)."""
    Um = U[..., mu, :, :]
    A = np.zeros_like(Um)
    for nu in range(4):
        if nu == mu:
            continue
        Un = U[..., nu, :, :]
        # upper: U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
        A += _mm(_sh(Un, mu, 1), _dag(_sh(Um, nu, 1)), _dag(Un))
        # lower: U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)
        Un_m = _sh(Un, nu, -1)
        A += _mm(_dag(_sh(Un_m, mu, 1)), _dag(_sh(Um, nu, -1)), Un_m)
    return A


def gauge_force(U, beta):
    """F_g = sum_a (dS_g/dw^a) T^a, array (T, X, Y, Z, 4, N, N)."""
    N = U.shape[-1]
    T = reps.fund_generators(N)
    out = np.zeros_like(U)
    for mu in range(4):
        M = _mm(U[..., mu, :, :], staples(U, mu))
        g = (beta / N) * np.einsum('kab,...ba->...k', T, M).imag
        out[..., mu, :, :] = reps.algebra_to_matrix(g, N)
    return out


def kinetic(pi):
    return float(np.sum(np.einsum('...ab,...ba->...', pi, pi)).real)


class Action:
    """S_g + S_f for fermions in representation rep; phi the pseudofermion.
    csw: clover coefficient (None: unimproved Wilson); exponential: the
    exponential clover form."""

    def __init__(self, beta, m, rep, bc, phi_e, tol=1e-13, with_fermions=True, csw=None, exponential=False):
        self.beta, self.m, self.rep, self.bc = beta, m, rep, bc
        self.phi, self.tol, self.with_fermions = phi_e, tol, with_fermions
        self.csw, self.exponential = csw, exponential

    def _solve(self, UR, dims):
        if self.csw is None:
            return cg_eo(self.phi, UR, self.m, self.bc, dims, self.tol, 50000)[0]
        M = CL.diagonal_blocks(UR, self.m, self.csw, self.exponential)
        def A(v):
            return CL.normal_op_clover(v, UR, self.m, self.csw, self.bc, dims, self.exponential, blocks=M)
        return cg(A, self.phi, self.tol, 50000)[0]

    def value(self, U):
        s = gauge_action(U, self.beta)
        if self.with_fermions:
            UR = reps.represent(U, self.rep)
            dims = U.shape[:4]
            s += inner(self.phi, self._solve(UR, dims)).real
            if self.csw is not None:
                s += CF.det_action(U, self.rep, self.m, self.csw, dims, self.exponential)
        return s

    def force(self, U):
        Fm = gauge_force(U, self.beta)
        if self.with_fermions:
            N = U.shape[-1]
            UR = reps.represent(U, self.rep)
            dims = U.shape[:4]
            x = self._solve(UR, dims)
            if self.csw is None:
                Fm = Fm + F.force(x, UR, self.m, self.bc, dims, N, self.rep)
            else:
                g = (CF.pseudofermion_force_components(x, U, self.rep, self.m, self.csw, self.bc, dims,
                                                       self.exponential)
                     + CF.det_force_components(U, self.rep, self.m, self.csw, dims, self.exponential))
                Fm = Fm + reps.algebra_to_matrix(g, N)
        return Fm


def leapfrog(U, pi, action, eps, nsteps):
    pi = pi - 0.5 * eps * action.force(U)
    for n in range(nsteps):
        U = exp_i(eps * pi) @ U
        pi = pi - (eps if n < nsteps - 1 else 0.5 * eps) * action.force(U)
    return U, pi


OMELYAN_LAMBDA = 0.1931833275037836


def omelyan2(U, pi, action, eps, nsteps, lam=OMELYAN_LAMBDA):
    for _ in range(nsteps):
        pi = pi - lam * eps * action.force(U)
        U = exp_i(0.5 * eps * pi) @ U
        pi = pi - (1.0 - 2.0 * lam) * eps * action.force(U)
        U = exp_i(0.5 * eps * pi) @ U
        pi = pi - lam * eps * action.force(U)
    return U, pi


def trajectory(U0, pi0, action, eps, nsteps, integrator='omelyan2'):
    """Returns (U1, pi1, H0, H1)."""
    H0 = kinetic(pi0) + action.value(U0)
    step = omelyan2 if integrator == 'omelyan2' else leapfrog
    U1, pi1 = step(U0, pi0, action, eps, nsteps)
    H1 = kinetic(pi1) + action.value(U1)
    return U1, pi1, H0, H1
