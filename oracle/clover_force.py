"""Link derivative of the clover-improved even-odd fermion actions (the force
that the clover term of Sec. 6.1.2, and its exponential form of Sec. 6.1.3,
add to the HMC of Sec. 5.3).  Test infrastructure: a plain CPU reference,
not used by the library.

Actions (readings; the paper states the operators, not these derivatives):
* pseudofermion  S_f = phi_e^+ (D-hat^+ D-hat)^{-1} phi_e with the general
  even-odd operator D-hat = D_ee - D_eo D_oo^{-1} D_oe of Sec. 5.3.3 (the
  diagonal blocks M(x) = D_ee(x) or D_oo(x) carry the clover term);
* determinant    S_det = -2 sum_{x odd} log det D_oo(x): det D = det D_oo
  det D-hat (Sec. 5.3.3), so two flavours need |det D_oo|^2 beside the
  pseudofermion.  For the exponential form det D_oo is a constant, since the
  clover term is traceless.

Link variation U(x,mu) -> exp(i w^a T^a_F) U(x,mu) as in oracle.force, so
U_R -> exp(i w^a T^a_R) U_R inside every clover leaf.

Derivation.  With x = A^{-1} phi, y = D-hat x, z_o = D_oo^{-1} D_oe x and
w_o = D_oo^{-+} D_eo^+ y, X = (x, z_o), Y = (y, w_o) on the full lattice:
    dS_f = -2 Re(y^+ dD-hat x) = 2 Re(Y^+ dH X) - 2 Re sum_x tr[dM(x) X(x) Y(x)^+],
and dS_det = -2 sum_{x odd} tr[M(x)^{-1} dM(x)].  Both diagonal parts have the
form -2 Re sum_x tr[dM(x) Omega(x)].  Regular clover: dM = dC with
C = c_sw (i/4) sum_{mu != nu} sigma_mu,nu (x) F_mu,nu.  Exponential:
M = (4 + m) exp(C / (4 + m)), and tr[dM Omega] = tr[dC Omega'] with
Omega' = int_0^1 exp((1-s) A) Omega exp(s A) ds, A = C / (4 + m), evaluated in
the eigenbasis of the Hermitian A (divided differences of exp).

With F = (Q - Q^+)/8, tr[dQ^+ Lam] = conj(tr[dQ Lam^+]); a leaf l = P U Q'
containing the link gives dl = P (i w T_R) U Q', and l = P U^+ Q' gives
dl = -P U^+ (i w T_R) Q'.
"""
import numpy as np

from . import lattice as L
from . import reps
from .clover import SIGMA_MUNU, clover_term, diagonal_blocks, half_blocks, apply_sitewise
from .dirac import hop_block

# The four leaves of the (mu, nu) plane at x, each as four steps
# (offset along mu, offset along nu, direction 0 = mu / 1 = nu, dagger):
# U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+, then its images turned by 90,
# 180 and 270 degrees, all starting and ending at x (oracle.clover.leaves).
LEAF_STEPS = (
    ((0, 0, 0, False), (1, 0, 1, False), (0, 1, 0, True), (0, 0, 1, True)),
    ((0, 0, 1, False), (-1, 1, 0, True), (-1, 0, 1, True), (-1, 0, 0, False)),
    ((-1, 0, 0, True), (-1, -1, 1, True), (-1, -1, 0, False), (0, -1, 1, False)),
    ((0, -1, 1, True), (0, -1, 0, False), (1, -1, 1, False), (0, 0, 0, True)),
)


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def _mm(A, B):
    return np.einsum('...ab,...bc->...ac', A, B)


def _shift(f, mu, a, nu, b):
    """f(x + a mu + b nu), periodic."""
    return np.roll(np.roll(f, -a, axis=mu), -b, axis=nu)


def step_matrix(UR, mu, nu, step):
    a, b, dirn, dag = step
    M = _shift(UR[..., mu if dirn == 0 else nu, :, :], mu, a, nu, b)
    return _dag(M) if dag else M


def leaf_product(UR, mu, nu, k):
    steps = LEAF_STEPS[k]
    out = step_matrix(UR, mu, nu, steps[0])
    for s in steps[1:]:
        out = _mm(out, step_matrix(UR, mu, nu, s))
    return out


def insertion_pseudofermion(X, Y):
    """Omega(x) = X(x) Y(x)^+ as (4d x 4d) matrices, row index spin * d + colour."""
    v = X.reshape(X.shape[:4] + (-1,))
    w = Y.reshape(Y.shape[:4] + (-1,))
    return np.einsum('...i,...j->...ij', v, np.conj(w))


def exp_adjoint(A, Om):
    """int_0^1 exp((1-s) A) Om exp(s A) ds for Hermitian A, via A = V diag(l) V^+:
    entry (i, j) in the eigenbasis is (V^+ Om V)_ij (e^{l_i} - e^{l_j}) / (l_i - l_j)."""
    lam, V = np.linalg.eigh(A)
    Ot = np.einsum('...ki,...kl,...lj->...ij', np.conj(V), Om, V)
    li, lj = lam[..., :, None], lam[..., None, :]
    dl = li - lj
    safe = np.where(dl == 0.0, 1.0, dl)
    ratio = np.where(dl == 0.0, 1.0, np.expm1(dl) / safe)
    phi = np.exp(lj) * ratio
    return np.einsum('...ik,...kl,...jl->...ij', V, Ot * phi, np.conj(V))


def diagonal_force_components(U, rep, Om, m, csw, exponential=False):
    """dS/dw^a_mu(x) for dS = -2 Re sum_x tr[dM(x) Om(x)], array (T,X,Y,Z,4,N^2-1)."""
    N = U.shape[-1]
    UR = reps.represent(U, rep)
    d = UR.shape[-1]
    TR = reps.rep_generators(N, rep)
    if exponential:
        A = clover_term(UR, csw) / (4.0 + m)
        Om = exp_adjoint(A, Om)
    Om6 = Om.reshape(Om.shape[:4] + (4, d, 4, d))
    out = np.zeros(U.shape[:4] + (4, N * N - 1))
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            # tr[(sigma (x) dF) Om] = tr_colour[dF Lam], Lam_ba = sum_st sigma_st Om_(t b),(s a)
            Lam = np.einsum('st,...tbsa->...ba', SIGMA_MUNU[mu, nu], Om6)
            for k in range(4):
                steps = LEAF_STEPS[k]
                mats = [step_matrix(UR, mu, nu, s) for s in steps]
                for f in range(4):
                    before = np.broadcast_to(np.eye(d), UR.shape[:4] + (d, d))
                    for j in range(f):
                        before = _mm(before, mats[j])
                    after = np.broadcast_to(np.eye(d), UR.shape[:4] + (d, d))
                    for j in range(f + 1, 4):
                        after = _mm(after, mats[j])
                    a, b, dirn, dag = steps[f]
                    link = mats[f]
                    comps = []
                    for Lk in (Lam, _dag(Lam)):
                        # d tr[l Lk] / dw^a at the link (complex)
                        if not dag:
                            Z = _mm(_mm(_mm(link, after), Lk), before)
                            comps.append(1j * np.einsum('kab,...ba->...k', TR, Z))
                        else:
                            Z = _mm(_mm(_mm(after, Lk), before), link)
                            comps.append(-1j * np.einsum('kab,...ba->...k', TR, Z))
                    # tr[dM Om] = (i c_sw / 4) (tr[dQ Lam] - conj(tr[dQ Lam^+])) / 8
                    dtr = 0.25j * csw * (comps[0] - np.conj(comps[1])) / 8.0
                    contrib = -2.0 * dtr.real
                    # the link sits at x + a mu + b nu: move the value there
                    out[..., mu if dirn == 0 else nu, :] += _shift(contrib, mu, -a, nu, -b)
    return out


def fields_XY(x_e, UR, m, csw, bc, dims, exponential=False):
    """X = (x, D_oo^{-1} D_oe x), Y = (D-hat x, D_oo^{-+} D_eo^+ D-hat x)."""
    M = diagonal_blocks(UR, m, csw, exponential)
    Me, Mo = half_blocks(M, dims, 0), half_blocks(M, dims, 1)
    Moi = np.linalg.inv(Mo)
    z_o = apply_sitewise(Moi, hop_block(x_e, UR, bc, dims, 1))
    y_e = apply_sitewise(Me, x_e) - hop_block(z_o, UR, bc, dims, 0)
    w_o = apply_sitewise(_dag(Moi), hop_block(y_e, UR, bc, dims, 1, dagger=True))
    X = L.from_half(x_e, dims, 0) + L.from_half(z_o, dims, 1)
    Y = L.from_half(y_e, dims, 0) + L.from_half(w_o, dims, 1)
    return X, Y


def hopping_force_components(X, Y, UR, bc, N, rep):
    """d/dw^a of 2 Re(Y^+ H X): the spin-traced outer products of oracle.force."""
    from .force import sigma
    S = sigma(X, Y, bc)
    TR = reps.rep_generators(N, rep)
    return np.einsum('kab,...ba->...k', TR, _mm(UR, S)).imag


def pseudofermion_force_components(x_e, U, rep, m, csw, bc, dims, exponential=False):
    """dS_f/dw^a_mu(x) at x = A^{-1} phi, array (T, X, Y, Z, 4, N^2-1)."""
    N = U.shape[-1]
    UR = reps.represent(U, rep)
    X, Y = fields_XY(x_e, UR, m, csw, bc, dims, exponential)
    g = hopping_force_components(X, Y, UR, bc, N, rep)
    return g + diagonal_force_components(U, rep, insertion_pseudofermion(X, Y), m, csw, exponential)


def logdet_odd(U, rep, m, csw, dims, exponential=False):
    """sum_{x odd} log det D_oo(x) (real: the blocks are Hermitian)."""
    M = diagonal_blocks(reps.represent(U, rep), m, csw, exponential)
    sign, ld = np.linalg.slogdet(half_blocks(M, dims, 1))
    return float(np.sum(ld))


def det_action(U, rep, m, csw, dims, exponential=False):
    """S_det = -2 sum_{x odd} log det D_oo(x)."""
    return -2.0 * logdet_odd(U, rep, m, csw, dims, exponential)


def det_force_components(U, rep, m, csw, dims, exponential=False):
    """dS_det/dw^a_mu(x): Om = M^{-1} on the odd sites, 0 on the even ones."""
    UR = reps.represent(U, rep)
    M = diagonal_blocks(UR, m, csw, exponential)
    par = L.parity_field(dims)
    Om = np.where(par[..., None, None] == 1, np.linalg.inv(M), 0.0)
    return diagonal_force_components(U, rep, Om, m, csw, exponential)
