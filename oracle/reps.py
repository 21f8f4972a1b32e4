"""Fermion representations of SU(N): FUND, ADJ, SYM, 2AS (paper Sec. 2.3,
table of supported representations).

The paper defines the represented link as U^R = exp(i omega^a T^a_R) where
U = exp(i omega^a T^a_F), and leaves the explicit maps to its earlier
reference.  The explicit forms below are one consistent choice of basis; any
orthonormal basis satisfies the invariants the tests check, so the GPU path
implements this same basis (stated in the design notes) independently.

Fundamental generators T^a (tr T^a T^b = delta^ab / 2), in this order:
  for each pair j < k in lexicographic order
      S_jk = (E_jk + E_kj) / 2,   A_jk = (-i E_jk + i E_kj) / 2,
  then for k = 1 .. N-1
      D_k  = diag(1, .., 1, -k, 0, .., 0) / sqrt(2 k (k+1))   (k ones).

Maps U -> U_R:
  FUND  U_R = U
  ADJ   (U_R)_ab = 2 tr(T^a U T^b U^dagger)              (real orthogonal)
  SYM   basis e_(ab), a <= b, lexicographic: e_(aa) = E_aa,
        e_(ab) = (E_ab + E_ba)/sqrt 2;
        (U_R)_(ab),(cd) = tr(e_(ab)^dagger U e_(cd) U^T)
  2AS   as SYM with a < b and e_(ab) = (E_ab - E_ba)/sqrt 2.

Generators T^a_R are the exact linearisation -i d/de R(exp(i e T^a)) at 0:
  ADJ       (T^a_R)_bc = 2 tr(T^b [T^a, T^c])
  SYM/2AS   (T^a_R)_(ab),(cd) = tr(e_(ab)^dagger (T^a e_(cd) + e_(cd) T^a^T)).

Normalisations T_R and Casimirs C_2(R) follow the paper's table of
representations.  The table prints T_R = (N-1)/2 for 2AS; the list of T_R
values in Sec. 7.6.5 prints (N-2)/2, and only (N-2)/2 satisfies
T_R (N^2 - 1) = C_2(R) d_R with the table's own Casimir, so (N-2)/2 is used.
"""
import numpy as np

FUND, ADJ, SYM, ASYM = 'FUND', 'ADJ', 'SYM', '2AS'
REPS = (FUND, ADJ, SYM, ASYM)


def fund_generators(N):
    """Array (N^2-1, N, N) of Hermitian traceless T^a with tr T^a T^b = delta/2."""
    gens = []
    for j in range(N):
        for k in range(j + 1, N):
            S = np.zeros((N, N), dtype=np.complex128)
            S[j, k] = S[k, j] = 0.5
            A = np.zeros((N, N), dtype=np.complex128)
            A[j, k] = -0.5j
            A[k, j] = 0.5j
            gens += [S, A]
    for k in range(1, N):
        D = np.zeros((N, N), dtype=np.complex128)
        for i in range(k):
            D[i, i] = 1.0
        D[k, k] = -k
        gens.append(D / np.sqrt(2.0 * k * (k + 1)))
    return np.array(gens)


def two_index_basis(N, symmetric):
    """Array (d, N, N) of the orthonormal basis e_(ab) of (anti)symmetric matrices."""
    basis = []
    for a in range(N):
        for b in range(a if symmetric else a + 1, N):
            e = np.zeros((N, N), dtype=np.complex128)
            if a == b:
                e[a, a] = 1.0
            else:
                e[a, b] = 1.0 / np.sqrt(2.0)
                e[b, a] = (1.0 if symmetric else -1.0) / np.sqrt(2.0)
            basis.append(e)
    return np.array(basis)


def dim(N, rep):
    """Dimension d_R (table of representations, Sec. 2.3)."""
    return {FUND: N, ADJ: N * N - 1, SYM: N * (N + 1) // 2, ASYM: N * (N - 1) // 2}[rep]


def is_real(rep):
    """ADJ is a real representation and is stored as real numbers (Sec. 4.1.2)."""
    return rep == ADJ


def T_R(N, rep):
    """Trace normalisation tr(T^a_R T^b_R) = T_R delta^ab (2AS per Sec. 7.6.5)."""
    return {FUND: 0.5, ADJ: float(N), SYM: (N + 2) / 2.0, ASYM: (N - 2) / 2.0}[rep]


def casimir(N, rep):
    """C_2(R) as printed in the table of representations."""
    cf = (N * N - 1) / (2.0 * N)
    return {FUND: cf, ADJ: float(N),
            SYM: cf * 2.0 * (N + 2) / (N + 1),
            ASYM: cf * 2.0 * (N - 2) / (N - 1)}[rep]


def represent(U, rep):
    """U_R = R(U) for links U of shape (..., N, N).  ADJ returns a real array."""
    N = U.shape[-1]
    if rep == FUND:
        return np.array(U, dtype=np.complex128, copy=True)
    if rep == ADJ:
        T = fund_generators(N)
        Ud = np.conj(np.swapaxes(U, -1, -2))
        # W_b = U T^b U^dagger, then (U_R)_ab = 2 tr(T^a W_b)
        W = np.einsum('...ij,bjk->...bik', U, T)
        W = np.einsum('...bik,...kl->...bil', W, Ud)
        R = 2.0 * np.einsum('aij,...bji->...ab', T, W)
        return np.ascontiguousarray(R.real)
    basis = two_index_basis(N, rep == SYM)
    # W_B = U e_B U^T, then (U_R)_AB = tr(e_A^dagger W_B) = sum_ij conj(e_A)_ij (W_B)_ij
    W = np.einsum('...ij,Bjk->...Bik', U, basis)
    W = np.einsum('...Bik,...lk->...Bil', W, U)
    return np.einsum('Aij,...Bij->...AB', np.conj(basis), W)


def rep_generators(N, rep):
    """Array (N^2-1, d_R, d_R) of the represented generators T^a_R."""
    T = fund_generators(N)
    if rep == FUND:
        return T
    if rep == ADJ:
        n = N * N - 1
        G = np.zeros((n, n, n), dtype=np.complex128)
        for a in range(n):
            for b in range(n):
                for c in range(n):
                    comm = T[a] @ T[c] - T[c] @ T[a]
                    G[a, b, c] = 2.0 * np.trace(T[b] @ comm)
        return G
    basis = two_index_basis(N, rep == SYM)
    d = len(basis)
    G = np.zeros((len(T), d, d), dtype=np.complex128)
    for a in range(len(T)):
        for A in range(d):
            for B in range(d):
                act = T[a] @ basis[B] + basis[B] @ T[a].T
                G[a, A, B] = np.trace(basis[A].conj().T @ act)
    return G


def algebra_to_matrix(omega, N):
    """Hermitian matrix sum_a omega^a T^a_F for omega of shape (..., N^2-1)."""
    return np.einsum('...a,aij->...ij', omega, fund_generators(N))


def matrix_to_algebra(H):
    """Components omega^a = 2 tr(T^a H) of a Hermitian traceless H (..., N, N)."""
    N = H.shape[-1]
    return 2.0 * np.einsum('aij,...ji->...a', fund_generators(N), H).real
