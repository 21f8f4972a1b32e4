"""Shifted solves and rational functions of A = D-hat^dagger D-hat, the
operator the RHMC of Sec. 5.3.2 approximates powers of.

Sec. 5.3.2 writes the approximation as a sum of poles,
r(x) = sum_k gamma_k (x + beta_k)^{-1}, applied to A = Q-hat^2 = D-hat^dagger
D-hat, and computes the shifted inverses (A + beta_k)^{-1} phi with a
multi-shift solver.  What that solver returns has a plain definition: the
solution of each shifted system.  Here every shifted system is solved by its
own textbook CG (oracle.cg.cg on A + beta_k), and r(A) phi is the weighted sum
of those solutions (plus an optional constant term gamma_0 phi, which the
printed sum omits; gamma_0 = 0 reproduces it).
"""
from . import dirac
from .cg import cg


def shifted_solves(b_e, UR, m, bc, dims, shifts, tol=1e-10, maxit=10000):
    """[(x_k, iterations, true relative residual)] with x_k = (A + shifts[k])^{-1} b."""
    out = []
    for s in shifts:
        def A(v, s=s):
            return dirac.normal_op(v, UR, m, bc, dims) + s * v
        out.append(cg(A, b_e, tol, maxit))
    return out


def rational_apply(b_e, UR, m, bc, dims, gammas, betas, gamma0=0.0, tol=1e-12, maxit=10000):
    """r(A) b = gamma0 b + sum_k gammas[k] (A + betas[k])^{-1} b (Sec. 5.3.2)."""
    sols = shifted_solves(b_e, UR, m, bc, dims, betas, tol, maxit)
    out = gamma0 * b_e
    for g, (x, _, _) in zip(gammas, sols):
        out = out + g * x
    return out
