"""Textbook conjugate gradient (Hestenes-Stiefel) on A = D-hat^dagger D-hat.

The paper names CG among its inverters (Sec. 5.1.2) without writing it out;
this is the classical algorithm:

    r = b - A x,  p = r,  rho = <r, r>
    repeat:  q = A p;  alpha = rho / <p, q>;  x += alpha p;  r -= alpha q;
             rho' = <r, r>;  beta = rho' / rho;  p = r + beta p;  rho = rho'
    until sqrt(rho) <= tol * ||b||.

Stopping reading: the tolerance is on the relative residual ||b - A x|| / ||b||
(not its square).  On return the true residual b - A x is recomputed.
"""
import math

import numpy as np

from . import dirac
from .reductions import inner, norm2


def cg(apply_A, b, tol, maxit, x0=None):
    """Solve A x = b.  Returns (x, iterations, true relative residual)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128, copy=True)
    r = b - apply_A(x)
    p = r.copy()
    rho = norm2(r)
    bnorm = math.sqrt(norm2(b))
    it = 0
    if bnorm == 0.0:
        return np.zeros_like(b), 0, 0.0
    while it < maxit and math.sqrt(rho) > tol * bnorm:
        q = apply_A(p)
        alpha = rho / inner(p, q).real
        x = x + alpha * p
        r = r - alpha * q
        rho_new = norm2(r)
        beta = rho_new / rho
        p = r + beta * p
        rho = rho_new
        it += 1
    true_res = math.sqrt(norm2(b - apply_A(x))) / bnorm
    return x, it, true_res


def cg_eo(b_e, UR, m, bc, dims, tol=1e-10, maxit=10000, x0=None):
    """CG on (D-hat^dagger D-hat) x = b over the even sites."""
    def A(v):
        return dirac.normal_op(v, UR, m, bc, dims)
    return cg(A, b_e, tol, maxit, x0)


def solve_dirac_eo(eta, UR, m, bc, dims, tol=1e-10, maxit=10000):
    """Solve D_m psi = eta through the even-odd system (Sec. 5.3.3):
    D-hat psi_e = b'_e, solved as D-hat^dagger D-hat psi_e = D-hat^dagger b'_e,
    then psi_o reconstructed.  Returns (psi, iterations)."""
    bprime = dirac.eo_source(eta, UR, m, bc, dims)
    rhs = dirac.Dhat_dag(bprime, UR, m, bc, dims)
    psi_e, it, _ = cg_eo(rhs, UR, m, bc, dims, tol, maxit)
    return dirac.eo_reconstruct(psi_e, eta, UR, m, bc, dims), it
