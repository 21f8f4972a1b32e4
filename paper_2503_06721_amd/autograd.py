"""torch.autograd wrappers of pseudofermion actions and their forces.

    S = FermionAction.apply(U, phi, lattice, m0, tol, maxit)
    S = TwistedMassAction.apply(U, phi, lattice, m0, mu, tol, maxit)
    S = HasenbuschAction.apply(U, phi, lattice, m0, mu1, mu2, tol, maxit)

U      complex128 GPU tensor [T, X, Y, Z, 4, N, N] (fundamental links)
phi    packed FP64 even half spinor (a ``Lattice.new_half()`` buffer)
S      0-dim float64 tensor: S_f = phi^+ (D-hat^+ D-hat)^{-1} phi, evaluated
       with the variational estimator 2 Re<phi, x> - ||D-hat x||^2 (equal to
       S at the exact solution, error quadratic in the solver residual).

Backward returns dS/dU in torch's convention for complex inputs,
dS = Re sum(conj(grad) * dU), for tangent variations dU = i w^a T^a U of the
links (the molecular-dynamics direction): grad = 2i P U with P the Hermitian
traceless force of ``wdirac_force_eo``.  Components of dU off the SU(N)
tangent space are not meaningful for a gauge action and are not represented.
Every computation runs in libwdirac's kernels (rep_links, CG, D-hat, dot,
force); this module only sequences the calls.
"""
import torch

from . import wdirac as W


class FermionAction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, phi, lat, m0, tol=1e-12, maxit=20000):
        U = U.contiguous()
        UR = lat.new_links(W.F64)
        lat.rep_links(UR, U, W.F64)
        x = lat.new_half()
        rc, st = lat.cg_eo(x, phi, UR, m0, tol=tol, maxit=maxit, mode=W.CG_F64)
        if rc != W.OK:
            raise W.WdiracError(rc, 'FermionAction.forward cg_eo')
        y = lat.new_half()
        lat.apply_dhat(y, x, UR, m0)
        s = 2.0 * lat.dot(phi, x)[0].real - lat.norm2(y)[0]
        ctx.lat, ctx.m0 = lat, m0
        ctx.save_for_backward(U)
        ctx.x, ctx.UR = x, UR
        ctx.cg_stats = st[0]
        return torch.tensor(s, dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, grad_s):
        (U,) = ctx.saved_tensors
        G = torch.empty_like(U)
        ctx.lat.force_eo(G, ctx.x, ctx.UR, ctx.m0, U=U, scale=float(grad_s), accumulate=0)
        return G, None, None, None, None, None


def fermion_action(U, phi, lat, m0, tol=1e-12, maxit=20000):
    return FermionAction.apply(U, phi, lat, m0, tol, maxit)


def _shifted_solve(lat, b, UR, m0, shift, tol, maxit):
    x = lat.new_shift_fields(1)
    rc, st = lat.cg_mshift_eo(x, b, UR, m0, [shift], tol=tol, maxit=maxit)
    if rc != W.OK:
        raise W.WdiracError(rc, 'shifted solve')
    return x


class TwistedMassAction(torch.autograd.Function):
    """S_tm = phi^+ (D-hat^+ D-hat + mu^2)^{-1} phi, the twisted-mass monomial
    det(W_+ W_-) of the even-odd Hasenbusch factorisation (Sec. 6.2.1).
    Backward: the force formula at x = (A + mu^2)^{-1} phi."""

    @staticmethod
    def forward(ctx, U, phi, lat, m0, mu, tol=1e-12, maxit=20000):
        U = U.contiguous()
        UR = lat.new_links(W.F64)
        lat.rep_links(UR, U, W.F64)
        x = _shifted_solve(lat, phi, UR, m0, mu * mu, tol, maxit)
        y = lat.new_half()
        lat.apply_dhat(y, x, UR, m0)
        # variational estimator 2 Re<phi, x> - <x, (A + mu^2) x>
        s = 2.0 * lat.dot(phi, x)[0].real - lat.norm2(y)[0] - mu * mu * lat.norm2(x)[0]
        ctx.lat, ctx.m0 = lat, m0
        ctx.save_for_backward(U)
        ctx.x, ctx.UR = x, UR
        return torch.tensor(s, dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, grad_s):
        (U,) = ctx.saved_tensors
        G = torch.empty_like(U)
        ctx.lat.force_eo(G, ctx.x, ctx.UR, ctx.m0, U=U, scale=float(grad_s), accumulate=0)
        return G, None, None, None, None, None, None


class HasenbuschAction(torch.autograd.Function):
    """S_H = psi^+ (D-hat^+ D-hat + mu2^2)^{-1} psi, psi = W_+(mu1) phi, the
    Hasenbusch monomial det[W_-(mu1) (W_+(mu2) W_-(mu2))^{-1} W_+(mu1)]
    (Sec. 6.2.1).  With y = (A + mu2^2)^{-1} psi the link derivative is
    dS = -y^+ dA y - 2 Re(Y'^+ dH X'), X' = (phi, D_oe phi),
    Y' = (gamma_5 y, D_eo^+ gamma_5 y): the force formula at y minus the
    bilinear derivative."""

    @staticmethod
    def forward(ctx, U, phi, lat, m0, mu1, mu2, tol=1e-12, maxit=20000):
        U = U.contiguous()
        UR = lat.new_links(W.F64)
        lat.rep_links(UR, U, W.F64)
        psi = lat.new_half()
        lat.apply_W(psi, phi, UR, m0, mu1, +1)
        y = _shifted_solve(lat, psi, UR, m0, mu2 * mu2, tol, maxit)
        t = lat.new_half()
        lat.apply_dhat(t, y, UR, m0)
        s = 2.0 * lat.dot(psi, y)[0].real - lat.norm2(t)[0] - mu2 * mu2 * lat.norm2(y)[0]
        ctx.lat, ctx.m0 = lat, m0
        ctx.save_for_backward(U)
        ctx.y, ctx.UR, ctx.phi = y, UR, phi
        return torch.tensor(s, dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, grad_s):
        (U,) = ctx.saved_tensors
        lat, UR, m0, y, phi = ctx.lat, ctx.UR, ctx.m0, ctx.y, ctx.phi
        G = torch.empty_like(U)
        lat.force_eo(G, y, UR, m0, U=U, scale=float(grad_s), accumulate=0)
        xo, g5y, yo = lat.new_half(), lat.new_half(), lat.new_half()
        lat.dslash_eo(xo, phi, UR, 1)                  # D_oe phi
        lat.gamma5(g5y, y)
        lat.dslash_eo(yo, g5y, UR, 1, dagger=1)        # D_eo^+ gamma_5 y
        lat.force_bilinear_eo(G, phi, xo, g5y, yo, UR, U=U, scale=-float(grad_s), accumulate=1)
        return G, None, None, None, None, None, None, None


def twisted_mass_action(U, phi, lat, m0, mu, tol=1e-12, maxit=20000):
    return TwistedMassAction.apply(U, phi, lat, m0, mu, tol, maxit)


def hasenbusch_action(U, phi, lat, m0, mu1, mu2, tol=1e-12, maxit=20000):
    return HasenbuschAction.apply(U, phi, lat, m0, mu1, mu2, tol, maxit)
