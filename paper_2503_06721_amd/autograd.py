"""torch.autograd wrapper of the pseudofermion action and its force.

    S = FermionAction.apply(U, phi, lattice, m0, tol, maxit)

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
