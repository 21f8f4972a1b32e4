"""Hybrid Monte Carlo molecular dynamics over libwdirac (Sec. 5.2, 5.3).

Conventions as in the library's HMC entry points: momenta pi are Hermitian
traceless matrices in the canonical link layout, dU/dtau = i pi U,
dpi/dtau = -F (F the force matrix of the gauge and fermion actions),
H = sum tr(pi^2) + S_g + S_f with the Wilson plaquette action S_g and the
even-odd pseudofermion action S_f = phi^+ (D-hat^+ D-hat)^{-1} phi; with a
clover term (csw given; regular, Sec. 6.1.2, or exponential, Sec. 6.1.3) the
clover D-hat = D_ee - D_eo D_oo^{-1} D_oe and the odd-block determinant term
S_det = -2 sum_{x odd} log|det D_oo| (det D = det D_oo det D-hat).
Integrators: leapfrog (PQP) and second-order Omelyan (PQPQP).  An HMC
update (Sec. 5.3) draws the momenta and the pseudofermion noise, integrates a
trajectory and accepts it with probability min(1, exp(-dH)).  Every
computation runs in the library's kernels; this module only sequences calls.
"""
import math

import torch

from . import wdirac as W

OMELYAN_LAMBDA = 0.1931833275037836


class HMC:
    def __init__(self, lat, beta, m0, tol=1e-12, maxit=20000, with_fermions=True, csw=None, exponential=0):
        self.lat, self.beta, self.m0 = lat, float(beta), float(m0)
        self.tol, self.maxit, self.with_fermions = tol, maxit, with_fermions
        self.csw, self.exponential = (None if csw is None else float(csw)), int(exponential)
        self.UR = lat.new_links(W.F64)
        self.x = lat.new_half()
        self.ws_cg = lat.new_workspace(W.OP_CG, 1, W.CG_F64)
        self.ws_force = lat.new_workspace(W.OP_FORCE)
        self.ws_gauge = lat.new_workspace(W.OP_GAUGE)
        if self.csw is not None:
            self.clov = lat.new_clover(W.F64)
            self.ws_clov = lat.new_workspace(W.OP_CLOVER, 1, W.F64)
            self.ws_cforce = lat.new_workspace(W.OP_CLOVER_FORCE, 1, W.F64)
        self.cg_iters = 0

    def _operator(self, U):
        """Represented links (and clover field) of U."""
        self.lat.rep_links(self.UR, U, W.F64)
        if self.csw is not None:
            self.lat.clover_field(self.clov, U, self.m0, self.csw, self.exponential, W.F64, workspace=self.ws_clov)

    def _solve(self, U, phi):
        self._operator(U)
        self.x.zero_()
        if self.csw is None:
            rc, st = self.lat.cg_eo(self.x, phi, self.UR, self.m0, tol=self.tol, maxit=self.maxit,
                                    workspace=self.ws_cg)
        else:
            rc, st = self.lat.cg_eo_clover(self.x, phi, self.UR, self.clov, tol=self.tol, maxit=self.maxit,
                                           workspace=self.ws_cg)
        if rc != W.OK:
            raise W.WdiracError(rc, 'HMC solve')
        self.cg_iters += st[0]['iters']

    def action(self, U, phi):
        s = self.lat.gauge_action(U, self.beta, workspace=self.ws_gauge)
        if self.with_fermions:
            self._solve(U, phi)
            s += self.lat.dot(phi, self.x)[0].real
            if self.csw is not None:
                s += -2.0 * self.lat.clover_logdet(self.clov, workspace=self.ws_cforce)
        return s

    def kinetic(self, pi):
        return self.lat.kinetic(pi, workspace=self.ws_gauge)

    def hamiltonian(self, U, pi, phi):
        return self.kinetic(pi) + self.action(U, phi)

    def kick(self, pi, U, phi, c):
        """pi <- pi - c F(U)."""
        self.lat.gauge_force(pi, U, self.beta, scale=-c, accumulate=1)
        if self.with_fermions:
            self._solve(U, phi)
            if self.csw is None:
                self.lat.force_eo(pi, self.x, self.UR, self.m0, scale=-c, accumulate=1, workspace=self.ws_force)
            else:
                self.lat.force_eo_clover(pi, self.x, self.UR, U, self.clov, self.m0, self.csw, self.exponential,
                                         scale=-c, accumulate=1, workspace=self.ws_cforce)
                self.lat.force_clover_logdet(pi, U, self.clov, self.m0, self.csw, self.exponential, scale=-c,
                                             accumulate=1, workspace=self.ws_cforce)

    def drift(self, U, pi, c):
        """U <- exp(i c pi) U."""
        self.lat.link_update(U, pi, c)

    def leapfrog(self, U, pi, phi, eps, nsteps):
        self.kick(pi, U, phi, 0.5 * eps)
        for n in range(nsteps):
            self.drift(U, pi, eps)
            self.kick(pi, U, phi, eps if n < nsteps - 1 else 0.5 * eps)

    def omelyan2(self, U, pi, phi, eps, nsteps, lam=OMELYAN_LAMBDA):
        for _ in range(nsteps):
            self.kick(pi, U, phi, lam * eps)
            self.drift(U, pi, 0.5 * eps)
            self.kick(pi, U, phi, (1.0 - 2.0 * lam) * eps)
            self.drift(U, pi, 0.5 * eps)
            self.kick(pi, U, phi, lam * eps)

    def trajectory(self, U, pi, phi, eps, nsteps, integrator='omelyan2'):
        """Evolves U and pi in place; returns (H0, H1)."""
        H0 = self.hamiltonian(U, pi, phi)
        (self.omelyan2 if integrator == 'omelyan2' else self.leapfrog)(U, pi, phi, eps, nsteps)
        return H0, self.hamiltonian(U, pi, phi)

    def refresh(self, U, w_momenta, eta):
        """pi = w^a T^a from Gaussian components w (device float64
        [..., 4, N^2-1]); phi = D-hat^+ eta from a Gaussian even field eta."""
        lat = self.lat
        pi = torch.empty(U.shape, dtype=torch.complex128, device=U.device)
        lat.algebra_from_components(pi, w_momenta.contiguous())
        phi = lat.new_half()
        if self.with_fermions:
            self._operator(U)
            if self.csw is None:
                lat.apply_dhat(phi, eta, self.UR, self.m0, dagger=1)
            else:
                lat.apply_dhat_clover(phi, eta, self.UR, self.clov, dagger=1)
        return pi, phi

    def update(self, U, eps, nsteps, generator, integrator='omelyan2'):
        """One HMC update of the single-lattice field U (in place): momenta
        with components pi^a ~ N(0, 1) (kinetic term sum tr pi^2 =
        sum_a (pi^a)^2 / 2), pseudofermion phi = D-hat^+ eta with complex
        Gaussian eta, E|eta_i|^2 = 1 (so that S_f(phi) = eta^+ eta), one
        trajectory, and the Metropolis test against a uniform draw.  The
        draws come from `generator` (a seeded torch.Generator on the GPU).
        Returns (dH, accepted)."""
        lat = self.lat
        N = lat.N
        dims = tuple(U.shape[:4])
        w = torch.randn(dims + (4, N * N - 1), dtype=torch.float64, device=U.device, generator=generator)
        eta_e = None
        if self.with_fermions:
            re = torch.randn((1,) + dims + (4, lat.d), dtype=torch.float64, device=U.device, generator=generator)
            im = torch.randn((1,) + dims + (4, lat.d), dtype=torch.float64, device=U.device, generator=generator)
            eta_e = lat.pack_half(torch.complex(re, im) * (0.5 ** 0.5), 0)
        pi, phi = self.refresh(U, w, eta_e)
        U0 = U.clone()
        H0, H1 = self.trajectory(U, pi, phi, eps, nsteps, integrator)
        dH = H1 - H0
        r = torch.rand((1,), dtype=torch.float64, device=U.device, generator=generator).item()
        accepted = dH <= 0.0 or r < math.exp(-dH)
        if not accepted:
            U.copy_(U0)
        return dH, accepted
