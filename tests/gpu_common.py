"""Shared helpers of the GPU parity tests: seeded inputs on both sides, the
oracle's expected values, and comparisons.  Nothing here computes any part of
the operator; expected values come from oracle/, results from libwdirac."""
import importlib
import sys

import numpy as np

from oracle import lattice as L
from oracle import reps as R
from paper_2503_06721_amd import synth

APBC = (-1, 1, 1, 1)
TOL = {0: 1e-13, 1: 1e-6}          # relative 2-norm, FP64 / FP32


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def wdirac():
    return importlib.import_module('paper_2503_06721_amd.wdirac')


def rel2(a, b):
    """||a - b||_2 / ||b||_2 over the whole output."""
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def relmax(a, b):
    """||a - b||_inf / ||b||_inf, the max norm taken over real and imaginary
    parts separately (the norm of the paper's Sec. 4.2.2)."""
    d = np.asarray(a) - np.asarray(b)
    b = np.asarray(b)
    parts = lambda v: np.concatenate([np.real(v).ravel(), np.imag(v).ravel()]) if np.iscomplexobj(v) else v.ravel()
    nb = np.abs(parts(b)).max() if b.size else 0.0
    return (np.abs(parts(d)).max() if d.size else 0.0) / (nb if nb > 0 else 1.0)


def rel(a, b):
    """Parity metric: the larger of the relative 2-norm and the relative max
    norm, so that one tolerance bounds both (a few wrong elements in a large
    output move the max norm even where the 2-norm hides them)."""
    return max(rel2(a, b), relmax(a, b))


class Setup:
    """Links, represented links (oracle and GPU) for one (N, rep, dims)."""

    def __init__(self, N, rep, dims, seed, links='haar', bc=APBC, eps=0.3, precs=(0, 1)):
        import torch
        W = wdirac()
        self.W = W
        self.N, self.rep, self.dims, self.bc = N, rep, tuple(dims), tuple(bc)
        self.U = synth.haar_links(dims, N, seed) if links == 'haar' else synth.expH_links(dims, N, eps, seed)
        self.UR = R.represent(self.U, rep)                      # oracle
        self.d = self.UR.shape[-1]
        self.lat = W.Lattice(N, rep, dims, bc)
        self.Ug = torch.from_numpy(self.U).cuda()
        self.URg = {}
        for p in precs:
            self.URg[p] = self.lat.new_links(p)
            self.lat.rep_links(self.URg[p], self.Ug, p)

    def spinor(self, seed, nrhs=1):
        return synth.gaussian_spinor((nrhs,) + self.dims + (4, self.d), seed)

    def half(self, full, parity):
        """Oracle half fields (nrhs, Vh, 4, d) of a batch of full fields."""
        return np.stack([L.to_half(f, self.dims, parity) for f in full])

    def to_gpu_half(self, full, parity, prec=0):
        import torch
        dt = np.complex128 if prec == 0 else np.complex64
        t = torch.from_numpy(np.ascontiguousarray(full.astype(dt))).cuda()
        return self.lat.pack_half(t, parity, full.shape[0], prec)

    def from_gpu_half(self, packed, parity, nrhs=1, prec=0):
        canon = self.lat.unpack_half(packed, parity, nrhs, prec).cpu().numpy().astype(np.complex128)
        return self.half(canon, parity)
