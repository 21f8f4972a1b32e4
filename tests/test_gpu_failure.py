"""Failure handling of the solvers on the GPU: a non-finite right-hand side and
an exactly singular operator must end in WDIRAC_EBREAKDOWN or
WDIRAC_ENOCONV with the statistics filled, never in a silent OK or a hang.
Every case is forced from the host through the inputs, with a small maxit, so
that every kernel runs to its normal end.

The singular case: with unit links, m0 = 0 and periodic boundaries the
constant spinor is an exact zero mode of the Wilson operator (free-field
eigenvalue m0 + sum_mu (1 - cos p_mu) at p = 0, Sec. 2.3), so the constant
even field lies in the null space of D-hat = (4+m0)^2 - D_eo D_oe (each hop
maps it to -4 times itself), and <p, A p> = ||D-hat p||^2 vanishes at the
first step of CG."""
import math

import numpy as np
import pytest
import torch

from gpu_common import log, wdirac
from paper_2503_06721_amd import synth

pytestmark = pytest.mark.gpu

DIMS = (4, 4, 4, 4)
PERIODIC = (1, 1, 1, 1)


@pytest.fixture(scope='module')
def W():
    assert torch.cuda.is_available(), 'GPU tests need a GPU'
    return wdirac()


def unit_links(dims, N):
    U = np.zeros(tuple(dims) + (4, N, N), dtype=np.complex128)
    U[..., :, :] = np.eye(N)
    return U


def setup(W, links, N=2, rep='FUND', bc=(-1, 1, 1, 1)):
    lat = W.Lattice(N, rep, DIMS, bc)
    UR64, UR32 = lat.new_links(W.F64), lat.new_links(W.F32)
    Ug = torch.from_numpy(links).cuda()
    lat.rep_links(UR64, Ug, W.F64)
    lat.rep_links(UR32, Ug, W.F32)
    return lat, UR64, UR32


def with_nan(lat, b_full, rhs):
    """Packed even field of b_full with one NaN planted in right-hand side `rhs`."""
    bad = b_full.copy()
    bad[rhs, 0, 0, 0, 0, 0, 0] = complex(math.nan, 0.0)
    return lat.pack_half(torch.from_numpy(bad).cuda(), 0, bad.shape[0])


@pytest.mark.parametrize('mode', [0, 1])
def test_cg_nan_source(W, mode):
    """A NaN in one right-hand side: that system reports EBREAKDOWN after zero
    iterations, the other one converges as usual, and the call returns
    EBREAKDOWN."""
    lat, UR64, UR32 = setup(W, synth.haar_links(DIMS, 2, 1000))
    b = synth.gaussian_spinor((2,) + DIMS + (4, lat.d), 2000)
    bg = with_nan(lat, b, 1)
    x = lat.new_half(2)
    rc, st = lat.cg_eo(x, bg, UR64, -0.2, tol=1e-10, maxit=500, nrhs=2, mode=mode, UR32=UR32)
    log(f'  mode {mode}: rc {rc}, stats {st}')
    assert rc == W.EBREAKDOWN
    assert st[1]['status'] == W.EBREAKDOWN and st[1]['iters'] == 0
    assert st[0]['status'] == W.OK and st[0]['true_rel_resid'] <= 1e-10
    assert 0 < st[0]['iters'] <= 500
    assert all(math.isfinite(s['seconds']) for s in st)


@pytest.mark.parametrize('mode', [0, 1])
def test_cg_exact_zero_mode(W, mode):
    """Constant even source on the periodic free field at m0 = 0: the source
    lies in the null space of A, so CG meets <p, A p> = 0 and stops with
    EBREAKDOWN (or, had rounding left <p, A p> > 0, with ENOCONV at maxit)."""
    lat, UR64, UR32 = setup(W, unit_links(DIMS, 2), bc=PERIODIC)
    b = np.ones((1,) + DIMS + (4, lat.d), dtype=np.complex128)
    bg = lat.pack_half(torch.from_numpy(b).cuda(), 0)
    x = lat.new_half()
    maxit = 40
    rc, st = lat.cg_eo(x, bg, UR64, 0.0, tol=1e-10, maxit=maxit, mode=mode, UR32=UR32)
    log(f'  mode {mode}: rc {rc}, stats {st}')
    assert rc in (W.EBREAKDOWN, W.ENOCONV)
    assert st[0]['status'] == rc and 0 <= st[0]['iters'] <= maxit
    # the operator really annihilates the source (exact in this arithmetic)
    u = lat.new_half()
    lat.apply_dhat(u, bg, UR64, 0.0)
    assert lat.norm2(u)[0] == 0.0


def test_cg_inconsistent_singular_system(W):
    """Gaussian source on the same singular operator: it has a component in
    the null space that no x can remove, so the solve ends at maxit with
    ENOCONV and a true residual far above the tolerance."""
    lat, UR64, _ = setup(W, unit_links(DIMS, 2), bc=PERIODIC)
    b = synth.gaussian_spinor((1,) + DIMS + (4, lat.d), 2001)
    bg = lat.pack_half(torch.from_numpy(b).cuda(), 0)
    x = lat.new_half()
    rc, st = lat.cg_eo(x, bg, UR64, 0.0, tol=1e-10, maxit=60)
    log(f'  rc {rc}, stats {st}')
    assert rc in (W.ENOCONV, W.EBREAKDOWN)
    if rc == W.ENOCONV:
        assert st[0]['iters'] == 60 and st[0]['true_rel_resid'] > 1e-6


def test_mshift_nan_source(W):
    """Multi-shift CG with a NaN in b: every shift reports EBREAKDOWN."""
    lat, UR64, _ = setup(W, synth.haar_links(DIMS, 2, 1000))
    b = synth.gaussian_spinor((1,) + DIMS + (4, lat.d), 2002)
    bg = with_nan(lat, b, 0)
    shifts = [0.0, 0.1, 1.0]
    x = lat.new_shift_fields(len(shifts))
    rc, st = lat.cg_mshift_eo(x, bg, UR64, -0.2, shifts, tol=1e-10, maxit=200)
    log(f'  rc {rc}, stats {st}')
    assert rc == W.EBREAKDOWN
    assert all(s['status'] == W.EBREAKDOWN and 0 <= s['iters'] <= 200 for s in st)


def test_mshift_exact_zero_mode(W):
    """Multi-shift CG on the singular free-field operator with the smallest
    shift zero and a constant source: breakdown at the first step."""
    lat, UR64, _ = setup(W, unit_links(DIMS, 2), bc=PERIODIC)
    b = np.ones((1,) + DIMS + (4, lat.d), dtype=np.complex128)
    bg = lat.pack_half(torch.from_numpy(b).cuda(), 0)
    shifts = [0.0, 0.5]
    x = lat.new_shift_fields(len(shifts))
    rc, st = lat.cg_mshift_eo(x, bg, UR64, 0.0, shifts, tol=1e-10, maxit=40)
    log(f'  rc {rc}, stats {st}')
    assert rc in (W.EBREAKDOWN, W.ENOCONV)
    assert all(s['status'] in (W.EBREAKDOWN, W.ENOCONV) and s['iters'] <= 40 for s in st)
