"""The allocation-free D-hat entry point (wdirac_apply_dhat_noalloc) against
wdirac_apply_dhat, through the C ABI: two calls in a row on one GPU, the
second with a smaller input, in FP64 and FP32, must give bit-identical output
at every site to the workspace form (same kernels, same launch shapes); an input whose odd
field exceeds the fixed scratch is rejected on the host."""
import numpy as np
import pytest
import torch

from gpu_common import Setup, log, rel, wdirac
from oracle import dirac as D

pytestmark = pytest.mark.gpu


@pytest.fixture(scope='module')
def W():
    assert torch.cuda.is_available(), 'GPU tests need a GPU'
    return wdirac()


def run_pair(W, s, nrhs, prec, dagger, m, seed):
    psi = s.spinor(seed, nrhs)
    inp = s.to_gpu_half(psi, 0, prec)
    ref, got = s.lat.new_half(nrhs, prec), s.lat.new_half(nrhs, prec, zero=False)
    got.fill_(0xFF)      # any byte pattern: every site's element is written
    s.lat.apply_dhat(ref, inp, s.URg[prec], m, dagger, nrhs, prec)
    s.lat.apply_dhat_noalloc(got, inp, s.URg[prec], m, dagger, nrhs, prec)
    torch.cuda.synchronize()
    # the sites of the field (its rows may carry unused padding past them)
    a, b = s.from_gpu_half(got, 0, nrhs, prec), s.from_gpu_half(ref, 0, nrhs, prec)
    assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (nrhs, prec, dagger)
    return psi, got


@pytest.mark.parametrize('prec', [0, 1])
def test_noalloc_matches_workspace_form(W, prec):
    m = -0.4
    big = Setup(3, 'FUND', (16, 16, 16, 16), 1200, links='expH', precs=(prec,))
    small = Setup(3, 'FUND', (8, 4, 4, 8), 1201, links='expH', precs=(prec,))
    log(f'  prec {prec}: scratch {W.noalloc_scratch_bytes()} bytes; '
        f'first call {big.lat.field_bytes(W.FIELD_HALF_SPINOR, 3, prec)} bytes')
    psi1, got1 = run_pair(W, big, 3, prec, 0, m, 1202)
    # second call, smaller input: the scratch keeps the first call's contents
    psi2, got2 = run_pair(W, small, 1, prec, 1, m, 1203)
    # and against the oracle, to the parity tolerance
    tol = 1e-13 if prec == 0 else 1e-6
    x = small.half(psi2, 0)[0]
    exp = D.Dhat_dag(x, small.UR, m, small.bc, small.dims)
    err = rel(small.from_gpu_half(got2, 0, 1, prec)[0], exp)
    log(f'  second call vs oracle: {err:.2e}')
    assert err < tol


def test_noalloc_rejects_oversize(W):
    """SU(3) SYM 48x24^3 in FP64: the odd field (127 MB) exceeds the 64 MiB
    scratch; the call fails on the host with EINVAL and launches nothing."""
    lat = W.Lattice(3, 'SYM', (48, 24, 24, 24))
    need = lat.field_bytes(W.FIELD_HALF_SPINOR, 1, W.F64)
    assert need > W.noalloc_scratch_bytes()
    out, inp = lat.new_half(), lat.new_half()
    UR = lat.new_links(W.F64)
    with pytest.raises(W.WdiracError) as e:
        lat.apply_dhat_noalloc(out, inp, UR, -0.4)
    assert e.value.code == W.EINVAL and 'scratch' in str(e.value)
    assert np.count_nonzero(out.cpu().numpy()) == 0
