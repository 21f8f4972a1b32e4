"""Full-size solves checked by the oracle's own operator.

Every solver result here is the library's x, copied back; the residual
b - A x with A = D-hat^+ D-hat (Sec. 5.3.3) is recomputed on the host by the
oracle (NumPy FP64, full 4x4 spin products), from the oracle's own links and
sources, and must satisfy the paper's stopping criterion read as
||b - A x||_2 / ||b||_2 <= 1e-10.  The relative max norm (Sec. 4.2.2: over
real and imaginary parts) is reported beside it.  For a right-hand side of
the form b = D-hat^+ s the residual is formed as D-hat^+ (s - D-hat x), the
same vector with two oracle hops fewer.

Workloads, in the launch shapes the benchmark times (the autotuner's pick):
  * SU(3) FUND 32^4, b = D-hat^+ eta_e: FP64 and mixed CG;
  * SU(3) SYM 48x24^3, 12 point sources at the origin solved in one batched
    call, b_k = D-hat^+ (4+m0) eta_k: three of the twelve solutions, FP64 and
    mixed;
  * the batch SU(3) SYM 8^4 + 12^4 + 32x16^3 in one launch per kernel,
    b = Gaussian even source per lattice: every lattice, FP64 and mixed;
  * SU(4) 2AS on 4x48^3 -- the per-site shape of the SU(4) 2AS 96x48^3
    workload (d_R = 6, N = 4, the same spatial extent and link recipe) on a
    lattice the oracle can hold -- b = D-hat^+ eta_e: FP64 and mixed.

Oracle residuals run in host threads (NumPy releases the interpreter lock in
its array loops)."""
import concurrent.futures
import math

import numpy as np
import pytest
import torch

from gpu_common import log, relmax, wdirac
from oracle import dirac as D
from oracle import lattice as L
from oracle import reps as R
from oracle.reductions import norm2
from paper_2503_06721_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-10
# the oracle recomputes the residual in a different summation order than the
# library: a relative change of the residual far below 1e-3 is rounding
SLACK = 1.001


@pytest.fixture(scope='module')
def W():
    assert torch.cuda.is_available(), 'GPU tests need a GPU'
    return wdirac()


def host_half(lat, packed, parity, dims):
    """Oracle half field (V/2, 4, d) of one packed right-hand side."""
    full = lat.unpack_half(packed, parity, 1).cpu().numpy()[0]
    return L.to_half(full, dims, parity)


def residual_dagger_form(x, s, UR, m, bc, dims):
    """b - A x for b = D-hat^+ s: D-hat^+ (s - D-hat x) (oracle operator)."""
    return D.Dhat_dag(s - D.Dhat(x, UR, m, bc, dims), UR, m, bc, dims)


def residual_plain(x, b, UR, m, bc, dims):
    return b - D.normal_op(x, UR, m, bc, dims)


def report(tag, r, b, st):
    """Relative 2-norm and max norm (over real and imaginary parts) of the
    residual r for the right-hand side b, logged beside the library's own."""
    res = math.sqrt(norm2(r) / norm2(b))
    rinf = relmax(b - r, b)      # = ||r||_inf / ||b||_inf
    log(f'  {tag}: oracle residual {res:.3e} (library {st["true_rel_resid"]:.3e}), max-norm ratio {rinf:.3e}, '
        f'{st["iters"]} iterations, {st["seconds"]:.3f} s')
    return res, rinf


def run_parallel(jobs):
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        futs = {k: ex.submit(f) for k, f in jobs.items()}
        return {k: f.result() for k, f in futs.items()}


def gpu_lattice(W, cfg, U):
    lat = W.Lattice(cfg['N'], cfg['rep'], cfg['dims'], cfg['bc'])
    Ug = torch.from_numpy(U).cuda()
    UR64, UR32 = lat.new_links(W.F64), lat.new_links(W.F32)
    lat.rep_links(UR64, Ug, W.F64)
    lat.rep_links(UR32, Ug, W.F32)
    return lat, UR64, UR32


def solve_both(W, lat, b, UR64, UR32, m0, nrhs=1):
    """FP64 and mixed solves from x0 = 0, in the tuned launch shapes."""
    lat.autotune(UR64, W.F64, nrhs)
    lat.autotune(UR32, W.F32, nrhs)
    ws = lat.new_workspace(W.OP_CG, nrhs, W.CG_MIXED)
    out = {}
    for mode, key in ((W.CG_F64, 'f64'), (W.CG_MIXED, 'mixed')):
        x = lat.new_half(nrhs)
        rc, st = lat.cg_eo(x, b, UR64, m0, tol=TOL, maxit=20000, nrhs=nrhs, mode=mode, UR32=UR32, workspace=ws)
        assert rc == W.OK, (key, st)
        out[key] = (x, st)
    return out


def test_su3_fund_32x32x32x32(W):
    cfg = synth.CONFIGS['su3_fund_32x32x32x32']
    dims, m0, bc = cfg['dims'], cfg['m0'], cfg['bc']
    log('SU(3) FUND 32^4: inputs')
    U = synth.links_for(cfg)
    eta = synth.gaussian_spinor((1,) + tuple(dims) + (4, 3), cfg['seed'] + 1000)
    lat, UR64, UR32 = gpu_lattice(W, cfg, U)
    eta_e = lat.pack_half(torch.from_numpy(eta).cuda(), 0)
    b = lat.new_half()
    lat.apply_dhat(b, eta_e, UR64, m0, dagger=1)
    sol = solve_both(W, lat, b, UR64, UR32, m0)
    xs = {k: host_half(lat, v[0], 0, dims) for k, v in sol.items()}
    del lat, UR64, UR32, b, eta_e
    sol_gpu_free(sol)
    log('  oracle residuals')
    UR = R.represent(U, cfg['rep'])
    s = L.to_half(eta[0], dims, 0)
    b_or = D.Dhat_dag(s, UR, m0, bc, dims)
    res = run_parallel({k: (lambda x=x: residual_dagger_form(x, s, UR, m0, bc, dims)) for k, x in xs.items()})
    for k, r in res.items():
        v, _ = report(k, r, b_or, sol[k][1][0])
        assert v <= TOL * SLACK, (k, v)


def sol_gpu_free(sol):
    """Drop the device copies of the solutions (host copies are taken)."""
    for k in list(sol):
        sol[k] = (None, sol[k][1])
    torch.cuda.empty_cache()
    return None


@pytest.fixture(scope='module')
def sym_point_sources(W):
    """SU(3) SYM 48x24^3, 12 point sources: one batched FP64 solve and one
    batched mixed solve; host copies of three solutions per mode."""
    cfg = synth.CONFIGS['su3_sym_48x24x24x24']
    dims, m0, nrhs = cfg['dims'], cfg['m0'], cfg['nrhs']
    log('SU(3) SYM 48x24^3, 12 point sources: inputs')
    U = synth.links_for(cfg)
    src = synth.point_sources(dims, 6, nrhs)
    lat, UR64, UR32 = gpu_lattice(W, cfg, U)
    srcg = torch.from_numpy(src).cuda()
    eta_e, eta_o = lat.pack_half(srcg, 0, nrhs), lat.pack_half(srcg, 1, nrhs)
    bp, b = lat.new_half(nrhs), lat.new_half(nrhs)
    lat.eo_source(bp, eta_e, eta_o, UR64, m0, nrhs)
    lat.apply_dhat(b, bp, UR64, m0, dagger=1, nrhs=nrhs)
    del srcg, eta_e, eta_o, bp
    sol = solve_both(W, lat, b, UR64, UR32, m0, nrhs)
    per = sol['f64'][0].numel() // nrhs
    picks = {'f64': (0, 11), 'mixed': (5,)}
    xs = {}
    for key, ks in picks.items():
        for k in ks:
            xs[(key, k)] = (host_half(lat, sol[key][0][k * per:(k + 1) * per], 0, dims), sol[key][1][k])
    del lat, UR64, UR32, b, sol
    torch.cuda.empty_cache()
    UR = R.represent(U, cfg['rep'])
    return cfg, UR, src, xs


def test_su3_sym_48x24x24x24_point_sources(sym_point_sources):
    """Three of the twelve batched solutions (two FP64, one mixed) against the
    oracle: the origin is even, so the even-odd source is (4+m0) eta_e and
    b = D-hat^+ (4+m0) eta_e."""
    cfg, UR, src, xs = sym_point_sources
    dims, m0, bc = cfg['dims'], cfg['m0'], cfg['bc']
    jobs = {}
    for (key, k), (x, st) in xs.items():
        s = (4.0 + m0) * L.to_half(src[k], dims, 0)
        jobs[(key, k)] = (lambda x=x, s=s: (residual_dagger_form(x, s, UR, m0, bc, dims),
                                            D.Dhat_dag(s, UR, m0, bc, dims)))
    log('  oracle residuals of three solutions')
    res = run_parallel(jobs)
    for (key, k), (r, b_or) in res.items():
        v, _ = report(f'{key} source {k}', r, b_or, xs[(key, k)][1])
        assert v <= TOL * SLACK, (key, k, v)


def test_lattice_batch_sym(W):
    """SU(3) SYM batch 8^4 + 12^4 + 32x16^3 (one launch per kernel, the
    benchmark's batch): every lattice's FP64 and mixed solution."""
    shapes = [(8, 8, 8, 8), (12, 12, 12, 12), (32, 16, 16, 16)]
    m0, bc, seed = -0.4, (-1, 1, 1, 1), 1003
    Us = [synth.expH_links(dd, 3, 0.3, seed + 10 + k) for k, dd in enumerate(shapes)]
    etas = [synth.gaussian_spinor((1,) + dd + (4, 6), seed + 20 + k) for k, dd in enumerate(shapes)]
    lat = W.Lattice(3, 'SYM', shapes, bc)
    UR64, UR32 = lat.new_links(W.F64), lat.new_links(W.F32)
    Ug = torch.cat([torch.from_numpy(u).reshape(-1, 4, 3, 3) for u in Us]).cuda()
    lat.rep_links(UR64, Ug, W.F64)
    lat.rep_links(UR32, Ug, W.F32)
    b = lat.pack_half(torch.cat([torch.from_numpy(e).reshape(-1, 4, 6) for e in etas]).cuda(), 0)
    sol = solve_both(W, lat, b, UR64, UR32, m0)
    offs = np.cumsum([0] + [int(np.prod(dd)) for dd in shapes])
    jobs, stats = {}, {}
    for key, (x, st) in sol.items():
        full = lat.unpack_half(x, 0).cpu().numpy()
        for k, dd in enumerate(shapes):
            xk = L.to_half(full[offs[k]:offs[k + 1]].reshape(dd + (4, 6)), dd, 0)
            bk = L.to_half(etas[k][0], dd, 0)
            URk = R.represent(Us[k], 'SYM')
            jobs[(key, k)] = (lambda xk=xk, bk=bk, URk=URk, dd=dd: (residual_plain(xk, bk, URk, m0, bc, dd), bk))
            stats[(key, k)] = st[k]
    res = run_parallel(jobs)
    for (key, k), (r, bk) in sorted(res.items()):
        v, _ = report(f'{key} lattice {shapes[k]}', r, bk, stats[(key, k)])
        assert v <= TOL * SLACK, (key, k, v)


def test_su4_2as_t_reduced(W):
    """SU(4) 2AS with the per-site shape of the 96x48^3 workload on 4x48^3
    (links exp(i 0.3 H), m0 = -0.3, b = D-hat^+ eta_e): FP64 and mixed."""
    base = synth.CONFIGS['su4_2as_96x48x48x48']
    cfg = dict(base, dims=(4, 48, 48, 48))
    dims, m0, bc = cfg['dims'], cfg['m0'], cfg['bc']
    log('SU(4) 2AS 4x48^3: inputs')
    U = synth.expH_links(dims, 4, cfg['eps'], cfg['seed'])
    eta = synth.gaussian_spinor((1,) + dims + (4, 6), cfg['seed'] + 11)
    lat, UR64, UR32 = gpu_lattice(W, cfg, U)
    eta_e = lat.pack_half(torch.from_numpy(eta).cuda(), 0)
    b = lat.new_half()
    lat.apply_dhat(b, eta_e, UR64, m0, dagger=1)
    sol = solve_both(W, lat, b, UR64, UR32, m0)
    xs = {k: host_half(lat, v[0], 0, dims) for k, v in sol.items()}
    del lat, UR64, UR32, b, eta_e
    sol_gpu_free(sol)
    log('  oracle residuals')
    UR = R.represent(U, cfg['rep'])
    s = L.to_half(eta[0], dims, 0)
    b_or = D.Dhat_dag(s, UR, m0, bc, dims)
    res = run_parallel({k: (lambda x=x: residual_dagger_form(x, s, UR, m0, bc, dims)) for k, x in xs.items()})
    for k, r in res.items():
        v, _ = report(k, r, b_or, sol[k][1][0])
        assert v <= TOL * SLACK, (k, v)
