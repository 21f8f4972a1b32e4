"""Benchmark of the even-odd Wilson-Dirac hot path on one MI355X.

Workload: SU(3) fundamental fermions on a 32^4 lattice, FP64, links
exp(i 0.3 H) with H Gaussian traceless Hermitian, Gaussian source, m0 = -0.4,
antiperiodic in time.  One step is one pass of the whole path over that input:
represented links (FP64 and FP32), a batch of even-odd hops, the FP64 CG solve
to a true residual of 1e-10 and the mixed-precision CG solve to the same
residual.

Headline value: hop bandwidth on compulsory bytes (8 links + 1 input spinor
+ 1 output spinor per output site), from HIP events around back-to-back
dslash_eo launches on the stream they run on.  Also reported: the roofline of
the hop kernel against the 8 TB/s HBM peak, CG time-to-solution in FP64 and
mixed precision, and the CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--hops H] [--no-cpu]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = 'su3_fund_32x32x32x32'
TRAFFIC_FILE = os.path.join(ROOT, 'profiles', 'dslash_eo_su3_fund_32x32x32x32_traffic.json')
HOP_SOURCE = os.path.join(ROOT, 'paper_2503_06721_amd', 'csrc', 'hop.hip')


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def hop_bytes_per_site(d, real, prec_bytes):
    """Compulsory bytes per output site of one even-odd hop: the 8 links it
    multiplies (each link is used once per hop), one input spinor (each read
    by 8 neighbours but needed once) and one output spinor."""
    link = d * d * prec_bytes * (1 if real else 2)
    spinor = 4 * d * 2 * prec_bytes
    return 8 * link + 2 * spinor


def measured_traffic(launch_bytes):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if the hop kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        with open(HOP_SOURCE, 'rb') as f:
            h = hashlib.sha256(f.read()).hexdigest()
        if rec.get('hop_source_sha256') != h:
            return None
        return rec['hbm_bytes_per_launch']
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(cfg, U, psi, seconds_target=15.0):
    """The CPU oracle (NumPy, FP64) timed on a bounded sample: repeated D_eo
    applications on the full lattice until ~seconds_target have elapsed."""
    from oracle import dirac as OD
    from oracle import lattice as OL
    from oracle import reps as OR
    t0 = time.perf_counter()
    UR = OR.represent(U, cfg['rep'])
    t_rep = time.perf_counter() - t0
    psi_o = OL.to_half(psi, cfg['dims'], 1)
    n, t_hop = 0, 0.0
    while t_hop < seconds_target and n < 20:
        t0 = time.perf_counter()
        OD.D_eo(psi_o, UR, cfg['bc'], cfg['dims'])
        t_hop += time.perf_counter() - t0
        n += 1
    Vh = psi_o.shape[0]
    d = UR.shape[-1]
    gbs = hop_bytes_per_site(d, False, 8) * Vh * n / t_hop / 1e9
    return {'value': round(gbs, 4), 'unit': 'GB/s', 'cores': 1, 'kind': 'oracle',
            'sample': f'{n} oracle D_eo applications on the full {cfg["dims"]} lattice '
                      f'({t_hop:.1f} s; NumPy einsum/roll, single thread), plus one U->U_R in {t_rep:.1f} s',
            'seconds_per_hop': t_hop / n}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=3)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--hops', type=int, default=50, help='dslash_eo launches timed per step')
    ap.add_argument('--no-cpu', action='store_true', help='skip the CPU-oracle baseline')
    ap.add_argument('--no-cg', action='store_true', help='profiling aid: hops and links only')
    args = ap.parse_args()
    if args.gpus != 1:
        print(f'bench.py measures one GPU only; --gpus {args.gpus} is not supported '
              f'(the multi-GPU decomposition is a design, not part of this build)', file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2503_06721_amd import synth
    from paper_2503_06721_amd import wdirac as W

    cfg = synth.CONFIGS[WORKLOAD]
    dims, N, rep, m0, bc = cfg['dims'], cfg['N'], cfg['rep'], cfg['m0'], cfg['bc']
    log(f'[bench] generating inputs for {WORKLOAD}')
    U = synth.links_for(cfg)
    lat = W.Lattice(N, rep, dims, bc)
    d = lat.d
    psi = synth.gaussian_spinor((1,) + tuple(dims) + (4, d), cfg['seed'] + 1000)
    torch.cuda.set_device(0)
    Ug = torch.from_numpy(U).cuda()
    psig = torch.from_numpy(psi).cuda()
    UR64, UR32 = lat.new_links(W.F64), lat.new_links(W.F32)
    lat.rep_links(UR64, Ug, W.F64)
    lat.rep_links(UR32, Ug, W.F32)
    # the CG right-hand side: b = D-hat^dagger (source on the even sites)
    eta_e = lat.pack_half(psig, 0)
    b = lat.new_half()
    lat.apply_dhat(b, eta_e, UR64, m0, dagger=1)
    halves = [lat.pack_half(psig, 1), lat.new_half(), lat.new_half()]
    x64, xmix = lat.new_half(), lat.new_half()
    ws_cg = lat.new_workspace(W.OP_CG, 1, W.CG_MIXED)
    stream = torch.cuda.current_stream()

    bytes_per_launch = hop_bytes_per_site(d, lat.real, 8) * lat.Vh
    # the library's autotuner picks the hop launch shape for both precisions
    tuned = {'f64': lat.autotune(UR64, W.F64, 1), 'f32': lat.autotune(UR32, W.F32, 1)}
    log(f'[bench] autotuned hop shapes: {tuned}')
    variant_name = {W.HOP_SITE: 'k_hop_sp (lane per site)', W.HOP_COLOUR: 'k_hop_cs (colour-split)',
                    W.HOP_COLOUR_PAIR: 'k_hop_cs (colour-split, paired directions)'}

    def step(record):
        lat.rep_links(UR64, Ug, W.F64)
        lat.rep_links(UR32, Ug, W.F32)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k in range(args.hops):
            # alternate D_eo and D_oe so that every launch reads a fresh input
            src, dst = (halves[0], halves[1]) if k % 2 == 0 else (halves[1], halves[2])
            lat.dslash_eo(dst, src, UR64, 0 if k % 2 == 0 else 1)
        e1.record(stream)
        res = {}
        if not args.no_cg:
            x64.zero_()
            _, st64 = lat.cg_eo(x64, b, UR64, m0, tol=1e-10, maxit=20000, mode=W.CG_F64, workspace=ws_cg)
            xmix.zero_()
            _, stmx = lat.cg_eo(xmix, b, UR64, m0, tol=1e-10, maxit=20000, mode=W.CG_MIXED, UR32=UR32,
                                workspace=ws_cg)
            res = {'f64': st64[0], 'mixed': stmx[0]}
        torch.cuda.synchronize()
        if record is not None:
            record.append({'hop_ms': e0.elapsed_time(e1) / args.hops, **res})

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    log(f'[bench] warmup done; timing {args.steps} steps')
    recs = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(recs)
        log(f'[bench] step {k}: hop {recs[-1]["hop_ms"] * 1e3:.1f} us' +
            ('' if args.no_cg else f', CG f64 {recs[-1]["f64"]["seconds"]:.3f} s '
             f'({recs[-1]["f64"]["iters"]} it), mixed {recs[-1]["mixed"]["seconds"]:.3f} s'))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    hop_ms = float(np.mean([r['hop_ms'] for r in recs]))
    gbs = bytes_per_launch / (hop_ms * 1e-3) / 1e9
    traffic = measured_traffic(bytes_per_launch)
    out = {
        'metric': 'dslash_eo bandwidth on compulsory bytes (FP64)',
        'value': round(gbs, 2),
        'unit': 'GB/s',
        'n_gpus': 1,
        'steps': args.steps,
        'warmup': args.warmup,
        'ms_per_step': round(wall / args.steps * 1e3, 3),
        'higher_is_better': True,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': 'f64',
        'data': 'synthetic',
        'config': {'workload': WORKLOAD, 'gauge_group': f'SU({N})', 'representation': rep,
                   'lattice_TXYZ': list(dims), 'm0': m0, 'bc': list(bc),
                   'links': 'exp(i 0.3 H), H Gaussian traceless Hermitian', 'source': 'Gaussian',
                   'hops_per_step': args.hops},
        'roofline': {'bound': 'hbm', 'achieved': round(gbs, 2), 'peak': HBM_PEAK_GBS, 'unit': 'GB/s',
                     'frac': round(gbs / HBM_PEAK_GBS, 4),
                     'traffic': traffic,
                     'kernel': variant_name[tuned['f64']['variant']] + f' d=3 complex FP64, '
                               f'xcd_remap={tuned["f64"]["xcd_remap"]}',
                     'bytes_per_launch': bytes_per_launch, 'us_per_launch': round(hop_ms * 1e3, 3)},
    }
    if not args.no_cg:
        def agg(key):
            return {'seconds': round(float(np.median([r[key]['seconds'] for r in recs])), 4),
                    'iters': recs[-1][key]['iters'], 'reliable_updates': recs[-1][key]['reliable_updates'],
                    'true_rel_resid': recs[-1][key]['true_rel_resid'], 'hops': recs[-1][key]['hops'],
                    'status': W.STATUS_NAMES.get(recs[-1][key]['status'])}
        out['cg_time_to_1e-10'] = {'f64': agg('f64'), 'mixed': agg('mixed')}
        out['cg_time_to_1e-10']['mixed_speedup'] = round(
            out['cg_time_to_1e-10']['f64']['seconds'] / out['cg_time_to_1e-10']['mixed']['seconds'], 3)
    if not args.no_cpu:
        log('[bench] timing the CPU oracle on a bounded sample')
        cb = cpu_baseline(cfg, U, psi[0])
        cb.pop('seconds_per_hop')
        out['cpu_baseline'] = cb
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()
