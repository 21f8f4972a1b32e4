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
mixed precision, and the CPU oracle timed on a bounded sample.  Once per run,
after the timed steps: 12 point sources on SU(3) SYM 48x24^3 solved as one
batched call and as 12 single calls (FP64 and mixed), FP64 against mixed CG on
SU(4) 2AS 96x48^3, the three-lattice SU(3) SYM batch against separate solves,
the force on SU(2) ADJ 32x16^3, on the benchmark lattice a 12-shift
multi-shift solve and the clover-improved CG, and one HMC trajectory on
SU(2) ADJ 32x16^3.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--hops H] [--no-cpu] [--no-multi]
"""
import argparse
import csv
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
HOP_SOURCES = [os.path.join(ROOT, 'paper_2503_06721_amd', 'csrc', f)
               for f in ('hop.hip', 'hop_mr.hip', 'wd_hop.h', 'wd_common.h')]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def hop_bytes_per_site(d, real, prec_bytes):
    """Compulsory bytes per output site of one even-odd hop: the 8 links it
    multiplies (each link is used once per hop), one input spinor (each read
    by 8 neighbours but needed once) and one output spinor."""
    link = d * d * prec_bytes * (1 if real else 2)
    spinor = 4 * d * 2 * prec_bytes
    return 8 * link + 2 * spinor


def effective_bytes_per_site(d, real, prec_bytes):
    """The paper's "effective" byte count per output site: 8 links, 8
    neighbour spinors and the output spinor, as if nothing were cached."""
    link = d * d * prec_bytes * (1 if real else 2)
    spinor = 4 * d * 2 * prec_bytes
    return 8 * link + 9 * spinor


def device_copy_gbps(torch, n=1 << 28, reps=3):
    """Read + write bandwidth of a 2 GiB device-to-device copy (HIP events)."""
    a = torch.ones(n, dtype=torch.float64, device='cuda')
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return ms, 2 * n * 8 / ms / 1e6


def hop_sources_sha256():
    """SHA-256 over the sources of the hop kernels and the link layout they
    read (hop.hip, hop_mr.hip, wd_hop.h, wd_common.h, in that order): a
    traffic record taken on other sources no longer applies."""
    h = hashlib.sha256()
    for p in HOP_SOURCES:
        with open(p, 'rb') as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(launch_bytes, shape):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if the hop kernel source changed since the counters were taken or
    the autotuner picked another launch shape than the one they were taken on."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        h = hop_sources_sha256()
        if rec.get('hop_sources_sha256') != h:
            return None
        for row in rec.get('per_launch_shape', []):
            if all(shape.get(k) == v for k, v in row['launch_shape'].items()):
                return row['hbm_bytes_per_launch']
        return None
    except (OSError, KeyError, ValueError):
        return None


def _counter_per_dispatch(path, counter):
    """(dispatch id, kernel name, value) of one rocprofv3 counter, summed over
    the rows of a dispatch, in dispatch order."""
    acc = {}
    with open(path, newline='') as f:
        for r in csv.DictReader(f):
            if r['Counter_Name'] == counter:
                k = int(r['Dispatch_Id'])
                name, v = acc.get(k, (r['Kernel_Name'], 0.0))
                acc[k] = (name, v + float(r['Counter_Value']))
    return [(k, n, v) for k, (n, v) in sorted(acc.items())]


def _calibration(cal, fetch_csv, write_csv):
    """Bytes per counted KiB of FETCH_SIZE and WRITE_SIZE for each kernel of
    known traffic in the calibration run."""
    fetch = _counter_per_dispatch(fetch_csv, 'FETCH_SIZE')
    write = _counter_per_dispatch(write_csv, 'WRITE_SIZE')
    out = {}
    for k in cal['kernels']:
        fv = [v for _, n, v in fetch if k['pattern'] in n]
        wv = [v for _, n, v in write if k['pattern'] in n]
        if not fv or not wv:
            raise SystemExit(f'calibration kernel {k["pattern"]} not found in the counter files')
        f_kib, w_kib = sum(fv) / len(fv), sum(wv) / len(wv)
        out[k['name']] = {'kernel_pattern': k['pattern'], 'dispatches': len(fv),
                          'bytes_read': k['bytes_read'], 'bytes_written': k['bytes_written'],
                          'fetch_size_kib': round(f_kib, 1), 'write_size_kib': round(w_kib, 1),
                          'fetch_factor': round(k['bytes_read'] / (f_kib * 1024), 4),
                          'write_factor': round(k['bytes_written'] / (w_kib * 1024), 4)}
    return out


def write_traffic_record(out_path, run_json, fetch_csv, write_csv, cal_json, cal_fetch_csv, cal_write_csv):
    """Per-launch HBM traffic of the hop for every launch shape of a
    --traffic-shapes / --traffic-multi run, from its FETCH_SIZE and WRITE_SIZE
    counter passes, calibrated on the kernels of known traffic of a
    --copy-calibration run (a device copy and the non-temporal streaming
    probe, whose loads are of the hop's kind; the probe's factors are the ones
    applied, the copy's are shown beside them).  The record carries the
    SHA-256 of the hop sources it was taken on."""
    with open(run_json) as f:
        run = json.load(f)
    with open(cal_json) as f:
        cal = _calibration(json.load(f), cal_fetch_csv, cal_write_csv)
    ff, wf = cal['stream_probe']['fetch_factor'], cal['stream_probe']['write_factor']
    pat, per = run['kernel_pattern'], run['launches_per_shape']
    fetch = [r for r in _counter_per_dispatch(fetch_csv, 'FETCH_SIZE') if pat in r[1]]
    write = [r for r in _counter_per_dispatch(write_csv, 'WRITE_SIZE') if pat in r[1]]
    need = per * len(run['shapes'])
    if len(fetch) < need or len(write) < need:
        raise SystemExit(f'{len(fetch)} / {len(write)} hop dispatches in the counter files, {need} expected')
    fetch, write = fetch[-need:], write[-need:]
    algo = run['algorithmic_bytes_per_launch']
    rows = []
    for i, shape in enumerate(run['shapes']):
        fr, wr = fetch[i * per:(i + 1) * per], write[i * per:(i + 1) * per]
        f_kib = sum(v for _, _, v in fr) / per
        w_kib = sum(v for _, _, v in wr) / per
        hbm = f_kib * 1024 * ff + w_kib * 1024 * wf
        rows.append({'launch_shape': shape, 'kernel': fr[0][1],
                     'fetch_size_kib_per_launch': round(f_kib, 1), 'write_size_kib_per_launch': round(w_kib, 1),
                     'raw_bytes_per_launch': int(round((f_kib + w_kib) * 1024)),
                     'hbm_bytes_per_launch': int(round(hbm)),
                     'traffic_over_algorithmic': round(hbm / algo, 4),
                     'reads_over_compulsory_reads': round(f_kib * 1024 * ff / run['compulsory_read_bytes'], 4)})
    rec = {'workload': run['workload'], 'hop_sources_sha256': run['hop_sources_sha256'],
           'calibration': cal, 'factors_applied': {'fetch': ff, 'write': wf, 'from': 'stream_probe'},
           'algorithmic_bytes_per_launch': algo, 'compulsory_read_bytes': run['compulsory_read_bytes'],
           'per_launch_shape': rows}
    with open(out_path, 'w') as f:
        json.dump(rec, f, indent=1)
        f.write('\n')
    print(json.dumps({'written': out_path, 'shapes': len(rows)}))


def kernel_durations(trace_csv, pattern, last):
    """Dispatch count and mean duration of the kernels whose name contains
    `pattern` in a rocprofv3 kernel_trace.csv, and the mean, median, min and
    max over the last `last` of them (the benchmark's timed launches)."""
    import statistics
    rows = []
    with open(trace_csv, newline='') as f:
        for r in csv.DictReader(f):
            if pattern in r['Kernel_Name']:
                rows.append((int(r['Dispatch_Id']), int(r['End_Timestamp']) - int(r['Start_Timestamp']),
                             r['Kernel_Name']))
    if not rows:
        raise SystemExit(f'no dispatch of {pattern!r} in {trace_csv}')
    rows.sort()
    d = [x[1] for x in rows]
    t = d[-last:]
    return (f'kernel: {rows[-1][2]}\n'
            f'dispatches: {len(d)}, mean over all: {statistics.mean(d):.0f} ns\n'
            f'last {len(t)} dispatches: mean {statistics.mean(t):.0f} ns, median {statistics.median(t):.0f} ns, '
            f'min {min(t)} ns, max {max(t)} ns')


def host_info():
    """The host the CPU baseline ran on: CPU model, logical CPUs, the CPUs this
    process may use, and the thread settings NumPy sees."""
    model = None
    try:
        with open('/proc/cpuinfo') as f:
            for line in f:
                if line.startswith('model name'):
                    model = line.split(':', 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = None
    return {'cpu_model': model, 'nproc': os.cpu_count(), 'usable_cpus': usable,
            'OMP_NUM_THREADS': os.environ.get('OMP_NUM_THREADS'),
            'threads_used': 1,
            'threads_note': 'the oracle is NumPy einsum/roll/elementwise code, which runs on one thread'}


BATCH_SHAPES = [(8, 8, 8, 8), (12, 12, 12, 12), (32, 16, 16, 16)]
BATCH_M0, BATCH_SEED = -0.4, 1003


def batch_inputs(synth):
    """Links and Gaussian sources of the three-lattice SU(3) SYM batch."""
    Us = [synth.expH_links(dd, 3, 0.3, BATCH_SEED + 10 + k) for k, dd in enumerate(BATCH_SHAPES)]
    etas = [synth.gaussian_spinor((1,) + dd + (4, 6), BATCH_SEED + 20 + k) for k, dd in enumerate(BATCH_SHAPES)]
    return Us, etas


def small_systems(synth):
    """The CG systems timed on both sides besides the benchmark lattice:
    SU(2) FUND 4^4, SU(2) ADJ 32x16^3 and each lattice of the SU(3) SYM batch,
    b = the even half of a Gaussian spinor.  Returns name -> (N, rep, dims,
    bc, m0, U, eta)."""
    out = {}
    for name in ('su2_fund_4x4x4x4', 'su2_adj_32x16x16x16'):
        cfg = synth.CONFIGS[name]
        d = {'FUND': cfg['N'], 'ADJ': cfg['N'] ** 2 - 1}[cfg['rep']]
        out[name] = (cfg['N'], cfg['rep'], cfg['dims'], cfg['bc'], cfg['m0'], synth.links_for(cfg),
                     synth.gaussian_spinor((1,) + tuple(cfg['dims']) + (4, d), cfg['seed'] + 1000))
    Us, etas = batch_inputs(synth)
    for k, dd in enumerate(BATCH_SHAPES):
        out['su3_sym_' + 'x'.join(map(str, dd))] = (3, 'SYM', dd, (-1, 1, 1, 1), BATCH_M0, Us[k], etas[k])
    return out


def gpu_small_solves(W, torch, systems):
    """FP64 CG to 1e-10 on the GPU for each small system (autotuned hop, one
    warm-up solve, then the median of three)."""
    out = {}
    for name, (N, rep, dims, bc, m0, U, eta) in systems.items():
        lat = W.Lattice(N, rep, dims, bc)
        UR = lat.new_links(W.F64)
        lat.rep_links(UR, torch.from_numpy(U).cuda())
        b = lat.pack_half(torch.from_numpy(eta).cuda(), 0)
        lat.autotune(UR, W.F64, 1)
        x = lat.new_half()
        secs = []
        for k in range(4):
            x.zero_()
            rc, st = lat.cg_eo(x, b, UR, m0, tol=1e-10, maxit=20000)
            if k:
                secs.append(st[0]['seconds'])
        out[name] = {'seconds': round(float(sorted(secs)[1]), 5), 'iters': st[0]['iters'],
                     'status': W.STATUS_NAMES.get(rc)}
    return out


def cpu_baseline(cfg, U, psi, gpu_c1, systems, gpu_small):
    """The CPU oracle (NumPy, FP64, one thread) on a bounded sample, beside
    the GPU:
      * hop rate: two oracle D_eo applications on the benchmark lattice
        (compulsory bytes per second, as the GPU's value);
      * CG time-to-1e-10: the whole oracle CG on SU(2) FUND 4^4; on the
        larger lattices one oracle application of A = D-hat^+ D-hat (the
        cost of one CG iteration, less its few vector operations) times the
        GPU's iteration count for the same system, a lower bound of the
        oracle's time to solution."""
    from oracle import cg as OCG
    from oracle import dirac as OD
    from oracle import lattice as OL
    from oracle import reps as OR
    t_start = time.perf_counter()
    dims, bc, m0 = cfg['dims'], cfg['bc'], cfg['m0']
    UR = OR.represent(U, cfg['rep'])
    psi_o = OL.to_half(psi, dims, 1)
    n, t_hop = 2, 0.0
    for _ in range(n):
        t0 = time.perf_counter()
        OD.D_eo(psi_o, UR, bc, dims)
        t_hop += time.perf_counter() - t0
    Vh = psi_o.shape[0]
    d = UR.shape[-1]
    gbs = hop_bytes_per_site(d, False, 8) * Vh * n / t_hop / 1e9
    cg = {}

    def per_iteration(URx, m, bcx, dd, x):
        t0 = time.perf_counter()
        OD.normal_op(x, URx, m, bcx, dd)
        return time.perf_counter() - t0

    t_it = per_iteration(UR, m0, bc, dims, OL.to_half(psi, dims, 0))
    cg[WORKLOAD] = {'oracle_seconds_per_iteration': round(t_it, 3), 'iters': gpu_c1['iters'],
                    'oracle_seconds_estimate': round(t_it * gpu_c1['iters'], 1),
                    'gpu_seconds': gpu_c1['seconds'],
                    'gpu_speedup': round(t_it * gpu_c1['iters'] / gpu_c1['seconds'], 1),
                    'how': 'one oracle A application x GPU FP64 iterations'}
    for name, (N, rep, dd, bcx, m, Ux, eta) in systems.items():
        URx = OR.represent(Ux, rep)
        b = OL.to_half(eta[0], dd, 0)
        g = gpu_small.get(name)
        if name == 'su2_fund_4x4x4x4':
            t0 = time.perf_counter()
            _, it, res = OCG.cg_eo(b, URx, m, bcx, dd, tol=1e-10, maxit=20000)
            t = time.perf_counter() - t0
            rec = {'oracle_seconds': round(t, 4), 'oracle_iters': it, 'oracle_true_rel_resid': res,
                   'how': 'whole oracle CG'}
            if g:
                rec.update({'gpu_seconds': g['seconds'], 'gpu_iters': g['iters'],
                            'gpu_speedup': round(t / g['seconds'], 2)})
        else:
            t_it = per_iteration(URx, m, bcx, dd, b)
            rec = {'oracle_seconds_per_iteration': round(t_it, 4), 'how': 'one oracle A application x GPU FP64 iterations'}
            if g:
                rec.update({'iters': g['iters'], 'oracle_seconds_estimate': round(t_it * g['iters'], 2),
                            'gpu_seconds': g['seconds'], 'gpu_speedup': round(t_it * g['iters'] / g['seconds'], 1)})
        cg[name] = rec
    total = time.perf_counter() - t_start
    return {'value': round(gbs, 4), 'unit': 'GB/s', 'cores': 1, 'kind': 'oracle',
            'sample': f'{n} oracle D_eo applications on the full {dims} lattice ({t_hop:.1f} s) for the hop rate; '
                      f'CG time-to-1e-10 on {len(cg)} systems (whole CG on 4^4, one A application elsewhere); '
                      f'{total:.1f} s of CPU work in all, NumPy on one thread',
            'host': host_info(), 'cg_time_to_1e-10': cg}


FORM_NAMES = {0: 'site-parallel', 1: 'colour-split', 2: 'colour-split, paired directions',
              3: 'colour-split, compact links', 4: 'colour-split, compact links, paired directions',
              5: 'colour-split, two directions per phase', 6: 'multi-rhs, links staged in LDS per block'}


def tuned_form(best):
    """Readable launch shape from an autotune result."""
    return {'form': FORM_NAMES.get(best['variant'], str(best['variant'])), 'rhs_per_block': best['nr'],
            'xcd_remap': best['xcd_remap'], 't_block': best['tblock']}


def hop_rate(W, torch, lat, UR, prec, nrhs, n=40, seed=5):
    """Mean time of one hop launch in the benchmark pattern (D_eo f0 -> f1,
    D_oe f1 -> f2 alternating; HIP events on the current stream) with the
    shape the context uses for (prec, nrhs), and its compulsory-byte rate."""
    eb = 8 if prec == W.F64 else 4
    g = torch.Generator(device='cuda')
    g.manual_seed(seed)
    f = [lat.new_half(nrhs, prec) for _ in range(3)]
    f[0].view(torch.float64 if prec == W.F64 else torch.float32).normal_(generator=g)

    def launch(k):
        src, dst = (f[0], f[1]) if k % 2 == 0 else (f[1], f[2])
        lat.dslash_eo(dst, src, UR, 0 if k % 2 == 0 else 1, nrhs=nrhs, prec=prec)

    for k in range(4):
        launch(k)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for k in range(n):
        launch(k)
    e1.record(st)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / n * 1e3
    link = lat.d * lat.d * eb * (1 if lat.real else 2)
    by = (8 * link + nrhs * 2 * 4 * lat.d * 2 * eb) * lat.Vh
    return us, by


def dslash_roofline(W, torch, lat, UR, prec, nrhs, tuned, n=40):
    """Hop rate of the tuned shape, against HBM peak.  Bytes are those of the
    form that ran: the compact forms read N^2 instead of d_R^2 complex entries
    per link, and their rate is quoted on their own (smaller) byte count; the
    best stored-link form is then timed as well, in a fresh context of the
    same geometry, for the rate on the stored-link bytes."""
    us, by = hop_rate(W, torch, lat, UR, prec, nrhs, n)
    eb = 8 if prec == W.F64 else 4
    compact = tuned['variant'] in (W.HOP_COMPACT, W.HOP_COMPACT_PAIR)
    if compact:
        by = (8 * lat.N * lat.N * eb * 2 + nrhs * 2 * 4 * lat.d * 2 * eb) * lat.Vh
    gbs = by / (us * 1e-6) / 1e9
    out = {'nrhs': nrhs, 'prec': 'f64' if prec == W.F64 else 'f32', 'form': tuned_form(tuned),
           'us_per_launch': round(us, 2), 'bytes_per_launch': by, 'GBps': round(gbs, 1),
           'frac': round(gbs / HBM_PEAK_GBS, 4)}
    out['tuner_spread'] = round(tuned.get('spread', 0.0), 4)
    out['tuner_runner_up_us'] = round(tuned.get('runner_up_us', 0.0), 2)
    if compact:
        # the best stored-link shape, autotuned in a context whose tuner skips
        # the compact forms
        stored = W.Lattice(lat.N, lat.rep_name, lat.dims, lat.bc)
        stored.set_option(W.OPT_TUNE_COMPACT, 0)
        ts = stored.autotune(UR, prec, nrhs)
        us_s, by_s = hop_rate(W, torch, stored, UR, prec, nrhs, n)
        gs = by_s / (us_s * 1e-6) / 1e9
        out['stored_links'] = {'form': tuned_form(ts), 'us_per_launch': round(us_s, 2), 'bytes_per_launch': by_s,
                               'GBps': round(gs, 1), 'frac': round(gs / HBM_PEAK_GBS, 4),
                               'tuner_spread': round(ts['spread'], 4)}
        del stored
    return out


def traffic_multi(W, torch, synth, name='su3_sym_48x24x24x24', nrhs=12, launches=6):
    """The batched FP64 hop of the 12-source solve (autotuned shape), launched
    `launches` times in the benchmark pattern so that its HBM counters can be
    taken; returns the run description the traffic record is written from."""
    cfg = synth.CONFIGS[name]
    lat = W.Lattice(cfg['N'], cfg['rep'], cfg['dims'], cfg['bc'])
    UR = lat.new_links(W.F64)
    lat.rep_links(UR, torch.from_numpy(synth.links_for(cfg)).cuda(), W.F64)
    best = lat.autotune(UR, W.F64, nrhs)
    f = [lat.new_half(nrhs) for _ in range(3)]
    g = torch.Generator(device='cuda')
    g.manual_seed(7)
    f[0].view(torch.float64).normal_(generator=g)
    for k in range(launches):
        src, dst = (f[0], f[1]) if k % 2 == 0 else (f[1], f[2])
        lat.dslash_eo(dst, src, UR, 0 if k % 2 == 0 else 1, nrhs=nrhs)
    torch.cuda.synchronize()
    link = lat.d * lat.d * 8 * (1 if lat.real else 2)
    spinor = 4 * lat.d * 2 * 8
    return {'workload': f'{name} FP64, {nrhs} right-hand sides in one launch, launches alternating D_eo / D_oe',
            'hop_sources_sha256': hop_sources_sha256(), 'kernel_pattern': 'k_hop', 'launches_per_shape': launches,
            'algorithmic_bytes_per_launch': (8 * link + 2 * nrhs * spinor) * lat.Vh,
            'compulsory_read_bytes': (8 * link + nrhs * spinor) * lat.Vh,
            'shapes': [{k: best[k] for k in ('variant', 'xcd_remap', 'tblock', 'nr')}],
            'tuned_us': best['us']}


def multi_rhs_cg(W, torch, synth, name='su3_sym_48x24x24x24'):
    """Time-to-1e-10 of the even-odd CG for 12 point sources on one gauge
    field: all 12 in one batched solve (every hop streams each link once for
    the 12 sources) against 12 single-source solves, in FP64 and in mixed
    precision.  Run once, after the timed steps."""
    cfg = synth.CONFIGS[name]
    dims, m0, nrhs = cfg['dims'], cfg['m0'], cfg['nrhs']
    log(f'[bench] multi-rhs CG on {name}: generating inputs')
    lat = W.Lattice(cfg['N'], cfg['rep'], dims, cfg['bc'])
    Ug = torch.from_numpy(synth.links_for(cfg)).cuda()
    UR64, UR32 = lat.new_links(W.F64), lat.new_links(W.F32)
    lat.rep_links(UR64, Ug, W.F64)
    lat.rep_links(UR32, Ug, W.F32)
    del Ug
    src = torch.from_numpy(synth.point_sources(dims, lat.d, nrhs)).cuda()
    eta_e, eta_o = lat.pack_half(src, 0, nrhs), lat.pack_half(src, 1, nrhs)
    del src
    bp, b = lat.new_half(nrhs), lat.new_half(nrhs)
    lat.eo_source(bp, eta_e, eta_o, UR64, m0, nrhs)
    lat.apply_dhat(b, bp, UR64, m0, dagger=1, nrhs=nrhs)
    del bp, eta_e, eta_o
    forms, rates = {}, []
    for prec, UR, key in ((W.F64, UR64, 'f64'), (W.F32, UR32, 'f32')):
        for k in (nrhs, 1):
            tuned = lat.autotune(UR, prec, k)
            forms[f'{key}_{k}rhs'] = tuned_form(tuned)
            rates.append(dslash_roofline(W, torch, lat, UR, prec, k, tuned))
            log(f'[bench]   hop {key} {k} rhs: {rates[-1]}')
    ws = lat.new_workspace(W.OP_CG, nrhs, W.CG_MIXED)
    x = lat.new_half(nrhs)
    per = x.numel() // nrhs
    out = {'workload': name, 'sources': f'{nrhs} point sources (spin k%4, colour k//4) at the origin',
           'hop_forms': forms, 'dslash_roofline': rates}
    for mode, key in ((W.CG_F64, 'f64'), (W.CG_MIXED, 'mixed')):
        def batched():
            x.zero_()
            rc, st = lat.cg_eo(x, b, UR64, m0, tol=1e-10, maxit=20000, nrhs=nrhs, mode=mode, UR32=UR32,
                               workspace=ws)
            return st[0]['seconds'], (rc, st)

        batched, (rc, st), batched_runs = median3(batched)
        worst = max(s['true_rel_resid'] for s in st)
        log(f'[bench]   batched {key}: {batched:.3f} s {batched_runs}, iters {[s["iters"] for s in st]}, '
            f'worst residual {worst:.2e}')

        def sequential():
            seq, its, res = 0.0, [], []
            for r in range(nrhs):
                xr, br = x[r * per:(r + 1) * per], b[r * per:(r + 1) * per]
                xr.zero_()
                rc1, st1 = lat.cg_eo(xr, br, UR64, m0, tol=1e-10, maxit=20000, nrhs=1, mode=mode, UR32=UR32,
                                     workspace=ws)
                seq += st1[0]['seconds']
                its.append(st1[0]['iters'])
                res.append(st1[0]['true_rel_resid'])
            return seq, (its, res)

        seq, (its, res), seq_runs = median3(sequential)
        worst = max([worst] + res)
        log(f'[bench]   {nrhs} single solves {key}: {seq:.3f} s {seq_runs}, iters {its}')
        out[key] = {'batched_seconds': round(batched, 4), 'batched_runs': batched_runs,
                    'sequential_seconds': round(seq, 4), 'sequential_runs': seq_runs,
                    'batched_speedup': round(seq / batched, 3), 'max_iters': max(s['iters'] for s in st),
                    'per_rhs_iters': [s['iters'] for s in st], 'reliable_updates': [s['reliable_updates'] for s in st],
                    'worst_true_rel_resid': worst, 'status': W.STATUS_NAMES.get(rc)}
    out['mixed_batched_vs_f64_sequential'] = round(out['f64']['sequential_seconds'] / out['mixed']['batched_seconds'],
                                                   3)
    return out


def mixed_cg_large(W, torch, synth, name='su4_2as_96x48x48x48'):
    """Time-to-1e-10 of FP64 CG and mixed-precision CG (FP32 hops, FP64
    reliable updates) on SU(4) 2AS 96x48^3, right-hand side D-hat^+ eta with
    Gaussian eta.  Run once, after the timed steps."""
    cfg = synth.CONFIGS[name]
    dims, m0 = cfg['dims'], cfg['m0']
    log(f'[bench] mixed vs FP64 CG on {name}: generating inputs')
    lat = W.Lattice(cfg['N'], cfg['rep'], dims, cfg['bc'])
    U = synth.expH_links_torch(dims, cfg['N'], cfg['eps'], cfg['seed'])
    UR64, UR32 = lat.new_links(W.F64), lat.new_links(W.F32)
    lat.rep_links(UR64, U, W.F64)
    lat.rep_links(UR32, U, W.F32)
    del U
    g = torch.Generator(device='cuda')
    g.manual_seed(cfg['seed'] + 11)
    eta = torch.randn((1,) + tuple(dims) + (4, lat.d), dtype=torch.complex128, device='cuda', generator=g)
    eta_e = lat.pack_half(eta, 0)
    del eta
    b = lat.new_half()
    lat.apply_dhat(b, eta_e, UR64, m0, dagger=1)
    del eta_e
    forms, rates = {}, []
    for prec, UR, key in ((W.F64, UR64, 'f64'), (W.F32, UR32, 'f32')):
        tuned = lat.autotune(UR, prec, 1)
        forms[key] = tuned_form(tuned)
        rates.append(dslash_roofline(W, torch, lat, UR, prec, 1, tuned, n=20))
        log(f'[bench]   hop {key}: {rates[-1]}')
    ws = lat.new_workspace(W.OP_CG, 1, W.CG_MIXED)
    x = lat.new_half()
    out = {'workload': name, 'source': 'D-hat^+ eta, eta Gaussian', 'hop_forms': forms, 'dslash_roofline': rates}
    for mode, key in ((W.CG_F64, 'f64'), (W.CG_MIXED, 'mixed')):
        def solve():
            x.zero_()
            rc, st = lat.cg_eo(x, b, UR64, m0, tol=1e-10, maxit=20000, mode=mode, UR32=UR32, workspace=ws)
            return st[0]['seconds'], (rc, st[0])

        secs, (rc, st), runs = median3(solve)
        log(f'[bench]   {key}: {secs:.3f} s {runs}, {st["iters"]} iterations, residual {st["true_rel_resid"]:.2e}')
        out[key] = {'seconds': round(secs, 4), 'runs': runs, 'iters': st['iters'], 'hops': st['hops'],
                    'reliable_updates': st['reliable_updates'], 'true_rel_resid': st['true_rel_resid'],
                    'status': W.STATUS_NAMES.get(rc)}
    out['mixed_speedup'] = round(out['f64']['seconds'] / out['mixed']['seconds'], 3)
    return out


def median3(run):
    """Median over three calls of run() -> (seconds, payload); returns
    (median seconds, payload of the last call, all three times)."""
    ts, last = [], None
    for _ in range(3):
        t, last = run()
        ts.append(t)
    return float(sorted(ts)[1]), last, [round(t, 4) for t in ts]


def lattice_batch_cg(W, torch, synth):
    """SU(3) SYM on 8^4, 12^4 and 16^3x32 (m0 = -0.4, Gaussian sources on the
    even sites): one batched CG call over the three lattices against three
    separate single-lattice calls, FP64 and mixed; medians of three solves
    after one warm-up."""
    log('[bench] batch of three lattices: generating inputs')
    Us, etas = batch_inputs(synth)
    Ug = [torch.from_numpy(u).cuda() for u in Us]
    eg = [torch.from_numpy(e).cuda() for e in etas]
    lat = W.Lattice(3, 'SYM', BATCH_SHAPES, (-1, 1, 1, 1))
    UR64, UR32 = lat.new_links(W.F64), lat.new_links(W.F32)
    Ucat = torch.cat([u.reshape(-1, 4, 3, 3) for u in Ug])
    lat.rep_links(UR64, Ucat, W.F64)
    lat.rep_links(UR32, Ucat, W.F32)
    b = lat.pack_half(torch.cat([e.reshape(-1, 4, 6) for e in eg]), 0)
    lat.autotune(UR64, W.F64, 1)
    lat.autotune(UR32, W.F32, 1)
    singles = []
    for k, dd in enumerate(BATCH_SHAPES):
        l1 = W.Lattice(3, 'SYM', dd, (-1, 1, 1, 1))
        u64, u32 = l1.new_links(W.F64), l1.new_links(W.F32)
        l1.rep_links(u64, Ug[k], W.F64)
        l1.rep_links(u32, Ug[k], W.F32)
        l1.autotune(u64, W.F64, 1)
        l1.autotune(u32, W.F32, 1)
        singles.append((l1, u64, u32, l1.pack_half(eg[k], 0)))
    out = {'lattices': ['x'.join(map(str, dd)) for dd in BATCH_SHAPES], 'repeats': 'median of 3 after a warm-up'}
    for mode, key in ((W.CG_F64, 'f64'), (W.CG_MIXED, 'mixed')):
        x = lat.new_half()

        def batched():
            x.zero_()
            rc, st = lat.cg_eo(x, b, UR64, BATCH_M0, tol=1e-10, maxit=20000, mode=mode, UR32=UR32)
            return st[0]['seconds'], (rc, st)

        batched()   # warm-up
        tb, (rc, st), tbs = median3(batched)

        def separate():
            tot, its, res = 0.0, [], []
            for l1, u64, u32, b1 in singles:
                x1 = l1.new_half()
                rc1, st1 = l1.cg_eo(x1, b1, u64, BATCH_M0, tol=1e-10, maxit=20000, mode=mode, UR32=u32)
                tot += st1[0]['seconds']
                its.append(st1[0]['iters'])
                res.append(st1[0]['true_rel_resid'])
            return tot, (its, res)

        separate()  # warm-up
        ts, (its, res), tss = median3(separate)
        out[key] = {'batched_seconds': round(tb, 4), 'batched_runs': tbs, 'batched_iters': [s_['iters'] for s_ in st],
                    'batched_worst_true_rel_resid': max(s_['true_rel_resid'] for s_ in st),
                    'status': W.STATUS_NAMES.get(rc), 'separate_seconds': round(ts, 4), 'separate_runs': tss,
                    'separate_iters': its, 'batched_speedup': round(ts / tb, 3)}
        log(f'[bench]   batch {key}: batched {tb:.4f} s vs separate {ts:.4f} s')
    out['mixed_batched_vs_f64_separate'] = round(out['f64']['separate_seconds'] / out['mixed']['batched_seconds'], 3)
    return out


def force_timing(W, torch, synth, name='su2_adj_32x16x16x16', reps=10):
    """The fermion force (three hops and the per-link kernel) and one
    autograd forward + backward of the pseudofermion action on SU(2) ADJ
    32x16^3, phi = D-hat^+ eta."""
    from paper_2503_06721_amd.autograd import fermion_action
    cfg = synth.CONFIGS[name]
    dims, m0 = cfg['dims'], cfg['m0']
    lat = W.Lattice(cfg['N'], cfg['rep'], dims, cfg['bc'])
    U = torch.from_numpy(synth.links_for(cfg)).cuda()
    UR = lat.new_links(W.F64)
    lat.rep_links(UR, U)
    lat.autotune(UR, W.F64, 1)
    eta = torch.from_numpy(synth.gaussian_spinor((1,) + dims + (4, lat.d), cfg['seed'] + 2)).cuda()
    phi = lat.new_half()
    lat.apply_dhat(phi, lat.pack_half(eta, 0), UR, m0, dagger=1)
    x = lat.new_half()
    lat.cg_eo(x, phi, UR, m0, tol=1e-10)
    G = torch.empty_like(U)
    ws = lat.new_workspace(W.OP_FORCE)
    lat.force_eo(G, x, UR, m0, U=U, workspace=ws)
    t0 = time.perf_counter()
    for _ in range(reps):
        lat.force_eo(G, x, UR, m0, U=U, workspace=ws)
    t_force = (time.perf_counter() - t0) / reps
    Uv = U.clone().requires_grad_(True)
    fermion_action(Uv, phi, lat, m0, tol=1e-10).backward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Uv.grad = None
    S = fermion_action(Uv, phi, lat, m0, tol=1e-10)
    S.backward()
    torch.cuda.synchronize()
    t_ag = time.perf_counter() - t0
    return {'workload': name, 'force_eo_ms': round(t_force * 1e3, 3),
            'autograd_action_and_gradient_ms': round(t_ag * 1e3, 3)}


def rhmc_and_clover(W, torch, synth, name='su3_fund_32x32x32x32'):
    """On the benchmark lattice: 12 shifts (a zero shift and 11 from 1e-4 to
    5.9) in one multi-shift call against 12 one-shift calls; and the
    clover-improved operator (c_sw = 1) -- clover field construction, FP64 and
    mixed CG to 1e-10 on D-hat^+ D-hat with the clover D-hat, and the clover
    force (pseudofermion and determinant terms, regular and exponential)."""
    cfg = synth.CONFIGS[name]
    dims, m0 = cfg['dims'], cfg['m0']
    lat = W.Lattice(cfg['N'], cfg['rep'], dims, cfg['bc'])
    U = torch.from_numpy(synth.links_for(cfg)).cuda()
    UR64, UR32 = lat.new_links(W.F64), lat.new_links(W.F32)
    lat.rep_links(UR64, U, W.F64)
    lat.rep_links(UR32, U, W.F32)
    lat.autotune(UR64, W.F64, 1)
    lat.autotune(UR32, W.F32, 1)
    g = torch.Generator(device='cuda')
    g.manual_seed(cfg['seed'] + 21)
    eta = torch.randn((1,) + tuple(dims) + (4, lat.d), dtype=torch.complex128, device='cuda', generator=g)
    b = lat.pack_half(eta, 0)
    del eta
    shifts = [0.0] + [1e-4 * 3.0 ** k for k in range(11)]
    x = lat.new_shift_fields(len(shifts))
    ws = lat.new_workspace(W.OP_MSHIFT, len(shifts), W.F64)
    lat.cg_mshift_eo(x, b, UR64, m0, shifts, tol=1e-10, maxit=20000, workspace=ws)    # warm-up
    rc, st = lat.cg_mshift_eo(x, b, UR64, m0, shifts, tol=1e-10, maxit=20000, workspace=ws)
    one, its = 0.0, []
    for k, sh in enumerate(shifts):
        rc1, st1 = lat.cg_mshift_eo(lat.shift_field(x, k), b, UR64, m0, [sh], tol=1e-10, maxit=20000, workspace=ws)
        one += st1[0]['seconds']
        its.append(st1[0]['iters'])
    log(f'[bench] multi-shift: {st[0]["seconds"]:.3f} s for 12 shifts, 12 single shifts {one:.3f} s')
    ms = {'shifts': len(shifts), 'seconds': round(st[0]['seconds'], 4), 'iters': [s['iters'] for s in st],
          'worst_true_rel_resid': max(s['true_rel_resid'] for s in st), 'status': W.STATUS_NAMES.get(rc),
          'single_shift_calls_seconds': round(one, 4), 'single_shift_iters': its,
          'speedup': round(one / st[0]['seconds'], 3)}
    del x, ws
    csw = 1.0
    c64, c32 = lat.new_clover(W.F64), lat.new_clover(W.F32)
    cws = lat.new_workspace(W.OP_CLOVER, 1, W.F64)
    lat.clover_field(c64, U, m0, csw, 0, W.F64, workspace=cws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.clover_field(c64, U, m0, csw, 0, W.F64, workspace=cws)
    torch.cuda.synchronize()
    t_field = time.perf_counter() - t0
    lat.clover_field(c32, U, m0, csw, 0, W.F32, workspace=cws)
    del cws
    cg_ws = lat.new_workspace(W.OP_CG, 1, W.CG_MIXED)
    xc = lat.new_half()
    cl = {'csw': csw, 'clover_field_ms': round(t_field * 1e3, 3)}
    for mode, key in ((W.CG_F64, 'f64'), (W.CG_MIXED, 'mixed')):
        xc.zero_()
        rc, stc = lat.cg_eo_clover(xc, b, UR64, c64, tol=1e-10, maxit=20000, mode=mode, UR32=UR32, clov32=c32,
                                   workspace=cg_ws)
        cl[key] = {'seconds': round(stc[0]['seconds'], 4), 'iters': stc[0]['iters'],
                   'true_rel_resid': stc[0]['true_rel_resid'], 'status': W.STATUS_NAMES.get(rc)}
    cl['mixed_speedup'] = round(cl['f64']['seconds'] / cl['mixed']['seconds'], 3)
    log(f'[bench] clover CG: {cl}')
    del cg_ws, c32

    def timed_ms(fn):
        fn()   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return round((time.perf_counter() - t0) * 1e3, 3)

    # clover force at the CG solution: pseudofermion force (3 hops, 3 clover
    # applications, hopping links, clover insertion, leaves, gather), the
    # odd-block determinant force and its action; regular then exponential
    N = cfg['N']
    P = torch.zeros(tuple(dims) + (4, N, N), dtype=torch.complex128, device='cuda')
    fws = lat.new_workspace(W.OP_CLOVER_FORCE, 1, W.F64)
    cws = lat.new_workspace(W.OP_CLOVER, 1, W.F64)
    forces = {}
    for expo, key in ((0, 'regular'), (1, 'exponential')):
        lat.clover_field(c64, U, m0, csw, expo, W.F64, workspace=cws)
        forces[key] = {
            'pseudofermion_force_ms': timed_ms(lambda: lat.force_eo_clover(P, xc, UR64, U, c64, m0, csw, expo,
                                                                           workspace=fws)),
            'logdet_force_ms': timed_ms(lambda: lat.force_clover_logdet(P, U, c64, m0, csw, expo, accumulate=1,
                                                                        workspace=fws)),
            'logdet_ms': timed_ms(lambda: lat.clover_logdet(c64, workspace=fws))}
    cl['force'] = forces
    log(f'[bench] clover force: {forces}')
    return {'workload': name, 'multi_shift_time_to_1e-10': ms, 'clover_cg_time_to_1e-10': cl}


def hmc_trajectory(W, torch, synth, name='su2_adj_32x16x16x16', n_therm=40, n_meas=4):
    """HMC on SU(2) ADJ 32x16^3 (second-order Omelyan, tau = 0.5 in 5
    steps, Wilson plaquette beta = 2.2 plus the two-flavour adjoint
    pseudofermion): n_therm thermalisation trajectories from the synthetic
    start (each accepted, fresh momenta and pseudofermions every time; the
    same tau in 10 steps, so that the integration stays stable while the
    smooth start heats up), then n_meas timed HMC updates with the Metropolis
    test: seconds per trajectory, CG iterations, dH and acceptance."""
    import numpy as np
    from paper_2503_06721_amd.hmc import HMC
    cfg = synth.CONFIGS[name]
    dims, m0, N = cfg['dims'], cfg['m0'], cfg['N']
    lat = W.Lattice(N, cfg['rep'], dims, cfg['bc'])
    U = torch.from_numpy(synth.links_for(cfg)).cuda()
    hmc = HMC(lat, 2.2, m0, tol=1e-10)
    lat.rep_links(hmc.UR, U)
    lat.autotune(hmc.UR, W.F64, 1)
    g = torch.Generator(device='cuda')
    g.manual_seed(cfg['seed'] + 31)
    eps, nsteps = 0.1, 5
    dH_therm = []
    t0 = time.perf_counter()
    for _ in range(n_therm):
        w = torch.randn(tuple(dims) + (4, N * N - 1), dtype=torch.float64, device='cuda', generator=g)
        re = torch.randn((1,) + tuple(dims) + (4, lat.d), dtype=torch.float64, device='cuda', generator=g)
        im = torch.randn((1,) + tuple(dims) + (4, lat.d), dtype=torch.float64, device='cuda', generator=g)
        pi, phi = hmc.refresh(U, w, lat.pack_half(torch.complex(re, im) * (0.5 ** 0.5), 0))
        H0, H1 = hmc.trajectory(U, pi, phi, eps / 2, 2 * nsteps, 'omelyan2')
        dH_therm.append(H1 - H0)
    torch.cuda.synchronize()
    t_therm = time.perf_counter() - t0
    it0 = hmc.cg_iters
    dH, acc, secs = [], [], []
    for _ in range(n_meas):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d, a = hmc.update(U, eps, nsteps, g, 'omelyan2')
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t0)
        dH.append(d)
        acc.append(bool(a))
    log(f'[bench] HMC: thermalisation dH {[round(v, 3) for v in dH_therm]}; measured dH {dH}, '
        f'{np.median(secs):.3f} s per trajectory')
    return {'workload': name, 'integrator': 'omelyan2', 'tau': eps * nsteps, 'steps': nsteps, 'beta': 2.2,
            'thermalisation': {'trajectories': n_therm, 'seconds': round(t_therm, 3),
                               'first_dH': dH_therm[0], 'last_dH': dH_therm[-1]},
            'seconds_per_trajectory': round(float(np.median(secs)), 4), 'dH': dH, 'accepted': acc,
            'cg_iterations_per_trajectory': (hmc.cg_iters - it0) / n_meas,
            'start': f'{n_therm} always-accepted trajectories ({2 * nsteps} steps) from the synthetic '
                     f'exp(i 0.3 H) links'}


SECTIONS = {'multi_rhs': multi_rhs_cg, 'mixed_large': mixed_cg_large, 'lattice_batch': lattice_batch_cg,
            'force': force_timing, 'rhmc_clover': rhmc_and_clover, 'hmc': hmc_trajectory}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=3)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--hops', type=int, default=200, help='dslash_eo launches timed per step')
    ap.add_argument('--no-cpu', action='store_true', help='skip the CPU-oracle baseline')
    ap.add_argument('--no-cg', action='store_true', help='profiling aid: hops and links only')
    ap.add_argument('--no-multi', action='store_true',
                    help='skip the one-off solver comparisons (12 sources batched vs single, SU(4) 2AS mixed vs '
                         'FP64, three-lattice batch) and the force timing')
    ap.add_argument('--only', choices=sorted(SECTIONS),
                    help='profiling aid: run one of the one-off sections alone and print its JSON')
    ap.add_argument('--traffic-shapes', action='store_true',
                    help='profiling aid: 6 hop launches (the benchmark pattern) for every FP64 launch shape the '
                         'autotuner may pick, in the order printed, to take HBM counters per shape')
    ap.add_argument('--traffic-multi', action='store_true',
                    help='profiling aid: 6 launches of the 12-source FP64 hop on SU(3) SYM 48x24^3 with the '
                         'autotuned shape, to take HBM counters on the batched hop')
    ap.add_argument('--copy-calibration', action='store_true',
                    help='run only the kernels of known traffic that calibrate the FETCH_SIZE / WRITE_SIZE '
                         'counters (a 2 GiB device copy x4, the 7-read/1-write streaming probe x4) and print '
                         'their byte counts')
    ap.add_argument('--traffic-record', nargs=7,
                    metavar=('OUT', 'RUN_JSON', 'FETCH_CSV', 'WRITE_CSV', 'CAL_JSON', 'CAL_FETCH_CSV',
                             'CAL_WRITE_CSV'),
                    help='no GPU: write the per-launch traffic record OUT from the JSON line of a '
                         '--traffic-shapes or --traffic-multi run, its rocprofv3 FETCH_SIZE and WRITE_SIZE '
                         'counter_collection.csv files, and the same three of a --copy-calibration run')
    ap.add_argument('--kernel-durations', nargs=3, metavar=('TRACE_CSV', 'PATTERN', 'LAST'),
                    help='no GPU: mean duration of one kernel in a rocprofv3 kernel_trace.csv, over all its '
                         'dispatches and over the last LAST (the timed launches)')
    args = ap.parse_args()
    if args.kernel_durations:
        print(kernel_durations(args.kernel_durations[0], args.kernel_durations[1], int(args.kernel_durations[2])))
        return
    if args.traffic_record:
        write_traffic_record(*args.traffic_record)
        return
    if args.gpus != 1:
        print(f'bench.py measures one GPU only; --gpus {args.gpus} is not supported '
              f'(how the path would shard over several GPUs is described in the design notes, not implemented)', file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = 1 << 28
        ms, g = device_copy_gbps(torch, n)
        from paper_2503_06721_amd import wdirac as W
        elems = 1 << 24
        sg = W.stream_probe(elems, 7, 3)
        print(json.dumps({'kernels': [
            {'name': 'device_copy', 'pattern': 'copyBuffer', 'bytes_read': n * 8, 'bytes_written': n * 8,
             'dispatches': 4, 'ms_per_copy': round(ms, 4), 'GBps_read_plus_write': round(g, 1)},
            {'name': 'stream_probe', 'pattern': 'k_stream<7>', 'bytes_read': 7 * elems * 16,
             'bytes_written': elems * 16, 'dispatches': 4, 'GBps_read_plus_write': round(sg, 1)}]}))
        return

    from paper_2503_06721_amd import synth
    from paper_2503_06721_amd import wdirac as W

    if args.traffic_multi:
        print(json.dumps(traffic_multi(W, torch, synth)), flush=True)
        return
    if args.only:
        print(json.dumps(SECTIONS[args.only](W, torch, synth)), flush=True)
        return

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
    if args.traffic_shapes:
        shapes = []
        for variant in (W.HOP_SITE, W.HOP_COLOUR, W.HOP_COLOUR_PAIR, W.HOP_COLOUR_QUAD):
            for remap in (0, 1):
                for tb in (0, 2, 4, 8):
                    lat.set_option(W.OPT_HOP_VARIANT_F64, variant)
                    lat.set_option(W.OPT_XCD_REMAP, remap)
                    lat.set_option(W.OPT_TILE_TBLOCK, tb)
                    lat.set_option(W.OPT_HOP_NR_F64, 1)
                    for k in range(6):
                        src, dst = (halves[0], halves[1]) if k % 2 == 0 else (halves[1], halves[2])
                        lat.dslash_eo(dst, src, UR64, 0 if k % 2 == 0 else 1)
                    shapes.append({'variant': variant, 'xcd_remap': remap, 'tblock': tb, 'nr': 1})
        torch.cuda.synchronize()
        print(json.dumps({'workload': f'{WORKLOAD} FP64, one right-hand side, launches alternating D_eo / D_oe '
                                      'as in the benchmark',
                          'hop_sources_sha256': hop_sources_sha256(), 'kernel_pattern': 'k_hop',
                          'launches_per_shape': 6, 'algorithmic_bytes_per_launch': bytes_per_launch,
                          'compulsory_read_bytes': bytes_per_launch - 4 * d * 2 * 8 * lat.Vh,
                          'shapes': shapes}))
        return
    # the library's autotuner picks the hop launch shape for both precisions
    tuned = {'f64': lat.autotune(UR64, W.F64, 1), 'f32': lat.autotune(UR32, W.F32, 1)}
    log(f'[bench] autotuned hop shapes: {tuned}')
    variant_name = {W.HOP_SITE: 'k_hop_sp (lane per site)', W.HOP_COLOUR: 'k_hop_cs (colour-split)',
                    W.HOP_COLOUR_PAIR: 'k_hop_cs (colour-split, paired directions)',
                    W.HOP_COLOUR_QUAD: 'k_hop_cs (colour-split, two directions per phase)',
                    W.HOP_MULTI: 'k_hop_mr (links staged per block)'}

    def step(record):
        lat.rep_links(UR64, Ug, W.F64)
        lat.rep_links(UR32, Ug, W.F32)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k in range(args.hops):
            # alternate D_eo (h0 -> h1) and D_oe (h1 -> h2): every other launch reads the output just written
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
    hop_ms_median = float(np.median([r['hop_ms'] for r in recs]))
    copy_gbs = round(device_copy_gbps(torch)[1], 1)
    # the library's streaming probe with the hop's read:write mix (7:1), its
    # streams 256 MiB + 4 KiB apart (offsets that are a multiple of 16 KiB
    # put the streams on the same HBM channel pattern and cost ~5%)
    stream_gbs = round(W.stream_probe((1 << 24) + 256, 7, 20), 1)
    gbs = bytes_per_launch / (hop_ms * 1e-3) / 1e9
    traffic = measured_traffic(bytes_per_launch, tuned['f64'])
    out = {
        'metric': 'Dslash GB/s & % HBM roofline; CG time-to-1e-10 (FP64 vs mixed/multi-RHS)',
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
                     'traffic_unit': 'HBM bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1, factors '
                                     'calibrated on the non-temporal streaming probe and a 2 GiB copy)',
                     'traffic_GBps': None if traffic is None else round(traffic / (hop_ms * 1e-3) / 1e9, 2),
                     'effective_GBps': round(effective_bytes_per_site(d, lat.real, 8) * lat.Vh / (hop_ms * 1e-3)
                                             / 1e9, 2),
                     'device_copy_GBps': copy_gbs,
                     'kernel': variant_name[tuned['f64']['variant']] + f' d=3 complex FP64, '
                               f'xcd_remap={tuned["f64"]["xcd_remap"]}, t-block={tuned["f64"]["tblock"]}',
                     'bytes_per_launch': bytes_per_launch, 'us_per_launch': round(hop_ms * 1e3, 3),
                     'us_per_launch_median_of_steps': round(hop_ms_median * 1e3, 3),
                     'frac_of_device_copy': round(gbs / copy_gbs, 4),
                     'stream_7r1w_GBps': stream_gbs,
                     'frac_of_stream_7r1w': round(gbs / stream_gbs, 4),
                     'tuner_spread': round(tuned['f64']['spread'], 4),
                     'tuner_runner_up_us': round(tuned['f64']['runner_up_us'], 2)},
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
    if not args.no_cg and not args.no_multi:
        del halves, x64, xmix, ws_cg, b, UR32
        torch.cuda.empty_cache()
        out['cg_multi_rhs_time_to_1e-10'] = multi_rhs_cg(W, torch, synth)
        torch.cuda.empty_cache()
        out['cg_mixed_vs_f64_time_to_1e-10'] = mixed_cg_large(W, torch, synth)
        torch.cuda.empty_cache()
        out['cg_lattice_batch_time_to_1e-10'] = lattice_batch_cg(W, torch, synth)
        out['force'] = force_timing(W, torch, synth)
        torch.cuda.empty_cache()
        out['rhmc_and_clover'] = rhmc_and_clover(W, torch, synth)
        torch.cuda.empty_cache()
        out['hmc_trajectory'] = hmc_trajectory(W, torch, synth)
    if not args.no_cpu:
        log('[bench] small CG systems on the GPU, then the CPU oracle on a bounded sample')
        systems = small_systems(synth)
        gpu_small = gpu_small_solves(W, torch, systems)
        gpu_c1 = out.get('cg_time_to_1e-10', {}).get('f64') or {'seconds': float('nan'), 'iters': 0}
        out['cpu_baseline'] = cpu_baseline(cfg, U, psi[0], gpu_c1, systems, gpu_small)
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()
