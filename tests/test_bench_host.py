"""Host logic of bench.py that needs no GPU: the compulsory-byte counts of the
hop, the traffic record written from rocprofv3 counter files, and kernel
durations read from a rocprofv3 kernel trace."""
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

HDR = ['Correlation_Id', 'Dispatch_Id', 'Agent_Id', 'Queue_Id', 'Process_Id', 'Thread_Id', 'Grid_Size',
       'Kernel_Id', 'Kernel_Name', 'Workgroup_Size', 'LDS_Block_Size', 'Scratch_Size', 'VGPR_Count',
       'Accum_VGPR_Count', 'SGPR_Count', 'Counter_Name', 'Counter_Value', 'Start_Timestamp', 'End_Timestamp']


def write_counters(path, counter, rows):
    """rows: (dispatch id, kernel name, value); a dispatch may appear twice
    (per-dimension rows), which the reader must sum."""
    with open(path, 'w', newline='') as f:
        w = csv.writer(f)
        w.writerow(HDR)
        for k, name, v in rows:
            r = dict.fromkeys(HDR, 0)
            r.update(Dispatch_Id=k, Kernel_Name=name, Counter_Name=counter, Counter_Value=v)
            w.writerow([r[h] for h in HDR])


def test_compulsory_bytes():
    # SU(3) FUND FP64: 8 links of 9 complex doubles, input and output spinor of 12
    assert bench.hop_bytes_per_site(3, False, 8) == 8 * 144 + 2 * 192
    assert bench.effective_bytes_per_site(3, False, 8) == 8 * 144 + 9 * 192
    # real representation: links of d^2 reals
    assert bench.hop_bytes_per_site(3, True, 8) == 8 * 72 + 2 * 192


def test_traffic_record(tmp_path):
    """Calibration factors from kernels of known bytes; per-shape means over
    the last launches of the hop, split per shape in order."""
    kib = 1024.0
    cal = {'kernels': [
        {'name': 'device_copy', 'pattern': 'copyBuffer', 'bytes_read': 4096 * 1024, 'bytes_written': 4096 * 1024},
        {'name': 'stream_probe', 'pattern': 'k_stream<7>', 'bytes_read': 7 * 1024 * 1024,
         'bytes_written': 1024 * 1024}]}
    (tmp_path / 'cal.json').write_text(json.dumps(cal))
    # FETCH_SIZE counts half the bytes read, WRITE_SIZE all bytes written
    write_counters(tmp_path / 'cf.csv', 'FETCH_SIZE', [(1, '__amd_rocclr_copyBuffer', 2048.0),
                                                       (2, 'void wd::k_stream<7>(...)', 3584.0)])
    write_counters(tmp_path / 'cw.csv', 'WRITE_SIZE', [(1, '__amd_rocclr_copyBuffer', 4096.0),
                                                       (2, 'void wd::k_stream<7>(...)', 1024.0)])
    run = {'workload': 'w', 'hop_sources_sha256': 'abc', 'kernel_pattern': 'k_hop', 'launches_per_shape': 2,
           'algorithmic_bytes_per_launch': 1000 * 1024, 'compulsory_read_bytes': 800 * 1024,
           'shapes': [{'variant': 1}, {'variant': 2}]}
    (tmp_path / 'run.json').write_text(json.dumps(run))
    # one hop dispatch before the measured ones (not counted), a foreign
    # kernel in between, and one dispatch split over two rows
    fetch = [(1, 'wd::k_hop_cs<A>', 9999.0), (2, 'wd::k_hop_cs<A>', 400.0), (3, 'other', 5.0),
             (4, 'wd::k_hop_cs<A>', 500.0), (5, 'wd::k_hop_sp<B>', 300.0), (5, 'wd::k_hop_sp<B>', 300.0),
             (6, 'wd::k_hop_sp<B>', 800.0)]
    write_counters(tmp_path / 'f.csv', 'FETCH_SIZE', fetch)
    write_counters(tmp_path / 'w.csv', 'WRITE_SIZE', [(1, 'wd::k_hop_cs<A>', 1.0), (2, 'wd::k_hop_cs<A>', 100.0),
                                                      (4, 'wd::k_hop_cs<A>', 100.0), (5, 'wd::k_hop_sp<B>', 200.0),
                                                      (6, 'wd::k_hop_sp<B>', 200.0)])
    out = tmp_path / 'rec.json'
    bench.write_traffic_record(str(out), str(tmp_path / 'run.json'), str(tmp_path / 'f.csv'),
                               str(tmp_path / 'w.csv'), str(tmp_path / 'cal.json'), str(tmp_path / 'cf.csv'),
                               str(tmp_path / 'cw.csv'))
    rec = json.loads(out.read_text())
    assert rec['calibration']['device_copy']['fetch_factor'] == 2.0
    assert rec['calibration']['stream_probe']['fetch_factor'] == 2.0
    assert rec['calibration']['stream_probe']['write_factor'] == 1.0
    assert rec['hop_sources_sha256'] == 'abc'
    a, b = rec['per_launch_shape']
    assert a['launch_shape'] == {'variant': 1} and b['launch_shape'] == {'variant': 2}
    assert a['fetch_size_kib_per_launch'] == 450.0 and a['write_size_kib_per_launch'] == 100.0
    assert a['hbm_bytes_per_launch'] == round((450.0 * 2 + 100.0) * kib)
    assert a['traffic_over_algorithmic'] == 1.0
    assert b['fetch_size_kib_per_launch'] == 700.0 and 'k_hop_sp' in b['kernel']
    assert b['reads_over_compulsory_reads'] == round(700.0 * 2 / 800, 4)


def test_kernel_durations(tmp_path):
    """Mean over all dispatches of the kernel and over the last ones, in
    dispatch order, other kernels ignored."""
    p = tmp_path / 'trace.csv'
    with open(p, 'w', newline='') as f:
        w = csv.writer(f)
        w.writerow(['Dispatch_Id', 'Kernel_Name', 'Start_Timestamp', 'End_Timestamp'])
        w.writerow([3, 'k_hop_cs<A>', 100, 400])     # 300
        w.writerow([1, 'k_hop_cs<A>', 0, 100])       # 100
        w.writerow([2, 'other', 0, 5000])
        w.writerow([4, 'k_hop_cs<A>', 500, 1000])    # 500
    out = bench.kernel_durations(str(p), 'k_hop_cs<A>', 2)
    assert 'dispatches: 3, mean over all: 300 ns' in out
    assert 'last 2 dispatches: mean 400 ns, median 400 ns, min 300 ns, max 500 ns' in out
