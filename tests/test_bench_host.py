"""Host logic of bench.py's profile summaries (no GPU): counter calibration
against the streaming probes and the traffic it records, on a synthetic run
directory laid out as the rocprofv3 commands of bench.PROFILE_COMMANDS write it."""

import csv
import json
import os

import bench

STEP = "void dvbm::k_collide_advect_sweep<2, dvbm::{}, 0, 0, 1>(float const*, float*, dvbm::KParams, int, int)"
PROBE = "void dvbm::k_stream<HIP_vector_type<unsigned int, 4u>, false>(void const*, void*, long, int)"
ADJ = ("void dvbm::k_adjoint_relax<2, dvbm::StoreF64, 1, double>(double const*)",
       "void dvbm::k_adjoint_flux<2, dvbm::StoreF64, 0, 0, double>(double const*)",
       "void dvbm::k_collide_advect_lds<2, dvbm::StoreF64, 0, 0, 1>(double const*)")
STORES = {"f32_dev": "StoreF32Dev", "f64": "StoreF64", "bf16_dev": "StoreBF16"}
VALU = ("SQ_INSTS_VALU", "SQ_WAVES", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
        "SQ_ACTIVE_INST_VALU", "GRBM_GUI_ACTIVE")


def _trace(path, launches):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z", "Start_Timestamp", "End_Timestamp"])
        t = 0
        for name, grid, ns in launches:
            w.writerow([name, grid, 1, 1, t, t + ns])
            t += ns + 10


def _pmc(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        for name, grid, counter, value in rows:
            w.writerow([name, grid, counter, value])


def _run_dir(tmp):
    n = 64
    line = {"value": 4096.0, "ms_per_step": 0.001, "config": {"nx": n, "ny": n, "split": 2, "storage": "f32_dev"},
            "roofline": {"kernel": "k_collide_advect_sweep", "bytes_per_update": 400, "achieved": 1638.4}}
    with open(os.path.join(tmp, "prof_trace.json"), "w") as fh:
        fh.write("[bench] a progress line\n" + json.dumps(line) + "\n")
    _trace(os.path.join(tmp, "prof_trace", "trace_kernel_trace.csv"),
           [(STEP.format(s), 1000, 1000) for s in STORES.values() for _ in range(3)]
           + [(STEP.format("StoreF32Dev"), 200, 50)])  # a smaller grid of the same instance: not the workload's
    for st, store in STORES.items():
        # probes: 4 GiB read (FETCH reads half of it) and 4 GiB written; the step kernel 1000 / 1600 KiB
        probe_fetch = [(PROBE, 262144, "FETCH_SIZE", 2097152.0)] * 3
        probe_write = [(PROBE, 262144, "WRITE_SIZE", 4194304.0)] * 3
        _pmc(os.path.join(tmp, f"prof_fetch_{st}", "pmc_counter_collection.csv"),
             probe_fetch + [(STEP.format(store), 1000, "FETCH_SIZE", 1000.0)] * 5)
        _pmc(os.path.join(tmp, f"prof_write_{st}", "pmc_counter_collection.csv"),
             probe_write + [(STEP.format(store), 1000, "WRITE_SIZE", 1600.0)] * 5)
        _pmc(os.path.join(tmp, f"prof_valu_{st}", "pmc_counter_collection.csv"),
             [(STEP.format(store), 1000, c, v) for c, v in zip(VALU, (2.4e6, 100, 1e4, 5e3, 5e3, 1.2e6, 8e4))])
        _pmc(os.path.join(tmp, f"prof_stall_{st}", "pmc_counter_collection.csv"),
             [(STEP.format(store), 1000, c, v) for c, v in zip(bench.STALL_COUNTERS.split(),
                                                               (4e5, 2e5, 1e6, 5e5, 900.0, 100.0))])
    for g in bench.ADJ_GRIDS:
        _trace(os.path.join(tmp, f"prof_adj{g}_trace", "trace_kernel_trace.csv"), [(k, 256, 500) for k in ADJ])
        _pmc(os.path.join(tmp, f"prof_adj{g}_fetch", "pmc_counter_collection.csv"),
             [(PROBE, 262144, "FETCH_SIZE", 2097152.0)] + [(k, 256, "FETCH_SIZE", 64.0) for k in ADJ])
        _pmc(os.path.join(tmp, f"prof_adj{g}_write", "pmc_counter_collection.csv"),
             [(PROBE, 262144, "WRITE_SIZE", 4194304.0)] + [(k, 256, "WRITE_SIZE", 32.0) for k in ADJ])
        _pmc(os.path.join(tmp, f"prof_adj{g}_valu", "pmc_counter_collection.csv"),
             [(k, 256, c, v) for k in ADJ for c, v in zip(VALU, (1e5, 4, 1e3, 100, 100, 5e4, 8e3))])
    return n


def test_write_profiles_calibrates_against_the_probes(tmp_path):
    run, out = str(tmp_path / "run"), str(tmp_path / "profiles")
    os.makedirs(run)
    _run_dir(run)
    bench.write_profiles(run, "thermal_wave_4096", out_dir=out)
    with open(os.path.join(out, "traffic.json")) as fh:
        data = json.load(fh)
    assert data["source_hash"] == bench.source_hash()
    for st in STORES:
        sc = data["copy_scale"][st]
        assert abs(sc["fetch"] - 2.0) < 1e-12 and abs(sc["write"] - 1.0) < 1e-12  # 4 GiB / counter bytes
        ent = data["kernels"][f"collide_advect/thermal_wave_4096/{st}"]
        assert ent["fetch_bytes"] == 1000 * 1024 and ent["write_bytes"] == 1600 * 1024
    # 2 x 1000 KiB read + 1600 KiB written = 2.25 x the algorithmic 400 B x 64^2 of an FP32-dev launch
    with open(os.path.join(out, "k_collide_advect_sweep_thermal_wave_4096_f32_dev_counters.md")) as fh:
        text = fh.read()
    assert "| FETCH_SIZE | 1000 KiB (5 dispatches) | x2.000 (3 probes) | 0.002 GB |" in text
    assert "Measured traffic per launch 0.004 GB = 2.250 x the algorithmic 0.002 GB" in text
    assert "3686 GB/s moved, 1638 GB/s algorithmic" in text  # over the 1 us traced launch
    # VALU: 2.4e6 instructions over 100 waves; x 4 cycles / 1024 SIMDs / 2.4 GHz = 3.906 us in a 1 us
    # launch; SQ_ACTIVE_INST_VALU 1.2e6 quad-cycles / 1024 SIMDs over 8e4 / 8 cycles per XCD = 0.47
    assert "| 1000 | 100 | 24000 | 100 | 100 | 3.9 | 1.0 | 3.91 | 0.47 |" in text
    # 4e5 / 1e6 wave cycles waiting on a dependency, 2e5 / 1e6 on anything; 900 L2 hits of 1000
    assert "(SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES) 0.40" in text and "SQ_WAVE_CYCLES), 0.20" in text
    assert "(TCC_HIT + TCC_MISS) 0.900" in text
    # the headline check uses the workload's grid only (1000 threads, 1000 ns) against the events' 1 us
    with open(os.path.join(out, "kernel_trace_thermal_wave_4096.md")) as fh:
        trace = fh.read()
    assert "average 1000 ns" in trace and "(+0.00 %)" in trace
    with open(os.path.join(out, "adjoint_kernels_256_1024.md")) as fh:
        adj = fh.read()
    # 64 KiB x 2 read and 32 KiB written over 256^2 cells: 2 and 0.5 bytes per cell in 0.5 us
    assert "| `k_adjoint_relax<2, StoreF64, 1, double>` | 256 | 1 | 0.5 | 2 | 0 | 328 |" in adj


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N with N > 1 exits (status 2) with a message saying the library runs on one GPU."""
    import subprocess
    import sys

    res = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    msg = json.loads(res.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]
