#!/usr/bin/env python3
"""Throughput of the fused DDF-QE DVBM step on one MI355X.

One "step" is one time step of Eq. (finalDiscretePDE) over the whole grid
(one launch of the fused collide-advect kernel). Default workload: the
4096 x 4096 periodic isobaric thermal wave with a seeded random velocity
perturbation (split II, D2Q25, Pr = 0.5, gamma = 1.4), populations stored
in float32 (float32 arithmetic, float64 per-node moment sums); the float64,
bfloat16-deviation and half-deviation storages of the same workload are
timed after it and reported under "modes".

Prints ONE JSON line. ``value`` is lattice updates per second (MLUPS) of
the default mode with the populations already resident in HBM; the
roofline entry divides the algorithmic HBM bytes of one launch (one read
and one write of the 2Q populations of every cell) by the average launch
duration measured with HIP events on the solver's stream.
"""

from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
STORAGE_BYTES = {"f64": 8, "f32": 4, "bf16_dev": 2, "fp16_dev": 2, "f32_dev": 4}


def source_hash() -> str:
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(ROOT, "paper_2510_04197_amd", "csrc", "*"))):
        with open(path, "rb") as fh:
            h.update(os.path.basename(path).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload_fields(name: str):
    from synth import isentropic_vortex, shock_vortex, thermal_wave

    if name == "thermal_wave_4096":
        wl = thermal_wave(4096, seed=0)
        phys = dict(split=2, Pr=0.5, gamma=1.4, tau_ref=5e-5, bc_x="periodic", bc_y="periodic")
    elif name == "vortex_1024":
        wl = isentropic_vortex(1024, seed=0, mach_adv=1.0, mach_v=0.3, r_frac=0.05)
        phys = dict(split=2, Pr=0.71, gamma=1.4, tau_ref=5e-5, bc_x="periodic", bc_y="periodic")
    elif name == "shock_vortex_2048x1024":
        wl = shock_vortex(2048, 1024, mach_s=1.2, mach_v=0.25, r_frac=0.075, gamma=1.4)
        phys = dict(split=2, Pr=0.71, gamma=1.4, tau_ref=wl.phys["mu"], bc_x="zero_gradient", bc_y="periodic")
    else:
        raise SystemExit(f"unknown workload {name}")
    return wl, phys


def traffic_entry(kernel_key: str):
    """Measured HBM bytes per launch from the committed counter summary, if current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    if data.get("source_hash") != source_hash():
        return None
    ent = data.get("kernels", {}).get(kernel_key)
    if not ent:
        return None
    sc = data["copy_scale"][kernel_key.rsplit("/", 1)[1]]
    return ent["fetch_bytes"] * sc["fetch"] + ent["write_bytes"] * sc["write"]


def step_kernel_name(storage: str, wl) -> str:
    """The step kernel the library launches for this storage and grid size."""
    big = wl.nx * wl.ny >= 3 << 18
    if storage == "f64":
        return "k_collide_advect_sweep" if big else "k_collide_advect_lds"
    pitch = (wl.nx + 63) // 64 * 64
    Q = 25
    if big and pitch * wl.ny * Q * STORAGE_BYTES[storage] <= 1 << 31:
        return "k_collide_advect_sweep"
    return "k_collide_advect"


# rocprofv3 commands whose outputs write_profiles() summarises (run from the repository root on the GPU;
# the trace run's stdout, the bench line, goes to gpurun_out/prof_trace.json)
PROFILE_STORAGES = ("f32_dev", "f64", "bf16_dev")
ADJ_GRIDS = (256, 1024)
_STEP_ARGS = "--steps 20 --warmup 2 --modes none --no-adjoint --no-cpu-baseline --no-shock-vortex"
VALU_COUNTERS = ("SQ_INSTS_VALU SQ_WAVES SQ_INSTS_SALU SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_ACTIVE_INST_VALU "
                 "SQ_BUSY_CYCLES GRBM_GUI_ACTIVE")
STALL_COUNTERS = "SQ_WAIT_INST_ANY SQ_WAIT_ANY SQ_WAVE_CYCLES SQ_BUSY_CYCLES TCC_HIT_sum TCC_MISS_sum"
PROFILE_COMMANDS = {
    "trace": "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_trace -o trace -- "
             "python bench.py",
    **{f"{c}_{st}": f"rocprofv3 --pmc {ctr} --output-format csv -d gpurun_out/prof_{c}_{st} -o pmc -- "
                    f"python bench.py --storage {st} {_STEP_ARGS}"
       for st in PROFILE_STORAGES for c, ctr in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE"),
                                                 ("valu", VALU_COUNTERS), ("stall", STALL_COUNTERS))},
    **{f"adj{n}_trace": f"rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_adj{n}_trace "
                        f"-o trace -- python bench.py --adjoint-kernels {n}" for n in ADJ_GRIDS},
    **{f"adj{n}_{c}": f"rocprofv3 --pmc {ctr} --output-format csv -d gpurun_out/prof_adj{n}_{c} -o pmc -- "
                      f"python bench.py --adjoint-kernels {n} --reps 5"
       for n in ADJ_GRIDS for c, ctr in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE"), ("valu", VALU_COUNTERS))},
}
SIMDS, CLOCK_GHZ = 1024, 2.4  # MI355X: 256 CUs x 4 SIMDs; peak engine clock


def _pmc_rows(path):
    import csv

    with open(path) as fh:
        return list(csv.DictReader(fh))


def _short(name: str) -> str:
    """Kernel instance name without namespaces and argument list."""
    return name.split("(")[0].replace("void ", "").replace("dvbm::", "")


def _counter_by_dispatch(rows, counter):
    """{(instance, grid): [value per dispatch]} of one counter (values summed over the device)."""
    out = {}
    for r in rows:
        if r["Counter_Name"] == counter:
            out.setdefault((_short(r["Kernel_Name"]), int(r["Grid_Size"])), []).append(float(r["Counter_Value"]))
    return out


def _copy_scale(rows, counter):
    """Bytes per counter unit: the probe dispatches that move 4 GiB this way against the counter (KiB)."""
    import statistics

    probes = [float(r["Counter_Value"]) * 1024.0 for r in rows
              if r["Counter_Name"] == counter and "k_stream<" in r["Kernel_Name"]]
    big = [v for v in probes if v >= 0.5 * max(probes)]
    return float(4 << 30) / statistics.median(big), len(big)


def _trace_by_grid(path):
    """{(instance, grid): [duration ns]} from a rocprofv3 kernel trace."""
    import csv
    import gzip

    out = {}
    with (gzip.open(path + ".gz", "rt") if not os.path.exists(path) else open(path)) as fh:
        for r in csv.DictReader(fh):
            g = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"] or 1) * int(r["Grid_Size_Z"] or 1)
            out.setdefault((_short(r["Kernel_Name"]), g), []).append(
                int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return out


def _valu_table(rows, durations, keys):
    """Markdown rows: per-wave VALU / SALU / VMEM instructions, and VALU issue time per SIMD (instructions x
    4 cycles, spread evenly over the SIMDs at the peak clock) against the kernel's traced duration."""
    import statistics

    ctr = {c: _counter_by_dispatch(rows, c) for c in ("SQ_INSTS_VALU", "SQ_WAVES", "SQ_INSTS_SALU",
                                                          "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
                                                          "SQ_ACTIVE_INST_VALU", "GRBM_GUI_ACTIVE")}
    lines = []
    for k in keys:
        if k not in ctr["SQ_INSTS_VALU"]:
            continue
        med = {c: statistics.median(v[k]) for c, v in ctr.items() if k in v}
        waves = med["SQ_WAVES"]
        valu_us = med["SQ_INSTS_VALU"] * 4 / SIMDS / (CLOCK_GHZ * 1e3)
        dur_us = statistics.mean(durations[k]) / 1e3 if k in durations else float("nan")
        # SQ_ACTIVE_INST_VALU counts quad-cycles; GRBM_GUI_ACTIVE sums the 8 XCDs' busy cycles
        busy = (med["SQ_ACTIVE_INST_VALU"] * 4 / SIMDS) / (med["GRBM_GUI_ACTIVE"] / 8)
        lines.append(f"| `{k[0][:70]}` | {k[1]} | {waves:.0f} | {med['SQ_INSTS_VALU'] / waves:.0f} | "
                     f"{med['SQ_INSTS_SALU'] / waves:.0f} | "
                     f"{(med['SQ_INSTS_VMEM_RD'] + med['SQ_INSTS_VMEM_WR']) / waves:.0f} | {valu_us:.1f} | "
                     f"{dur_us:.1f} | {valu_us / dur_us:.2f} | {busy:.2f} |")
    head = ("| kernel | grid (threads) | waves | VALU / wave | SALU / wave | VMEM / wave | VALU issue per SIMD (us) "
            "| duration (us) | issue / duration | SQ_ACTIVE_INST_VALU busy |\n|---|---|---|---|---|---|---|---|---|---|\n")
    return head + "\n".join(lines) + "\n"


def write_profiles(run_dir: str, workload: str, out_dir: str = os.path.join(ROOT, "profiles")) -> None:
    """Summaries in out_dir (profiles/) of the PROFILE_COMMANDS runs, whose outputs are in run_dir (host only).

    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are calibrated against the streaming probes that every
    profiled run makes (stream_ceiling: each dispatch reads or writes 4 GiB, or both): scale = known
    bytes / counter bytes.  Kernel durations come from the kernel traces, split by launch grid."""
    import statistics

    with open(os.path.join(run_dir, "prof_trace.json")) as fh:
        line = json.loads([ln for ln in fh if ln.startswith("{")][-1])
    kname = line["roofline"]["kernel"]
    cells = line["config"]["nx"] * line["config"]["ny"]
    trace = _trace_by_grid(os.path.join(run_dir, "prof_trace", "trace_kernel_trace.csv"))
    os.makedirs(os.path.join(out_dir), exist_ok=True)
    store = {"f64": "StoreF64", "f32": "StoreF32", "bf16_dev": "StoreBF16", "fp16_dev": "StoreF16",
             "f32_dev": "StoreF32Dev"}
    data = {"kernels": {}, "source_hash": source_hash()}

    # ---- kernel trace of the default bench run, by instance and grid
    name = f"kernel_trace_{workload}"
    with open(os.path.join(out_dir, f"{name}.md"), "w") as fh:
        fh.write(f"# Kernel trace of the default bench run ({workload} and the bench's other workloads)\n\n")
        fh.write(f"Command (repository root, one MI355X):\n\n    {PROFILE_COMMANDS['trace']} "
                 f"> gpurun_out/prof_trace.json\n\n")
        fh.write("Launches of the library's kernels, split by launch grid (threads), the 14 largest by total "
                 "time:\n\n| kernel | grid (threads) | calls | average us | total ms |\n|---|---|---|---|---|\n")
        lib = {k: v for k, v in trace.items() if k[0].startswith(("k_", "dvbm"))}
        for k in sorted(lib, key=lambda k: -sum(lib[k]))[:14]:
            v = lib[k]
            fh.write(f"| `{k[0][:80]}` | {k[1]} | {len(v)} | {statistics.mean(v) / 1e3:.1f} | {sum(v) / 1e6:.1f} |\n")
        inst = f"{kname}<{line['config']['split']}, {store[line['config']['storage']]},"
        keys = [k for k in trace if k[0].startswith(inst)]
        kmax = max(keys, key=lambda k: k[1])
        avg_ns = statistics.mean(trace[kmax])
        ms_ev = line["ms_per_step"]
        alg = line["roofline"]["bytes_per_update"] * cells
        fh.write(f"\nHeadline check: the {len(trace[kmax])} launches of `{kmax[0]}` on the "
                 f"{line['config']['nx']} x {line['config']['ny']} grid ({kmax[1]} threads) average {avg_ns:.0f} ns; "
                 f"the bench line of the same run times a launch at {ms_ev * 1e6:.0f} ns with HIP events on the "
                 f"solver stream ({100 * (avg_ns / (ms_ev * 1e6) - 1):+.2f} %). Algorithmic bytes per launch "
                 f"{alg / 1e9:.3f} GB -> {alg / avg_ns:.0f} GB/s by the trace, {line['roofline']['achieved']} GB/s "
                 f"by the events ({line['value']} MLUPS).\n")

    # ---- per storage: calibrated HBM traffic and VALU issue of the step kernel on the workload's grid
    for st in PROFILE_STORAGES:
        fr = _pmc_rows(os.path.join(run_dir, f"prof_fetch_{st}", "pmc_counter_collection.csv"))
        wr = _pmc_rows(os.path.join(run_dir, f"prof_write_{st}", "pmc_counter_collection.csv"))
        vr = _pmc_rows(os.path.join(run_dir, f"prof_valu_{st}", "pmc_counter_collection.csv"))
        sf, nsf = _copy_scale(fr, "FETCH_SIZE")
        sw, nsw = _copy_scale(wr, "WRITE_SIZE")
        inst = f"{kname}<{line['config']['split']}, {store[st]},"
        fd = {k: v for k, v in _counter_by_dispatch(fr, "FETCH_SIZE").items() if k[0].startswith(inst)}
        wd = {k: v for k, v in _counter_by_dispatch(wr, "WRITE_SIZE").items() if k[0].startswith(inst)}
        k = max(fd, key=lambda k: k[1])
        fetch, write = statistics.median(fd[k]) * 1024.0, statistics.median(wd[k]) * 1024.0
        alg = 2 * 2 * 25 * STORAGE_BYTES[st] * cells
        data["kernels"][f"collide_advect/{workload}/{st}"] = {"fetch_bytes": fetch, "write_bytes": write,
                                                              "kernel": kname}
        data.setdefault("copy_scale", {})[st] = {"fetch": sf, "write": sw}
        tk = [t for t in trace if t[0].startswith(inst)]
        tk = max(tk, key=lambda t: t[1]) if tk else None
        dur = statistics.mean(trace[tk]) if tk else float("nan")
        tot = fetch * sf + write * sw
        with open(os.path.join(out_dir, f"{kname}_{workload}_{st}_counters.md"), "w") as fh:
            fh.write(f"# {kname}: HBM traffic and instruction issue, {workload}, {st} storage\n\n")
            fh.write("Commands (repository root, one MI355X):\n\n")
            for c in ("fetch", "write", "valu", "stall"):
                fh.write(f"    {PROFILE_COMMANDS[f'{c}_{st}']}\n")
            fh.write(f"\nKernel duration from `{PROFILE_COMMANDS['trace']}` (the {st} launches on the full grid).\n\n")
            fh.write("| counter | kernel, per dispatch (median) | calibration (4 GiB probes) | scaled bytes | "
                     "algorithmic |\n|---|---|---|---|---|\n")
            fh.write(f"| FETCH_SIZE | {fetch / 1024:.0f} KiB ({len(fd[k])} dispatches) | x{sf:.3f} ({nsf} probes) | "
                     f"{fetch * sf / 1e9:.3f} GB | {alg / 2e9:.3f} GB read |\n")
            fh.write(f"| WRITE_SIZE | {write / 1024:.0f} KiB ({len(wd[k])} dispatches) | x{sw:.3f} ({nsw} probes) | "
                     f"{write * sw / 1e9:.3f} GB | {alg / 2e9:.3f} GB written |\n")
            fh.write(f"\nMeasured traffic per launch {tot / 1e9:.3f} GB = {tot / alg:.3f} x the algorithmic "
                     f"{alg / 1e9:.3f} GB (one read and one write of the 2Q populations of every cell); "
                     f"over the traced duration {dur / 1e3:.0f} us: {tot / dur:.0f} GB/s moved, "
                     f"{alg / dur:.0f} GB/s algorithmic.\n\n")
            vk = [t for t in _counter_by_dispatch(vr, "SQ_INSTS_VALU") if t[0].startswith(inst)]
            fh.write("Instruction issue (VALU issue per SIMD = VALU instructions x 4 cycles / 1024 SIMDs at "
                     f"{CLOCK_GHZ} GHz, the share of the duration the SIMDs would need for VALU issue alone):\n\n")
            fh.write(_valu_table(vr, {t: trace[tk] for t in vk} if tk else {}, vk))
            sr = _pmc_rows(os.path.join(run_dir, f"prof_stall_{st}", "pmc_counter_collection.csv"))
            sc = {c: _counter_by_dispatch(sr, c) for c in STALL_COUNTERS.split()}
            sk = [t for t in sc["SQ_WAVE_CYCLES"] if t[0].startswith(inst)]
            if sk:
                t = max(sk, key=lambda t: t[1])
                med = {c: statistics.median(v[t]) for c, v in sc.items() if t in v}
                hit = med["TCC_HIT_sum"] / (med["TCC_HIT_sum"] + med["TCC_MISS_sum"])
                fh.write(f"\nStalls and L2 (median over {len(sc['SQ_WAVE_CYCLES'][t])} dispatches): waves wait on a "
                         f"dependency (SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES) {med['SQ_WAIT_INST_ANY'] / med['SQ_WAVE_CYCLES']:.2f} "
                         f"of their cycles and on anything, barriers included (SQ_WAIT_ANY / SQ_WAVE_CYCLES), "
                         f"{med['SQ_WAIT_ANY'] / med['SQ_WAVE_CYCLES']:.2f}; L2 hit rate "
                         f"TCC_HIT / (TCC_HIT + TCC_MISS) {hit:.3f}.\n")

    # ---- the adjoint kernels (and the forward step they are compared with) at 256^2 and 1024^2
    with open(os.path.join(out_dir, "adjoint_kernels_256_1024.md"), "w") as fh:
        fh.write("# Adjoint and forward step kernels, 256^2 and 1024^2 periodic (smooth random T)\n\n")
        fh.write("Commands (repository root, one MI355X):\n\n")
        for n in ADJ_GRIDS:
            for c in ("trace", "fetch", "write", "valu"):
                fh.write(f"    {PROFILE_COMMANDS[f'adj{n}_{c}']}\n")
        fh.write("\nDurations from the traces; HBM bytes per cell from FETCH_SIZE and WRITE_SIZE calibrated on the "
                 "4 GiB probes of the same run. Instances: split II; storage F64 / F32 / F32-dev; the last template "
                 "argument of the adjoint kernels is the cotangent type.\n")
        for n in ADJ_GRIDS:
            at = _trace_by_grid(os.path.join(run_dir, f"prof_adj{n}_trace", "trace_kernel_trace.csv"))
            fr = _pmc_rows(os.path.join(run_dir, f"prof_adj{n}_fetch", "pmc_counter_collection.csv"))
            wr = _pmc_rows(os.path.join(run_dir, f"prof_adj{n}_write", "pmc_counter_collection.csv"))
            vr = _pmc_rows(os.path.join(run_dir, f"prof_adj{n}_valu", "pmc_counter_collection.csv"))
            sf, _ = _copy_scale(fr, "FETCH_SIZE")
            sw, _ = _copy_scale(wr, "WRITE_SIZE")
            fd, wd = _counter_by_dispatch(fr, "FETCH_SIZE"), _counter_by_dispatch(wr, "WRITE_SIZE")
            keys = sorted(k for k in at if k[0].startswith(("k_adjoint_relax", "k_adjoint_flux", "k_collide_advect")))
            cells = n * n
            fh.write(f"\n## {n} x {n} (calibration x{sf:.3f} fetch, x{sw:.3f} write)\n\n"
                     "| kernel | grid (threads) | calls | average us | read B/cell | written B/cell | GB/s |\n"
                     "|---|---|---|---|---|---|---|\n")
            for k in keys:
                us = statistics.mean(at[k]) / 1e3
                rb = statistics.median(fd[k]) * 1024.0 * sf / cells if k in fd else float("nan")
                wb = statistics.median(wd[k]) * 1024.0 * sw / cells if k in wd else float("nan")
                fh.write(f"| `{k[0][:78]}` | {k[1]} | {len(at[k])} | {us:.1f} | {rb:.0f} | {wb:.0f} | "
                         f"{(rb + wb) * cells / (us * 1e3):.0f} |\n")
            fh.write("\nInstruction issue (as in the step kernels' counter summaries):\n\n")
            vk = [k for k in keys if k in _counter_by_dispatch(vr, "SQ_INSTS_VALU")]
            fh.write(_valu_table(vr, {k: at[k] for k in vk}, vk))
    with open(os.path.join(out_dir, "traffic.json"), "w") as fh:
        json.dump(data, fh, indent=1)
        fh.write("\n")
    print("profiles written:", ", ".join(sorted(data["kernels"])))


def wave_amplitude(T):
    """|T_k| of the y-mode sin(2 pi y / L) of a field T[y, x] (float64 projection of the x-average)."""
    import math

    import torch

    ny = T.shape[0]
    y = (torch.arange(ny, dtype=torch.float64, device=T.device) + 0.5) / ny
    prof = (T - T.mean()).mean(dim=1)
    re = (prof * torch.cos(2 * math.pi * y)).mean()
    im = (prof * torch.sin(2 * math.pi * y)).mean()
    return 2.0 * math.hypot(float(re), float(im))


def time_mode(wl, phys, storage, steps, warmup, device, total_steps=0, amplitude=False):
    """Times ``steps`` launches after ``warmup``; then, untimed, runs on to
    ``total_steps`` in all before the fields are read (the precision sweep's
    step count).  With ``amplitude``, the thermal wave's mode is also projected
    at step 0 and at the end, and its decay rate over the run gives the thermal
    diffusivity alpha (T_k(t) = T_k(0) exp(-alpha k^2 t))."""
    import math

    import torch

    from paper_2510_04197_amd import Solver, make_params

    p = make_params(wl.nx, wl.ny, dx=wl.dx, dy=wl.dy, storage=storage, **phys)
    s = Solver(p, wl.rho, wl.ux, wl.uy, wl.T, device=device)
    stream = s.stream
    amp0 = wave_amplitude(s.moments(fields=True, sums=False)["T"]) if amplitude else None
    s.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    if total_steps > warmup + steps:
        s.step(total_steps - warmup - steps)
    mom = s.moments(fields=True)
    sums = mom["sums"]
    fields = {"rho": mom["rho"], "T": mom["T"]}
    Q = s.Q
    cells = wl.nx * wl.ny
    bytes_per_update = 2 * (2 * Q) * STORAGE_BYTES[storage]
    ms_launch = ms / steps
    out = {
        "storage": storage,
        "ms_per_step": ms_launch,
        "MLUPS": cells * steps / (ms * 1e-3) / 1e6,
        "GBps": bytes_per_update * cells / (ms_launch * 1e-3) / 1e9,
        "bytes_per_update": bytes_per_update,
        "wall_s": wall,
        "finite": bool(all(map(lambda v: v == v, sums))),
        "dt": s.dt,
    }
    out["frac"] = out["GBps"] / HBM_PEAK_GBPS
    if amplitude:
        t = max(total_steps, warmup + steps) * s.dt
        amp1 = wave_amplitude(fields["T"])
        out["alpha"] = math.log(amp0 / amp1) / ((2 * math.pi / wl.Ly) ** 2 * t) if amp1 > 0 else None
    s.close()
    del s
    torch.cuda.empty_cache()
    return out, fields


def precision_errors(fields, ref):
    """Relative L2 errors of rho and T against the float64-storage run of the same steps."""
    import torch

    out = {}
    for k in ("rho", "T"):
        out[f"rel_L2_{k}"] = float(torch.linalg.vector_norm(fields[k] - ref[k]) / torch.linalg.vector_norm(ref[k]))
        dev = ref[k] - ref[k].mean()
        out[f"rel_L2_{k}_of_variation"] = float(torch.linalg.vector_norm(fields[k] - ref[k])
                                                / torch.linalg.vector_norm(dev))
    return out


def vortex_precision(device, nsteps=5000):
    """The 1024^2 Mach-1 isentropic vortex over its 5000 steps: relative L2 of
    rho and T of each float32 storage against the float64-storage run, on the
    full grid and on the 128^2 grid of 8 x 8 block averages."""
    import torch

    from paper_2510_04197_amd import Solver, make_params

    wl, phys = workload_fields("vortex_1024")
    fields = {}
    for st in ("f64", "f32", "f32_dev"):
        s = Solver(make_params(wl.nx, wl.ny, dx=wl.dx, dy=wl.dy, storage=st, **phys), wl.rho, wl.ux, wl.uy, wl.T,
                   device=device)
        s.step(nsteps)
        m = s.moments(fields=True, sums=False)
        fields[st] = {k: m[k] for k in ("rho", "T")}
        s.close()
    pool = torch.nn.functional.avg_pool2d
    out = {"workload": "vortex_1024", "steps": nsteps, "reference": "float64-storage GPU run"}
    for st in ("f32", "f32_dev"):
        for k in ("rho", "T"):
            a, b = fields[st][k], fields["f64"][k]
            out.setdefault(st, {})[f"rel_L2_{k}"] = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
            a8, b8 = pool(a[None, None], 8), pool(b[None, None], 8)
            out[st][f"rel_L2_{k}_128"] = float(torch.linalg.vector_norm(a8 - b8) / torch.linalg.vector_norm(b8))
    return out


def shock_vortex_runs(device, nsteps=8000, timed=50):
    """The 2048 x 1024 shock-vortex workload (Ma_s 1.2, Ma_v 0.25, x zero-gradient, y periodic) for
    the six (Pr, gamma) pairs Pr in {0.1, 0.71, 2}, gamma in {1.4, 5/3}: each float32 storage against
    the float64-storage run after nsteps steps (relative L2 of rho and T, full grid and 8 x 8 block
    averages), and the step throughput of each storage (HIP events over the first `timed` steps)."""
    import torch

    from paper_2510_04197_amd import Solver, make_params
    from synth import shock_vortex

    pool = torch.nn.functional.avg_pool2d
    out = {"workload": "shock_vortex_2048x1024", "steps": nsteps, "reference": "float64-storage GPU run",
           "pairs": []}
    for Pr in (0.1, 0.71, 2.0):
        for gamma in (1.4, 5.0 / 3.0):
            wl = shock_vortex(2048, 1024, mach_s=1.2, mach_v=0.25, r_frac=0.075, gamma=gamma)
            res, fields = {"Pr": Pr, "gamma": round(gamma, 6)}, {}
            for st in ("f64", "f32", "f32_dev"):
                p = make_params(wl.nx, wl.ny, dx=wl.dx, dy=wl.dy, split=2, storage=st, Pr=Pr, gamma=gamma,
                                tau_ref=wl.phys["mu"], bc_x="zero_gradient", bc_y="periodic")
                s = Solver(p, wl.rho, wl.ux, wl.uy, wl.T, device=device)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(s.stream)
                s.step(timed)
                e1.record(s.stream)
                s.step(nsteps - timed)
                m = s.moments(fields=True, sums=False)
                ms = e0.elapsed_time(e1) / timed
                res[f"{st}_MLUPS"] = round(wl.nx * wl.ny / (ms * 1e-3) / 1e6, 1)
                res[f"{st}_frac"] = round(2 * 50 * STORAGE_BYTES[st] * wl.nx * wl.ny / (ms * 1e-3) / 1e9
                                          / HBM_PEAK_GBPS, 4)
                fields[st] = {k: m[k] for k in ("rho", "T")}
                s.close()
            for st in ("f32", "f32_dev"):
                for k in ("rho", "T"):
                    a, b = fields[st][k], fields["f64"][k]
                    res[f"{st}_rel_L2_{k}"] = float("%.3g" % float(torch.linalg.vector_norm(a - b)
                                                                   / torch.linalg.vector_norm(b)))
                    a8, b8 = pool(a[None, None], 8), pool(b[None, None], 8)
                    res[f"{st}_rel_L2_{k}_8x8"] = float("%.3g" % float(torch.linalg.vector_norm(a8 - b8)
                                                                       / torch.linalg.vector_norm(b8)))
            out["pairs"].append(res)
            del fields
            torch.cuda.empty_cache()
    return out


def adjoint_cost(device, n=256, nsteps=200, storages=("f64", "f32", "f32_dev"), Ks=(10, 50)):
    """Gradient of L = sum (T(200 steps) - T_target)^2 w.r.t. T0, tau_ref, Pr on the 256^2 periodic
    Gaussian-bump workload: time of forward + checkpointed recomputation + reverse sweep, divided by
    the time of the plain forward run, for each storage, checkpoint interval and cotangent type.
    Each float32 storage's gradient is compared with the float64-storage one, which the tests check
    against the oracle's reverse mode (1e-10); the "at 1e-5" ratio is that of the cheapest storage
    whose gradient is within 1e-5 of it."""
    import numpy as np
    import torch

    from paper_2510_04197_amd import Solver, make_params, rollout_temperature
    from synth import gaussian_bump, smooth_random

    bump = gaussian_bump(n, seed=7, amp=0.1, width=0.1)
    T0 = smooth_random(n, n, seed=13, amp_rho=0.0, amp_u=0.0, amp_T=0.05, mean_u=(0.0, 0.0)).T
    ones, zeros = np.ones((n, n)), np.zeros((n, n))
    tau0, Pr = 2e-3, 0.71

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    res = {"workload": f"gaussian bump {n}x{n} periodic, {nsteps} steps, dt 1e-4", "storages": {}}
    grads, grads32 = {}, {}
    # one target for every storage: the float64 run from the hidden bump
    tgt = rollout_temperature(torch.tensor(bump.T, device=device), torch.tensor(tau0, dtype=torch.float64),
                              torch.tensor(Pr, dtype=torch.float64), ones, zeros, zeros, nsteps, K=50,
                              dx=1.0 / n, dy=1.0 / n, split=2, storage="f64", dt=1e-4).detach()
    for storage in storages:
        kw = dict(dx=1.0 / n, dy=1.0 / n, split=2, storage=storage, dt=1e-4)
        p = make_params(n, n, tau_ref=tau0, Pr=Pr, **kw)

        def forward_only():
            s = Solver(p, ones, zeros, zeros, T0, device=device)
            s.step(nsteps)
            T = s.moments(fields=True, sums=False)["T"]
            s.close()
            return T

        def with_gradient(K, cotangent="f64", overlap=False):
            T0t = torch.tensor(T0, device=device, requires_grad=True)
            tau = torch.tensor(tau0, dtype=torch.float64, requires_grad=True)
            prt = torch.tensor(Pr, dtype=torch.float64, requires_grad=True)
            out = rollout_temperature(T0t, tau, prt, ones, zeros, zeros, nsteps, K=K, cotangent=cotangent,
                                      overlap=overlap, **kw)
            ((out - tgt) ** 2).sum().backward()
            return T0t.grad, tau.grad, prt.grad

        t_fwd = timed(forward_only)
        r = {"forward_s": t_fwd}
        for K in Ks:
            r[f"K{K}_ratio"] = timed(lambda: with_gradient(K)) / t_fwd
            r[f"K{K}_f32_cotangent_ratio"] = timed(lambda: with_gradient(K, "f32")) / t_fwd
            # the next segment recomputed on a second stream during each reverse sweep (same gradient, bit for bit)
            r[f"K{K}_overlap_ratio"] = timed(lambda: with_gradient(K, overlap=True)) / t_fwd
            r[f"K{K}_f32_cotangent_overlap_ratio"] = timed(lambda: with_gradient(K, "f32", True)) / t_fwd
        grads[storage] = with_gradient(Ks[0])
        grads32[storage] = g32 = with_gradient(Ks[0], "f32")
        r["f32_cotangent_rel_err"] = float(torch.linalg.vector_norm(g32[0] - grads[storage][0])
                                           / torch.linalg.vector_norm(grads[storage][0]))
        res["storages"][storage] = r
    g64 = grads["f64"]

    def errs(g):
        return {"T0": float(torch.linalg.vector_norm(g[0] - g64[0]) / torch.linalg.vector_norm(g64[0])),
                "tau_ref": float(abs(g[1] - g64[1]) / abs(g64[1])), "Pr": float(abs(g[2] - g64[2]) / abs(g64[2]))}

    for storage in storages:
        r = res["storages"][storage]
        r["gradient_rel_err_vs_f64"] = errs(grads[storage])
        r["f32_cotangent_gradient_rel_err_vs_f64"] = errs(grads32[storage])
        r[f"K{Ks[0]}_gradient_s"] = r[f"K{Ks[0]}_ratio"] * r["forward_s"]
    # every (storage, cotangent) pair whose gradient is within 1e-5 of the float64 one, with or without
    # the overlapped recomputation; the headline ratio is the lowest among them
    ok = [(st, cot) for st in storages for cot in ("f64", "f32")
          if max(res["storages"][st]["gradient_rel_err_vs_f64" if cot == "f64"
                                     else "f32_cotangent_gradient_rel_err_vs_f64"].values()) <= 1e-5]

    def ratio(st, cot, ovl, K):
        return res["storages"][st][f"K{K}_{'f32_cotangent_' if cot == 'f32' else ''}{'overlap_' if ovl else ''}ratio"]

    best = min(((st, cot, ovl) for st, cot in ok for ovl in (False, True)), key=lambda c: ratio(*c, Ks[0]))
    res["at_1e-5"] = {"storage": best[0], "cotangent": best[1], "overlap": best[2],
                      **{f"K{K}_ratio": ratio(*best, K) for K in Ks},
                      "within_1e-5": [f"{st}/{cot}" for st, cot in ok]}
    return res


def adjoint_kernels(device, n, reps):
    """Per-step times (HIP events on the solver stream) of the forward step and of the adjoint step with
    float64 and float32 cotangents, for the F64, F32 and F32-dev storages on an n x n periodic grid with a
    smooth random temperature (split II, tau_ref 2e-3, Pr 0.71, dt 1e-4): the kernels whose costs make up
    the gradient/forward ratio, for profiling them by launch."""
    import numpy as np
    import torch

    from paper_2510_04197_amd import Solver, make_params
    from synth import smooth_random

    T0 = smooth_random(n, n, seed=13, amp_rho=0.0, amp_u=0.0, amp_T=0.05, mean_u=(0.0, 0.0)).T
    ones, zeros = np.ones((n, n)), np.zeros((n, n))
    out = {"grid": n, "reps": reps, "storages": {}}
    for st in ("f64", "f32", "f32_dev"):
        p = make_params(n, n, dx=1.0 / n, dy=1.0 / n, split=2, storage=st, tau_ref=2e-3, Pr=0.71, dt=1e-4)
        s = Solver(p, ones, zeros, zeros, T0, device=device)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.step(2)
        e0.record(s.stream)
        s.step(reps)
        e1.record(s.stream)
        torch.cuda.synchronize()
        r = {"forward_us": e0.elapsed_time(e1) / reps * 1e3}
        state = s.state_buffer.clone()
        gen = torch.Generator(device=device).manual_seed(17)
        for dt in (torch.float64, torch.float32):
            lam = s.new_cotangent(dt)
            lam.copy_(torch.randn(lam.shape, generator=gen, device=device, dtype=torch.float64))
            lam2 = torch.empty_like(lam)
            dp = torch.zeros(2, dtype=torch.float64, device=device)
            s.adjoint_step(state, lam, lam2, dp)
            e0.record(s.stream)
            for _ in range(reps):
                s.adjoint_step(state, lam, lam2, dp)
            e1.record(s.stream)
            torch.cuda.synchronize()
            r[f"adjoint_us_{'f64' if dt == torch.float64 else 'f32'}_cotangent"] = e0.elapsed_time(e1) / reps * 1e3
        out["storages"][st] = r
        s.close()
        torch.cuda.empty_cache()
    return out


def stream_ceiling(device, nbytes=4 << 30, reps=5):
    """HBM GB/s of the library's plain streaming kernels (dvbm_stream_probe) over 4 GiB buffers:
    copy and read with 16-byte lane accesses, plain and non-temporal, write with 16-byte accesses,
    and copy with 4-byte ones (the width of the step kernels' loads).  The best copy is the
    practical ceiling of a kernel that reads and writes about equally."""
    import torch

    from paper_2510_04197_amd import dvbm

    a = torch.zeros(nbytes, dtype=torch.uint8, device=device)
    b = torch.zeros_like(a)
    stream = torch.cuda.current_stream(device)
    out = {}
    for name, mode, width, moved in (("copy16", 0, 16, 2), ("copy16_nt", 4, 16, 2), ("read16", 1, 16, 1),
                                     ("read16_nt", 5, 16, 1), ("write16", 2, 16, 1), ("copy4", 0, 4, 2)):
        dvbm.stream_probe(a, b, nbytes, mode, width, stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            dvbm.stream_probe(a, b, nbytes, mode, width, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = round(moved * nbytes / (ms * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n=256, steps=200, n1=128, steps1=20):
    """The FP64 oracle on the host, timed on the thermal-wave family: an n x n
    sample of `steps` steps with torch's default thread count, and an n1 x n1
    sample of `steps1` steps on one thread (about the same CPU time)."""
    import numpy as np
    import torch

    from oracle import dvbm_oracle as O
    from synth import thermal_wave

    def timed(m, k):
        wl = thermal_wave(m, seed=0)
        cfg = O.Config(nx=m, ny=m, split=2, dx=wl.dx, dy=wl.dy, Pr=0.5, gamma=1.4, tau_ref=5e-5)
        f, g = O.initial_state(wl.rho, wl.ux, wl.uy, wl.T, cfg)
        dt = O.time_step(wl.rho, np.stack([wl.ux, wl.uy], -1), wl.T, cfg)
        t0 = time.perf_counter()
        O.run(f, g, cfg, dt, k)
        return time.perf_counter() - t0

    threads = torch.get_num_threads()
    t = timed(n, steps)
    torch.set_num_threads(1)
    try:
        t1 = timed(n1, steps1)
    finally:
        torch.set_num_threads(threads)
    return {"value": n * n * steps / t / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"thermal wave on a {n}x{n} periodic grid, {steps} float64 steps (split II, D2Q25)",
            "seconds": t, "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "single_thread": {"value": n1 * n1 * steps1 / t1 / 1e6, "unit": "MLUPS", "seconds": t1,
                              "sample": f"{n1}x{n1} grid, {steps1} steps, 1 thread"}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="thermal_wave_4096")
    # float32 deviations from the rest state: float32's bytes and speed, and within 1e-5 of float64 storage
    # over the thermal wave's 2000 steps, where float32 values drift by 2e-5
    ap.add_argument("--storage", default="f32_dev", choices=sorted(STORAGE_BYTES))
    ap.add_argument("--modes", default="f64,f32,bf16_dev,fp16_dev",
                    help="extra storages timed after the main one ('none' to skip)")
    ap.add_argument("--precision-steps", type=int, default=2000,
                    help="steps (timed ones included) after which the storage modes are compared with float64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward cost measurement")
    ap.add_argument("--no-shock-vortex", action="store_true", help="skip the 2048x1024 shock-vortex runs")
    ap.add_argument("--adjoint-kernels", type=int, metavar="N",
                    help="only time the forward and adjoint step kernels on an N x N grid (for profiling)")
    ap.add_argument("--reps", type=int, default=50, help="launches per kernel timed by --adjoint-kernels")
    ap.add_argument("--write-profiles", metavar="RUN_DIR",
                    help="host only: summarise the rocprofv3 runs of PROFILE_COMMANDS (outputs in RUN_DIR) into "
                         "profiles/")
    args = ap.parse_args()

    if args.write_profiles:
        write_profiles(args.write_profiles, workload=args.workload)
        return

    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; multi-GPU runs (domain decomposition with "
                                   "halo exchange) are not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    device = "cuda:0"
    if args.adjoint_kernels:
        res = adjoint_kernels(device, args.adjoint_kernels, args.reps)
        res["stream_probe_GBps"] = stream_ceiling(device)  # the counter calibration of a profiled run
        print(json.dumps({"adjoint_kernels": res}))
        return
    print(f"[bench] workload {args.workload}, storage {args.storage}, steps {args.steps}, warmup {args.warmup}",
          file=sys.stderr, flush=True)
    wl, phys = workload_fields(args.workload)
    mode_list = [st for st in args.modes.split(",") if st and st != args.storage] if args.modes != "none" else []
    total = args.precision_steps if "f64" in mode_list + [args.storage] and mode_list else 0
    wave = args.workload == "thermal_wave_4096" and total > 0
    main, main_fields = time_mode(wl, phys, args.storage, args.steps, args.warmup, device, total, amplitude=wave)
    print(f"[bench] {args.storage}: {main['MLUPS']:.1f} MLUPS, {main['GBps']:.1f} GB/s", file=sys.stderr, flush=True)
    modes = {}
    fields = {args.storage: main_fields}
    for st in mode_list:
        modes[st], fields[st] = time_mode(wl, phys, st, args.steps, args.warmup, device, total, amplitude=wave)
        print(f"[bench] {st}: {modes[st]['MLUPS']:.1f} MLUPS, {modes[st]['GBps']:.1f} GB/s",
              file=sys.stderr, flush=True)
    precision = None
    if "f64" in fields and len(fields) > 1:
        precision = {"reference": "float64-storage GPU run of the same workload and step count",
                     "steps": max(total, args.warmup + args.steps)}
        for st, fl in fields.items():
            if st != "f64":
                precision[st] = precision_errors(fl, fields["f64"])
        if wave:
            # decay rate of the thermal wave's mode in each storage's run.  The run lasts 4e-3 time
            # units, 0.5 % of the acoustic time L / c, so the density has not moved: T decays at the
            # isochoric diffusivity kappa / (rho c_v) = gamma nu / Pr (nu = mu / rho, rho ~ 1), and the
            # heat flux, zero in the initial equilibrium, reaches its Fourier value after about the
            # thermal relaxation time tau_alpha = mu / (p Pr), which the elapsed time loses
            alphas = {args.storage: main["alpha"], **{k: v["alpha"] for k, v in modes.items()}}
            nu_pr = phys["tau_ref"] / phys["Pr"]  # mu / (rho Pr), rho ~ 1 (mu = tau_ref p_ref, p_ref = 1)
            tau_alpha = phys["tau_ref"] / phys["Pr"]  # mu / (p Pr), the wave being isobaric at p = 1
            t_run = precision["steps"] * main["dt"]
            expected = phys["gamma"] * nu_pr * (1.0 - tau_alpha / t_run)
            precision["conductivity"] = {
                "nu_over_Pr": nu_pr, "t": t_run,
                "expected_decay_rate_over_k2": expected,
                "note": "expected = gamma (nu/Pr) (1 - tau_alpha/t): isochoric decay over a run much shorter "
                        "than the acoustic time, heat flux starting from zero",
                **{st: {"alpha": a, "over_expected": a / expected if a else None,
                        "rel_to_f64": (a / alphas["f64"] - 1) if a and alphas.get("f64") else None}
                   for st, a in alphas.items()}}
    del fields, main_fields
    vortex = None
    if precision is not None:
        print("[bench] float32 precision on the 1024x1024 vortex, 5000 steps", file=sys.stderr, flush=True)
        vortex = vortex_precision(device)
    shock = None
    if not args.no_shock_vortex and args.workload == "thermal_wave_4096":
        print("[bench] shock-vortex 2048x1024, six (Pr, gamma), 8000 steps", file=sys.stderr, flush=True)
        shock = shock_vortex_runs(device)
    adjoint = None
    if not args.no_adjoint:
        print("[bench] adjoint cost on the 256x256 gradient workload", file=sys.stderr, flush=True)
        adjoint = adjoint_cost(device)
    ceiling = stream_ceiling(device)

    kernel_key = f"collide_advect/{args.workload}/{args.storage}"
    traffic = traffic_entry(kernel_key)
    roofline = {"bound": "hbm", "achieved": round(main["GBps"], 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(main["frac"], 4), "traffic": traffic,
                "bytes_per_update": main["bytes_per_update"], "kernel": step_kernel_name(args.storage, wl),
                "copy_kernel_GBps": max(ceiling["copy16"], ceiling["copy16_nt"]), "stream_probe_GBps": ceiling,
                "frac_of_copy": round(main["GBps"] / max(ceiling["copy16"], ceiling["copy16_nt"]), 4)}
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline()
    split = phys["split"]
    line = {
        "metric": "MLUPS + % HBM peak (FP32 vs FP64 vs BF16-store); adjoint/forward time at 1e-5 err",
        "value": round(main["MLUPS"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.storage == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}", "nx": wl.nx, "ny": wl.ny, "split": split,
                   "velocity_set": "D2Q25" if split == 2 else "D2Q16", "storage": args.storage,
                   "Pr": phys["Pr"], "gamma": phys["gamma"], "bc": [phys["bc_x"], phys["bc_y"]]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "modes": {k: {kk: (float("%.5g" % vv) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                  for k, v in modes.items()},
        "precision": precision,
        "precision_vortex": vortex,
        "shock_vortex": shock,
        "adjoint": adjoint,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
