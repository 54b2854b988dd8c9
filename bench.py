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
    return ent["fetch_bytes"] * data["copy_scale_fetch"] + ent["write_bytes"] * data["copy_scale_write"]


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


# rocprofv3 commands whose outputs write_profiles() summarises (run from the repository root on the GPU)
PROFILE_COMMANDS = {
    "trace": "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_trace -o trace -- "
             "python bench.py",
    "fetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/prof_fetch -o pmc -- "
             "python bench.py --steps 20 --warmup 2 --modes none --no-adjoint --no-cpu-baseline",
    "write": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/prof_write -o pmc -- "
             "python bench.py --steps 20 --warmup 2 --modes none --no-adjoint --no-cpu-baseline",
}


def write_profiles(trace_dir: str, fetch_csv: str, write_csv: str, bench_json: str, workload: str,
                   storage: str) -> None:
    """Summaries of the three PROFILE_COMMANDS runs under profiles/ (host only, no GPU).

    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are calibrated against the
    streaming probes that bench.py runs (stream_ceiling: every dispatch reads
    or writes 4 GiB, or both): scale = known bytes / counter bytes.
    """
    import csv
    import statistics

    with open(bench_json) as fh:
        line = json.loads([ln for ln in fh if ln.startswith("{")][-1])
    kname = line["roofline"]["kernel"]

    def per_kernel(path, counter):
        vals, copies = [], []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"]) * 1024.0
                if kname + "<" in r["Kernel_Name"]:
                    vals.append(v)
                elif "k_stream<" in r["Kernel_Name"]:
                    copies.append(v)
        big = [v for v in copies if v >= 0.5 * max(copies)]  # the probes that move 4 GiB this way
        return statistics.median(vals), statistics.median(big), len(vals), len(big)

    fetch, fcopy, nf, ncf = per_kernel(fetch_csv, "FETCH_SIZE")
    write, wcopy, nw, ncw = per_kernel(write_csv, "WRITE_SIZE")
    copy_bytes = float(4 << 30)
    sf, sw = copy_bytes / fcopy, copy_bytes / wcopy
    cells = line["config"]["nx"] * line["config"]["ny"]
    alg = line["roofline"]["bytes_per_update"] * cells
    with open(os.path.join(trace_dir, "trace_kernel_stats.csv")) as fh:
        stats = list(csv.DictReader(fh))
    # per-dispatch durations of the step kernel at the bench workload's grid (the largest grid it was
    # launched with: the adjoint measurement launches the same kernel on a small grid)
    store = {"f64": "StoreF64", "f32": "StoreF32", "bf16_dev": "StoreBF16", "fp16_dev": "StoreF16",
             "f32_dev": "StoreF32Dev"}[storage]
    inst = f"{kname}<{line['config']['split']}, dvbm::{store},"
    durs = {}
    with open(os.path.join(trace_dir, "trace_kernel_trace.csv")) as fh:
        for r in csv.DictReader(fh):
            if inst in r["Kernel_Name"]:
                g = int(r["Grid_Size_X"])
                durs.setdefault(g, []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    gmax = max(durs)
    avg_ns = sum(durs[gmax]) / len(durs[gmax])
    key = f"collide_advect/{workload}/{storage}"
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    data = {}
    if os.path.exists(tpath):
        with open(tpath) as fh:
            data = json.load(fh)
    if data.get("source_hash") != source_hash():
        data = {"kernels": {}}
    data.update({"source_hash": source_hash(), "copy_scale_fetch": sf, "copy_scale_write": sw})
    data["kernels"][key] = {"fetch_bytes": fetch, "write_bytes": write, "kernel": kname}
    with open(tpath, "w") as fh:
        json.dump(data, fh, indent=1)
        fh.write("\n")
    name = f"{kname}_{workload}_{storage}"
    rows = sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:8]
    with open(os.path.join(ROOT, "profiles", f"{name}_kernel_trace.md"), "w") as fh:
        fh.write(f"# {kname}: kernel trace, {workload}, {storage} storage\n\n")
        fh.write(f"Command (repository root, one MI355X):\n\n    {PROFILE_COMMANDS['trace']}\n\n")
        fh.write("| kernel | calls | average ns | total ns |\n|---|---|---|---|\n")
        for r in rows:
            fh.write(f"| `{r['Name'][:110]}` | {r['Calls']} | {float(r['AverageNs']):.0f} | {r['TotalDurationNs']} |\n")
        ms_ev = line["ms_per_step"]
        other = sorted(g for g in durs if g != gmax)
        note = (f" (the same instance was also launched with grids of {', '.join(map(str, other))} threads)"
                if other else "")
        fh.write(f"\nThe table averages every launch of a kernel instance{note}. The {len(durs[gmax])} launches "
                 f"of {kname} on the "
                 f"{line['config']['nx']} x {line['config']['ny']} grid ({gmax} threads) average {avg_ns:.0f} ns; "
                 f"the bench line of the same run times it at {ms_ev * 1e6:.0f} ns per launch with HIP events "
                 f"on the solver stream ("
                 f"{100 * (avg_ns / (ms_ev * 1e6) - 1):+.2f} %). Algorithmic bytes per launch "
                 f"{alg / 1e9:.3f} GB -> {alg / avg_ns:.0f} GB/s by the trace average, "
                 f"{line['roofline']['achieved']} GB/s by the events.\n")
    with open(os.path.join(ROOT, "profiles", f"{name}_hbm_traffic.md"), "w") as fh:
        fh.write(f"# {kname}: HBM traffic, {workload}, {storage} storage\n\n")
        fh.write("Commands (repository root, one MI355X):\n\n")
        fh.write(f"    {PROFILE_COMMANDS['fetch']}\n    {PROFILE_COMMANDS['write']}\n\n")
        fh.write("| counter | kernel, per dispatch (median) | copy calibration | scaled bytes | algorithmic |\n")
        fh.write("|---|---|---|---|---|\n")
        fh.write(f"| FETCH_SIZE | {fetch / 1024:.0f} KiB ({nf} dispatches) | 4 GiB probe reads {fcopy / 1024:.0f} KiB "
                 f"-> x{sf:.3f} | {fetch * sf / 1e9:.3f} GB | {alg / 2e9:.3f} GB read |\n")
        fh.write(f"| WRITE_SIZE | {write / 1024:.0f} KiB ({nw} dispatches) | 4 GiB probe writes {wcopy / 1024:.0f} KiB "
                 f"-> x{sw:.3f} | {write * sw / 1e9:.3f} GB | {alg / 2e9:.3f} GB written |\n")
        tot = fetch * sf + write * sw
        fh.write(f"\nMeasured traffic per launch {tot / 1e9:.3f} GB = {tot / alg:.3f} x the algorithmic "
                 f"{alg / 1e9:.3f} GB (one read and one write of the 2Q populations of every cell).\n")
    print(f"profiles written for {key}: trace {avg_ns:.0f} ns, traffic {tot / 1e9:.3f} GB "
          f"(fetch x{sf:.3f}, write x{sw:.3f})")


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
    grads = {}
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

        def with_gradient(K, cotangent="f64"):
            T0t = torch.tensor(T0, device=device, requires_grad=True)
            tau = torch.tensor(tau0, dtype=torch.float64, requires_grad=True)
            prt = torch.tensor(Pr, dtype=torch.float64, requires_grad=True)
            out = rollout_temperature(T0t, tau, prt, ones, zeros, zeros, nsteps, K=K, cotangent=cotangent, **kw)
            ((out - tgt) ** 2).sum().backward()
            return T0t.grad, tau.grad, prt.grad

        t_fwd = timed(forward_only)
        r = {"forward_s": t_fwd}
        for K in Ks:
            r[f"K{K}_ratio"] = timed(lambda: with_gradient(K)) / t_fwd
            r[f"K{K}_f32_cotangent_ratio"] = timed(lambda: with_gradient(K, "f32")) / t_fwd
        grads[storage] = with_gradient(Ks[0])
        g32 = with_gradient(Ks[0], "f32")
        r["f32_cotangent_rel_err"] = float(torch.linalg.vector_norm(g32[0] - grads[storage][0])
                                           / torch.linalg.vector_norm(grads[storage][0]))
        res["storages"][storage] = r
    g64 = grads["f64"]
    for storage in storages:
        g = grads[storage]
        res["storages"][storage]["gradient_rel_err_vs_f64"] = {
            "T0": float(torch.linalg.vector_norm(g[0] - g64[0]) / torch.linalg.vector_norm(g64[0])),
            "tau_ref": float(abs(g[1] - g64[1]) / abs(g64[1])), "Pr": float(abs(g[2] - g64[2]) / abs(g64[2]))}
    for storage in storages:
        r = res["storages"][storage]
        r[f"K{Ks[0]}_gradient_s"] = r[f"K{Ks[0]}_ratio"] * r["forward_s"]
    ok = [st for st in storages if max(res["storages"][st]["gradient_rel_err_vs_f64"].values()) <= 1e-5]
    best = min(ok, key=lambda st: res["storages"][st][f"K{Ks[0]}_ratio"])
    res["at_1e-5"] = {"storage": best, **{f"K{K}_ratio": res["storages"][best][f"K{K}_ratio"] for K in Ks},
                      "storages_within_1e-5": ok}
    return res


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
    ap.add_argument("--write-profiles", nargs=4, metavar=("TRACE_DIR", "FETCH_CSV", "WRITE_CSV", "BENCH_JSON"),
                    help="host only: summarise the rocprofv3 runs of PROFILE_COMMANDS into profiles/")
    args = ap.parse_args()

    if args.write_profiles:
        write_profiles(*args.write_profiles, workload=args.workload, storage=args.storage)
        return

    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; multi-GPU runs (domain decomposition with "
                                   "halo exchange) are not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    device = "cuda:0"
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
