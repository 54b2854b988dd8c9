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
STORAGE_BYTES = {"f64": 8, "f32": 4, "bf16_dev": 2, "fp16_dev": 2}


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


def time_mode(wl, phys, storage, steps, warmup, device):
    import torch

    from paper_2510_04197_amd import Solver, make_params

    p = make_params(wl.nx, wl.ny, dx=wl.dx, dy=wl.dy, storage=storage, **phys)
    s = Solver(p, wl.rho, wl.ux, wl.uy, wl.T, device=device)
    stream = s.stream
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


def adjoint_cost(device, n=256, nsteps=200, storage="f32", Ks=(10, 50)):
    """Gradient of L = sum (T(200 steps) - T_target)^2 w.r.t. T0, tau_ref, Pr on the 256^2 periodic
    Gaussian-bump workload: time of forward + checkpointed recomputation + reverse sweep, divided by
    the time of the plain forward run."""
    import numpy as np
    import torch

    from paper_2510_04197_amd import Solver, make_params, rollout_temperature
    from synth import gaussian_bump, smooth_random

    bump = gaussian_bump(n, seed=7, amp=0.1, width=0.1)
    T0 = smooth_random(n, n, seed=13, amp_rho=0.0, amp_u=0.0, amp_T=0.05, mean_u=(0.0, 0.0)).T
    ones, zeros = np.ones((n, n)), np.zeros((n, n))
    kw = dict(dx=1.0 / n, dy=1.0 / n, split=2, storage=storage, dt=1e-4)
    tau0, Pr = 2e-3, 0.71
    tgt = rollout_temperature(torch.tensor(bump.T, device=device), torch.tensor(tau0, dtype=torch.float64),
                              torch.tensor(Pr, dtype=torch.float64), ones, zeros, zeros, nsteps, K=50,
                              **kw).detach()
    p = make_params(n, n, tau_ref=tau0, Pr=Pr, **kw)

    def forward_only():
        s = Solver(p, ones, zeros, zeros, T0, device=device)
        s.step(nsteps)
        T = s.moments(fields=True, sums=False)["T"]
        s.close()
        return T

    def with_gradient(K):
        T0t = torch.tensor(T0, device=device, requires_grad=True)
        tau = torch.tensor(tau0, dtype=torch.float64, requires_grad=True)
        prt = torch.tensor(Pr, dtype=torch.float64, requires_grad=True)
        out = rollout_temperature(T0t, tau, prt, ones, zeros, zeros, nsteps, K=K, **kw)
        ((out - tgt) ** 2).sum().backward()
        return T0t.grad

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_fwd = timed(forward_only)
    res = {"workload": f"gaussian bump {n}x{n} periodic, {nsteps} steps, {storage} storage",
           "forward_s": t_fwd}
    for K in Ks:
        t = timed(lambda: with_gradient(K))
        res[f"K{K}_s"] = t
        res[f"K{K}_ratio"] = t / t_fwd
    return res


def copy_bandwidth(device, nbytes=4 << 30, reps=5):
    import torch

    a = torch.empty(nbytes, dtype=torch.uint8, device=device)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(n=512, steps=40):
    """The FP64 oracle on the host: same workload family on an n x n sample."""
    import numpy as np
    import torch

    from oracle import dvbm_oracle as O
    from synth import thermal_wave

    wl = thermal_wave(n, seed=0)
    cfg = O.Config(nx=n, ny=n, split=2, dx=wl.dx, dy=wl.dy, Pr=0.5, gamma=1.4, tau_ref=5e-5)
    f, g = O.initial_state(wl.rho, wl.ux, wl.uy, wl.T, cfg)
    dt = O.time_step(wl.rho, np.stack([wl.ux, wl.uy], -1), wl.T, cfg)
    t0 = time.perf_counter()
    O.run(f, g, cfg, dt, steps)
    t = time.perf_counter() - t0
    return {"value": n * n * steps / t / 1e6, "unit": "MLUPS", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"thermal wave on a {n}x{n} periodic grid, {steps} float64 steps (split II, D2Q25)",
            "seconds": t}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="thermal_wave_4096")
    ap.add_argument("--storage", default="f32", choices=sorted(STORAGE_BYTES))
    ap.add_argument("--modes", default="f64,bf16_dev,fp16_dev",
                    help="extra storages timed after the main one ('none' to skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward cost measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs (domain decomposition with "
                                   "halo exchange) are not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    device = "cuda:0"
    print(f"[bench] workload {args.workload}, storage {args.storage}, steps {args.steps}, warmup {args.warmup}",
          file=sys.stderr, flush=True)
    wl, phys = workload_fields(args.workload)
    main, main_fields = time_mode(wl, phys, args.storage, args.steps, args.warmup, device)
    print(f"[bench] {args.storage}: {main['MLUPS']:.1f} MLUPS, {main['GBps']:.1f} GB/s", file=sys.stderr, flush=True)
    modes = {}
    fields = {args.storage: main_fields}
    if args.modes != "none":
        for st in args.modes.split(","):
            if st and st != args.storage:
                modes[st], fields[st] = time_mode(wl, phys, st, args.steps, args.warmup, device)
                print(f"[bench] {st}: {modes[st]['MLUPS']:.1f} MLUPS, {modes[st]['GBps']:.1f} GB/s",
                      file=sys.stderr, flush=True)
    precision = None
    if "f64" in fields:
        precision = {"reference": "float64-storage GPU run of the same workload and step count",
                     "steps": args.warmup + args.steps}
        for st, fl in fields.items():
            if st != "f64":
                precision[st] = precision_errors(fl, fields["f64"])
    del fields, main_fields
    adjoint = None
    if not args.no_adjoint:
        print("[bench] adjoint cost on the 256x256 gradient workload", file=sys.stderr, flush=True)
        adjoint = adjoint_cost(device)
    copy_gbps = copy_bandwidth(device)
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=device)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    kernel_key = f"collide_advect/{args.workload}/{args.storage}"
    traffic = traffic_entry(kernel_key)
    roofline = {"bound": "hbm", "achieved": round(main["GBps"], 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(main["frac"], 4), "traffic": traffic,
                "bytes_per_update": main["bytes_per_update"], "kernel": "k_collide_advect",
                "copy_kernel_GBps": round(copy_gbps, 1)}
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
        "adjoint": adjoint,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
