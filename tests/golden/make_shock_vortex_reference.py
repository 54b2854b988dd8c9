"""Write the oracle's reference for the full-size shock-vortex parity test.

Runs the float64 CPU oracle on the 2048 x 1024 shock-vortex workload (Ma_s
1.2, Ma_v 0.25, vortex radius 0.075, split II, CFL 0.01, x zero-gradient, y
periodic; the seeded generator of the workload) at one (Pr, gamma) pair for
100 steps and stores the time step it used, the 128 x 64 grid of 16 x 16
block averages of rho and T, and rho and T at 256 seeded cells (the x edges
included).  Calls only the oracle and the input generator (about 35 minutes
on 8 host threads per pair):
    python tests/golden/make_shock_vortex_reference.py            # Pr 0.71, gamma 1.4
    python tests/golden/make_shock_vortex_reference.py 2.0 5/3    # Pr 2, gamma 5/3
The output is shock_vortex_2048x1024_oracle_100.npz for the first pair and
shock_vortex_2048x1024_Pr2_gamma5-3_oracle_100.npz for the second.
"""

import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

from oracle import dvbm_oracle as O  # noqa: E402
from synth import shock_vortex  # noqa: E402

NX, NY, STEPS, SAMPLES = 2048, 1024, 100, 256
HERE = os.path.dirname(os.path.abspath(__file__))
PAIRS = {(0.71, "1.4"): "shock_vortex_2048x1024_oracle_100.npz",
         (2.0, "5/3"): "shock_vortex_2048x1024_Pr2_gamma5-3_oracle_100.npz"}


def main():
    Pr = float(sys.argv[1]) if len(sys.argv) > 1 else 0.71
    gs = sys.argv[2] if len(sys.argv) > 2 else "1.4"
    gamma = 5.0 / 3.0 if gs == "5/3" else float(gs)
    out = os.path.join(HERE, PAIRS[(Pr, gs)])
    wl = shock_vortex(NX, NY, mach_s=1.2, mach_v=0.25, r_frac=0.075, gamma=gamma)
    cfg = O.Config(nx=NX, ny=NY, split=2, dx=wl.dx, dy=wl.dy, Pr=Pr, gamma=gamma, tau_ref=wl.phys["mu"], cfl=0.01,
                   bc_x=O.ZERO_GRADIENT, bc_y=O.PERIODIC)
    dt = O.time_step(torch.as_tensor(wl.rho), torch.as_tensor(np.stack([wl.ux, wl.uy], -1)),
                     torch.as_tensor(wl.T), cfg)
    f, g = O.initial_state(wl.rho, wl.ux, wl.uy, wl.T, cfg)
    t0 = time.time()
    for k in range(STEPS):
        f, g = O.step(f, g, cfg, dt)
        if (k + 1) % 10 == 0:
            print(f"step {k + 1}/{STEPS}, {time.time() - t0:.0f} s", flush=True)
    d = O.diagnostics(f, g, cfg)
    rng = np.random.default_rng(12)
    ys = np.concatenate([rng.integers(0, NY, SAMPLES - 4), [0, NY - 1, 0, NY - 1]])
    xs = np.concatenate([rng.integers(0, NX, SAMPLES - 4), [0, 0, NX - 1, NX - 1]])
    pool = torch.nn.functional.avg_pool2d
    np.savez_compressed(
        out, dt=np.float64(dt), steps=np.int64(STEPS), ys=ys, xs=xs,
        rho_blocks=pool(d["rho"][None, None], 16)[0, 0].numpy(), T_blocks=pool(d["T"][None, None], 16)[0, 0].numpy(),
        rho_samples=d["rho"].numpy()[ys, xs], T_samples=d["T"].numpy()[ys, xs])
    print("wrote", out)


if __name__ == "__main__":
    main()
