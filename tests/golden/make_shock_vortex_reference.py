"""Write the oracle's reference for the full-size shock-vortex parity test.

Runs the float64 CPU oracle on the 2048 x 1024 shock-vortex workload (Ma_s
1.2, Ma_v 0.25, vortex radius 0.075, split II, Pr 0.71, gamma 1.4, CFL 0.01,
x zero-gradient, y periodic; the seeded generator of the workload) for 100
steps and stores, in shock_vortex_2048x1024_oracle_100.npz: the time step it
used, the 128 x 64 grid of 16 x 16 block averages of rho and T, and rho and T
at 256 seeded cells (the x edges included).  Calls only the oracle and the
input generator (about 40 minutes on 8 host threads):
    python tests/golden/make_shock_vortex_reference.py
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
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "shock_vortex_2048x1024_oracle_100.npz")


def main():
    wl = shock_vortex(NX, NY, mach_s=1.2, mach_v=0.25, r_frac=0.075, gamma=1.4)
    cfg = O.Config(nx=NX, ny=NY, split=2, dx=wl.dx, dy=wl.dy, Pr=0.71, gamma=1.4, tau_ref=wl.phys["mu"], cfl=0.01,
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
        OUT, dt=np.float64(dt), steps=np.int64(STEPS), ys=ys, xs=xs,
        rho_blocks=pool(d["rho"][None, None], 16)[0, 0].numpy(), T_blocks=pool(d["T"][None, None], 16)[0, 0].numpy(),
        rho_samples=d["rho"].numpy()[ys, xs], T_samples=d["T"].numpy()[ys, xs])
    print("wrote", OUT)


if __name__ == "__main__":
    main()
