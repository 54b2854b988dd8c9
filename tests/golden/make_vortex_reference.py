"""Write the oracle's reference for the full-size vortex parity test.

Runs the float64 CPU oracle on the 1024 x 1024 Mach-1 isentropic vortex
(split II, Pr 0.71, gamma 1.4, mu 5e-5, CFL 0.01, periodic; the seeded
generator of the precision workload) for 300 steps and stores, in
vortex_1024_oracle_300.npz: the time step it used, the 128 x 128 grid of
8 x 8 block averages of rho and T, and rho and T at 256 seeded cells.
Calls only the oracle and the input generator (about an hour on 8 host
threads):  python tests/golden/make_vortex_reference.py
"""

import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

from oracle import dvbm_oracle as O  # noqa: E402
from synth import isentropic_vortex  # noqa: E402

N, STEPS, SAMPLES = 1024, 300, 256
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "vortex_1024_oracle_300.npz")


def main():
    wl = isentropic_vortex(N, seed=0, mach_adv=1.0, mach_v=0.3, r_frac=0.05)
    cfg = O.Config(nx=N, ny=N, split=2, dx=wl.dx, dy=wl.dy, Pr=0.71, gamma=1.4, tau_ref=5e-5, cfl=0.01)
    dt = O.time_step(torch.as_tensor(wl.rho), torch.as_tensor(np.stack([wl.ux, wl.uy], -1)),
                     torch.as_tensor(wl.T), cfg)
    f, g = O.initial_state(wl.rho, wl.ux, wl.uy, wl.T, cfg)
    t0 = time.time()
    for k in range(STEPS):
        f, g = O.step(f, g, cfg, dt)
        if (k + 1) % 10 == 0:
            print(f"step {k + 1}/{STEPS}, {time.time() - t0:.0f} s", flush=True)
    d = O.diagnostics(f, g, cfg)
    rng = np.random.default_rng(11)
    ys, xs = rng.integers(0, N, SAMPLES), rng.integers(0, N, SAMPLES)
    pool = torch.nn.functional.avg_pool2d
    np.savez_compressed(
        OUT, dt=np.float64(dt), steps=np.int64(STEPS), ys=ys, xs=xs,
        rho_128=pool(d["rho"][None, None], 8)[0, 0].numpy(), T_128=pool(d["T"][None, None], 8)[0, 0].numpy(),
        rho_samples=d["rho"].numpy()[ys, xs], T_samples=d["T"].numpy()[ys, xs])
    print("wrote", OUT)


if __name__ == "__main__":
    main()
