"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances (relative L2 over all populations of both distributions):
* float64 storage: 1e-12 for the state and, to make the comparison sensitive
  to the update itself, 1e-9 on the increment X(t+n dt) - X(t);
* float32 storage (float32 arithmetic, float64 moment sums): 1e-5;
* 16-bit deviation storage: the final rounding of (X - X_ref)/w dominates,
  so the bound is the format's unit roundoff (2^-8 bfloat16, 2^-11 half)
  times the norm of the deviation, plus float32 arithmetic.
"""

import ctypes
import math
import os

import numpy as np
import pytest
import torch

from oracle import dvbm_oracle as O
from paper_2510_04197_amd import DVBMError, Solver, dvbm, make_params
from closed_forms import sound_decay_rate
from synth import isentropic_vortex, shear_wave, shock_vortex, smooth_random, sod_tube, thermal_wave, uniform

pytestmark = pytest.mark.gpu
DEV = "cuda"


def oracle_cfg(p) -> O.Config:
    inv_bc = {0: O.PERIODIC, 1: O.ZERO_GRADIENT, 2: O.WALL}
    return O.Config(nx=p.nx, ny=p.ny, split=p.split, bc_x=inv_bc[p.bc_x], bc_y=inv_bc[p.bc_y],
                    visc_mode=O.CONST_MU if p.visc_mode == 0 else O.CONST_TAU, dx=p.dx, dy=p.dy, R=p.R,
                    gamma=p.gamma, Pr=p.Pr, tau_ref=p.tau_ref, p_ref=p.p_ref, T_ref=p.T_ref, beta=p.beta,
                    cfl=p.cfl, dt=p.dt, wall_T=(p.wall_T[0], p.wall_T[1]), wall_ux=(p.wall_ux[0], p.wall_ux[1]))


def solver(wl, **kw):
    p = make_params(wl.nx, wl.ny, dx=wl.dx, dy=wl.dy, **kw)
    return Solver(p, wl.rho, wl.ux, wl.uy, wl.T, device=DEV), p


def rel(a, b):
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def oracle_state(s: Solver):
    X = s.store_populations().cpu()
    return X[0], X[1]


# ---------------------------------------------------------------- initial state
@pytest.mark.parametrize("split", (1, 2))
@pytest.mark.parametrize("storage,tol", (("f64", 1e-14), ("f32", 1e-7)))
def test_initial_equilibrium(split, storage, tol):
    wl = smooth_random(70, 37, seed=1)
    s, p = solver(wl, split=split, storage=storage, tau_ref=0.02)
    f, g = oracle_state(s)
    fo, go = O.initial_state(wl.rho, wl.ux, wl.uy, wl.T, oracle_cfg(p))
    assert rel(f, fo) < tol and rel(g, go) < tol


# ---------------------------------------------------------------- time step (Sec. III A 3)
def _dt_case(case):
    """Initial fields and parameters of the time-step cases: smooth random
    fields, the Mach-1 vortex, a shock-vortex field with zero-gradient x, the
    Sod tube and a flow between no-slip walls."""
    if case == "smooth":
        return smooth_random(70, 37, seed=21), dict(split=2, tau_ref=0.02, cfl=0.1)
    if case == "vortex":
        return isentropic_vortex(128, seed=3), dict(split=2, tau_ref=0.02)
    if case == "shock":
        wl = shock_vortex(256, 128, mach_s=1.2, mach_v=0.25, r_frac=0.075, gamma=5.0 / 3.0)
        return wl, dict(split=2, gamma=5.0 / 3.0, bc_x="zero_gradient", tau_ref=0.02, Pr=2.0)
    if case == "sod":
        return sod_tube(128, 4), dict(split=1, tau_ref=0.02, cfl=0.2, Pr=0.5)
    wl = smooth_random(33, 20, seed=22, amp_u=0.3)
    return wl, dict(split=1, bc_y="wall", wall_T=(0.9, 1.2), wall_ux=(0.0, 0.5), tau_ref=0.02, cfl=0.05, R=1.7,
                    T_ref=1.3)


@pytest.mark.parametrize("storage", ("f64", "f32"))
@pytest.mark.parametrize("case", ("smooth", "vortex", "shock", "sod", "wall"))
def test_time_step_matches_oracle(case, storage):
    """dvbm_init's time step (reduction of |u| + sqrt(gamma R T) over the
    initial fields) equals the oracle's CFL rule to 1e-15 relative."""
    wl, kw = _dt_case(case)
    s, p = solver(wl, storage=storage, **kw)
    dt_o = O.time_step(wl.rho, np.stack([wl.ux, wl.uy], -1), wl.T, oracle_cfg(p))
    assert abs(s.dt - dt_o) <= 1e-15 * dt_o, (s.dt, dt_o)
    s.close()


def test_time_step_override():
    """A given dt > 0 replaces the CFL rule on both sides, bit for bit."""
    wl, kw = _dt_case("smooth")
    s, p = solver(wl, storage="f64", dt=3.25e-5, **kw)
    assert s.dt == 3.25e-5 == O.time_step(wl.rho, np.stack([wl.ux, wl.uy], -1), wl.T, oracle_cfg(p))
    s.close()


@pytest.mark.parametrize("rule", ("dt", "cfl"))
@pytest.mark.parametrize("Pr", (0.5, 1.0, 2.0))
@pytest.mark.parametrize("visc_mode", ("const_mu", "const_tau"))
def test_stiffness_threshold(visc_mode, Pr, rule):
    """dvbm_init rejects a step with dt / tau_1 > 2 on the initial fields
    (ESTIFF) and accepts one just below: 1e-9 either side of the oracle's
    threshold, with the step given (rule 'dt') or from the CFL rule with
    tau_ref moved across the threshold (rule 'cfl')."""
    wl = smooth_random(16, 12, seed=23, amp_rho=0.2, amp_T=0.2)
    base = dict(split=2, storage="f64", visc_mode=visc_mode, Pr=Pr, cfl=0.1, p_ref=1.3, R=1.2)
    cfg = oracle_cfg(make_params(wl.nx, wl.ny, dx=wl.dx, dy=wl.dy, tau_ref=1e-3, **base))
    if rule == "dt":
        dt_c = 2.0 / O.max_relaxation_rate(wl.rho, wl.T, cfg, 1.0)
        cases = [(dict(tau_ref=1e-3, dt=dt_c * (1 - 1e-9)), True), (dict(tau_ref=1e-3, dt=dt_c * (1 + 1e-9)), False)]
    else:
        dt = O.time_step(wl.rho, np.stack([wl.ux, wl.uy], -1), wl.T, cfg)
        tau_c = 1e-3 * O.max_relaxation_rate(wl.rho, wl.T, cfg, dt) / 2.0
        cases = [(dict(tau_ref=tau_c * (1 + 1e-9)), True), (dict(tau_ref=tau_c * (1 - 1e-9)), False)]
    for extra, ok in cases:
        p = make_params(wl.nx, wl.ny, dx=wl.dx, dy=wl.dy, **base, **extra)
        c = oracle_cfg(p)
        rate = O.max_relaxation_rate(wl.rho, wl.T, c, O.time_step(wl.rho, np.stack([wl.ux, wl.uy], -1), wl.T, c))
        assert (rate <= 2.0) == ok, (rate, extra)
        if ok:
            Solver(p, wl.rho, wl.ux, wl.uy, wl.T, device=DEV).close()
        else:
            with pytest.raises(DVBMError) as e:
                Solver(p, wl.rho, wl.ux, wl.uy, wl.T, device=DEV)
            assert e.value.code == dvbm.DVBM_ESTIFF


# ---------------------------------------------------------------- multi-step parity, small grids
CASES = [(split, Pr, bc) for split in (1, 2) for Pr in (0.5, 1.0, 2.0) for bc in ("periodic", "zero_gradient")]


@pytest.mark.parametrize("kernel", ("tile", "cell", "sweep"))
@pytest.mark.parametrize("split,Pr,bc", CASES)
def test_steps_fp64(split, Pr, bc, kernel):
    wl = smooth_random(70, 37, seed=2)  # two 64-wide tiles in x with a ragged tail, ragged rows in y
    s, p = solver(wl, split=split, storage="f64", Pr=Pr, tau_ref=0.02, bc_x=bc, cfl=0.1, kernel=kernel)
    cfg = oracle_cfg(p)
    f0, g0 = O.initial_state(wl.rho, wl.ux, wl.uy, wl.T, cfg)
    s.step(8)
    f, g = oracle_state(s)
    fo, go = O.run(f0, g0, cfg, s.dt, 8)
    assert rel(f, fo) < 1e-12 and rel(g, go) < 1e-12
    assert rel(f - f0, fo - f0) < 1e-9 and rel(g - g0, go - g0) < 1e-9


@pytest.mark.parametrize("storage", ("f32", "f32_dev"))
@pytest.mark.parametrize("kernel", ("cell", "sweep", "tile"))
@pytest.mark.parametrize("split,Pr,bc", CASES)
def test_steps_fp32(split, Pr, bc, kernel, storage):
    wl = smooth_random(70, 37, seed=3)  # sweep: two 60-column strips, the second ragged; 37 rows in ranges of 3 m
    s, p = solver(wl, split=split, storage=storage, Pr=Pr, tau_ref=0.02, bc_x=bc, bc_y=bc, cfl=0.1, kernel=kernel)
    cfg = oracle_cfg(p)
    f0, g0 = O.initial_state(wl.rho, wl.ux, wl.uy, wl.T, cfg)
    s.step(8)
    f, g = oracle_state(s)
    fo, go = O.run(f0, g0, cfg, s.dt, 8)
    assert rel(f, fo) < 1e-5 and rel(g, go) < 1e-5


@pytest.mark.parametrize("mode", ("const_mu", "const_tau"))
def test_off_equilibrium_single_step_fp64(mode):
    """One step from a perturbed (non-equilibrium) state loaded through the ABI."""
    wl = smooth_random(67, 9, seed=4)
    s, p = solver(wl, split=2, storage="f64", Pr=0.6, tau_ref=0.02, visc_mode=mode, R=1.1, T_ref=0.9,
                  gamma=1.3, dt=2e-4)
    cfg = oracle_cfg(p)
    f0, g0 = O.initial_state(wl.rho, wl.ux, wl.uy, wl.T, cfg)
    rng = np.random.default_rng(0)
    f0 = f0 * (1 + 0.01 * torch.tensor(rng.standard_normal(f0.shape)))
    g0 = g0 * (1 + 0.01 * torch.tensor(rng.standard_normal(g0.shape)))
    s.load_populations(torch.stack([f0, g0]))
    s.step(1)
    f, g = oracle_state(s)
    fo, go = O.step(f0, g0, cfg, 2e-4)
    assert rel(f - f0, fo - f0) < 1e-10 and rel(g - g0, go - g0) < 1e-10


def test_minimal_grid():
    wl = smooth_random(4, 4, seed=5)
    s, p = solver(wl, split=2, storage="f64", tau_ref=0.02, cfl=0.1)
    cfg = oracle_cfg(p)
    f0, g0 = O.initial_state(wl.rho, wl.ux, wl.uy, wl.T, cfg)
    s.step(3)
    f, g = oracle_state(s)
    fo, go = O.run(f0, g0, cfg, s.dt, 3)
    assert rel(f, fo) < 1e-12 and rel(g, go) < 1e-12


# ---------------------------------------------------------------- the 64^2 shear-wave workload, 1000 steps
def test_shear_wave_64_fp64_1000_steps():
    """64^2 periodic shear wave (u_y = 1e-3 sin, Ma = 0.1), 1000 FP64 steps.

    On L = 1 with dx = 1/64 the paper's mu = 5e-5 gives dt/tau = 2.4 at
    CFL 0.01 (beyond the explicit Euler relaxation limit), so the workload
    uses mu = 2e-3, well above the scheme's numerical viscosity at 64 cells.
    The shear mode decays at nu k^2 with nu = mu - U^2 dt / 2 (shear
    viscosity less forward Euler's term, as on the moving background of
    test_shear_viscosity_on_a_flow): measured 0.57 % below it over the
    run's 0.94 % decay, the initial relaxation from equilibrium included.
    """
    wl = shear_wave(64, amp=1e-3, mach=0.1)
    s, p = solver(wl, split=2, storage="f64", Pr=0.71, tau_ref=2e-3)
    cfg = oracle_cfg(p)
    f0, g0 = O.initial_state(wl.rho, wl.ux, wl.uy, wl.T, cfg)
    sums0 = s.moments(fields=False)["sums"]
    e = torch.tensor(np.exp(-2j * np.pi * (np.arange(64) + 0.5) / 64), device=DEV)

    def mode():
        return float(torch.abs(2 * (s.moments(fields=True, sums=False)["uy"].mean(dim=0) * e).mean()))

    a0 = mode()
    s.step(1000)
    U = 0.1 * math.sqrt(1.4)
    nu = math.log(a0 / mode()) / ((2 * math.pi) ** 2 * 1000 * s.dt)
    print(f"[shear 64] nu / (mu - U^2 dt / 2) - 1 = {nu / (2e-3 - 0.5 * U * U * s.dt) - 1:.2e}", flush=True)
    assert abs(nu / (2e-3 - 0.5 * U * U * s.dt) - 1) < 1.5e-2
    f, g = oracle_state(s)
    fo, go = O.run(f0, g0, cfg, s.dt, 1000)
    assert rel(f, fo) < 1e-12 and rel(g, go) < 1e-12
    assert rel(f - f0, fo - f0) < 1e-8
    sums = s.moments(fields=False)["sums"]
    drift = np.abs(sums - sums0) / np.maximum(np.abs(sums0), 1.0)
    assert drift.max() < 1e-12


# ---------------------------------------------------------------- diagnostics and conservation
def test_moment_fields_match_oracle():
    wl = smooth_random(70, 37, seed=6)
    s, p = solver(wl, split=2, storage="f64", tau_ref=0.02, cfl=0.1)
    s.step(5)
    m = s.moments()
    f, g = oracle_state(s)
    d = O.diagnostics(f, g, oracle_cfg(p))
    for k in ("rho", "ux", "uy", "T"):
        assert rel(m[k].cpu(), d[k]) < 1e-14, k
    np.testing.assert_allclose(m["sums"], d["sums"].numpy(), rtol=1e-13)


@pytest.mark.parametrize("split", (1, 2))
@pytest.mark.parametrize("Pr", (0.5, 2.0))
def test_periodic_conservation_fp64(split, Pr):
    wl = smooth_random(96, 80, seed=7)
    s, _ = solver(wl, split=split, storage="f64", Pr=Pr, tau_ref=0.02, cfl=0.1)
    s0 = s.moments(fields=False)["sums"]
    s.step(200)
    s1 = s.moments(fields=False)["sums"]
    drift = np.abs(s1 - s0) / np.abs(s0)
    assert drift.max() < 1e-16 * 96 * 80 * 200 / 100, drift


@pytest.mark.parametrize("kernel", ("auto", "cell", "sweep", "tile"))
def test_uniform_state_fixed_point_all_storages(kernel):
    wl = uniform(70, 12, rho=1.1, ux=0.3, uy=-0.1, T=1.05)
    for storage in ("f64", "f32", "f32_dev", "bf16_dev", "fp16_dev"):
        s, _ = solver(wl, split=2, storage=storage, tau_ref=0.02, cfl=0.1, kernel=kernel)
        X0 = s.store_populations()
        s.step(10)
        X1 = s.store_populations()
        # 16-bit formats: the stored equilibrium is itself rounded, so relaxation may
        # move it by at most the rounding of the deviation (~0.3 * 2^-8 or 2^-11)
        tol = {"f64": 1e-15, "f32": 1e-6, "f32_dev": 1e-6, "bf16_dev": 3e-3, "fp16_dev": 4e-4}[storage]
        assert rel(X1, X0) < tol, storage


# ---------------------------------------------------------------- column-sweep geometry
@pytest.mark.parametrize("nx,ny", ((4, 4), (59, 5), (60, 7), (61, 40), (241, 13), (250, 9), (480, 6)))
@pytest.mark.parametrize("bc", ("periodic", "zero_gradient"))
@pytest.mark.parametrize("storage", ("f32", "f64", "f32_dev"))
def test_sweep_strips_and_row_ranges(nx, ny, bc, storage):
    """Strips of 60 columns in groups of 4 (float32) or 2 (float64), with empty strips at the end of the last
    group, row ranges of 3 m rows with the last one overlapping its predecessor, grids narrower than a strip."""
    wl = smooth_random(nx, ny, seed=31, amp_T=0.05)
    s, p = solver(wl, split=2, storage=storage, Pr=0.6, tau_ref=0.02, bc_x=bc, bc_y=bc, cfl=0.1, kernel="sweep")
    cfg = oracle_cfg(p)
    f0, g0 = O.initial_state(wl.rho, wl.ux, wl.uy, wl.T, cfg)
    s.step(4)
    f, g = oracle_state(s)
    fo, go = O.run(f0, g0, cfg, s.dt, 4)
    tol, tol_inc = (1e-12, 1e-9) if storage == "f64" else (1e-5, 1e-3)
    assert rel(f, fo) < tol and rel(g, go) < tol
    assert rel(f - f0, fo - f0) < tol_inc and rel(g - g0, go - g0) < tol_inc


# ---------------------------------------------------------------- 16-bit deviation storage
@pytest.mark.parametrize("kernel", ("cell", "sweep", "tile"))
@pytest.mark.parametrize("split", (1, 2))
@pytest.mark.parametrize("storage,u", (("bf16_dev", 2.0 ** -8), ("fp16_dev", 2.0 ** -11)))
def test_deviation_storage_step(split, storage, u, kernel):
    wl = smooth_random(70, 20, seed=8, amp_T=0.05)
    s, p = solver(wl, split=split, storage=storage, Pr=0.7, tau_ref=0.02, cfl=0.1, kernel=kernel)
    cfg = oracle_cfg(p)
    f0, g0 = oracle_state(s)  # decoded (already rounded) initial state
    fo_ic, go_ic = O.initial_state(wl.rho, wl.ux, wl.uy, wl.T, cfg)
    v, w = O.velocity_set(cfg)
    wq = w.reshape(-1, 1, 1)
    fref = wq * torch.ones_like(fo_ic)
    s_g = s.store_populations().cpu()[1]
    # rounding of the stored deviation bounds the initial error
    assert float(((f0 - fo_ic).abs() / wq).max()) <= u * float(((fo_ic - fref).abs() / wq).max()) * 1.01 + 1e-7
    s.step(1)
    f1, g1 = oracle_state(s)
    fo, go = O.step(f0, g0, cfg, s.dt)
    dev_f = torch.linalg.vector_norm((fo - fref))
    assert float(torch.linalg.vector_norm(f1 - fo)) <= 1.5 * u * float(dev_f) + 1e-6 * float(torch.linalg.vector_norm(fo))
    assert torch.isfinite(s_g).all()


def test_load_store_roundtrip():
    wl = smooth_random(66, 10, seed=9)
    for storage in ("f64", "f32", "f32_dev"):
        s, p = solver(wl, split=2, storage=storage, tau_ref=0.02)
        X = s.store_populations()
        Y = X * (1 + 1e-3 * torch.sin(torch.arange(X.numel(), device=DEV, dtype=torch.float64)).reshape(X.shape))
        s.load_populations(Y)
        Z = s.store_populations()
        assert rel(Z, Y) < (1e-16 if storage == "f64" else 1e-7)


# ---------------------------------------------------------------- full-size workloads, sampled cells
def sampled_check(s: Solver, p, nsamples=96, seed=0):
    """Run one GPU step and compare sampled cells with the oracle's update of the same state."""
    cfg = oracle_cfg(p)
    rng = np.random.default_rng(seed)
    ys = torch.tensor(np.concatenate([rng.integers(0, p.ny, nsamples - 4), [0, p.ny - 1, 0, p.ny - 1]]))
    xs = torch.tensor(np.concatenate([rng.integers(0, p.nx, nsamples - 4), [0, p.nx - 1, p.nx - 1, 0]]))
    yi, xi = O.window_indices(cfg, ys, xs)
    X = s.store_populations()
    win = X[:, :, yi.to(DEV)[:, :, None], xi.to(DEV)[:, None, :]].cpu()  # [2, Q, S, 5, 5]
    del X
    s.step(1)
    X1 = s.store_populations()
    got = X1[:, :, ys.to(DEV), xs.to(DEV)].cpu()
    del X1
    fo, go = O.window_step(win[0], win[1], cfg, s.dt)
    return got, torch.stack([fo, go]), win[:, :, :, 2, 2]


# One float32 step from a stored state: the oracle updates the same (float32)
# state in float64, so the GPU's result differs by the float32 rounding of one
# update only.  A step moves these states by about 1e-6 relative, so the state
# tolerance of 1e-5 alone could not see an error in the float32 update; the
# bound of 16 float32 ulps (2^-24 relative) can.
F32_STEP = 16 * 2.0 ** -24


def check_sampled(got, ref, before, storage, tol, what):
    e = rel(got, ref)
    print(f"[{what}] {storage}: relative L2 against the oracle {e:.2e}, increment {rel(got - before, ref - before):.2e}",
          flush=True)
    assert e < tol
    if storage == "f64":
        assert rel(got - before, ref - before) < 1e-9
    else:
        assert e < F32_STEP


@pytest.mark.parametrize("storage,tol", (("f32", 1e-5), ("f64", 1e-12), ("f32_dev", 1e-5)))
def test_vortex_1024_sampled(storage, tol):
    wl = isentropic_vortex(1024, seed=0, mach_adv=1.0, mach_v=0.3, r_frac=0.05)
    s, p = solver(wl, split=2, storage=storage, Pr=0.71, tau_ref=5e-5)
    s.step(2)
    got, ref, before = sampled_check(s, p)
    check_sampled(got, ref, before, storage, tol, "vortex 1024")


def test_vortex_1024_300_steps_against_the_oracle():
    """The 1024^2 Mach-1 vortex workload over 300 steps against the oracle's
    own run of the same steps at full size (tests/golden/vortex_1024_oracle_300.npz,
    written by tests/golden/make_vortex_reference.py from the oracle alone,
    with the time step it used): rho and T on the 128^2 grid of 8 x 8 block
    averages and at 256 sampled cells.  This ties the long runs, which compare
    float32 storage with the float64-storage GPU run, to the oracle at the
    workload's size: float64 storage within 1e-12 (measured 0.8e-15 to
    1.3e-15), FP32 and FP32-dev within 2e-6 (measured 3.1e-7 to 6.4e-7 and
    1.9e-7 to 3.4e-7)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "vortex_1024_oracle_300.npz")
    ref = np.load(path)
    ys, xs = torch.tensor(ref["ys"]), torch.tensor(ref["xs"])
    wl = isentropic_vortex(1024, seed=0, mach_adv=1.0, mach_v=0.3, r_frac=0.05)
    pool = torch.nn.functional.avg_pool2d
    for storage, tol in (("f64", 1e-12), ("f32", 2e-6), ("f32_dev", 2e-6)):
        s, _ = solver(wl, split=2, storage=storage, Pr=0.71, gamma=1.4, tau_ref=5e-5, dt=float(ref["dt"]))
        s.step(int(ref["steps"]))
        m = s.moments(fields=True, sums=False)
        s.close()
        errs = {}
        for k in ("rho", "T"):
            f = m[k]
            errs[k + "_128"] = rel(pool(f[None, None], 8)[0, 0].cpu(), torch.tensor(ref[k + "_128"]))
            errs[k + "_samples"] = rel(f[ys.to(f.device), xs.to(f.device)].cpu(), torch.tensor(ref[k + "_samples"]))
        print(f"[vortex 1024, 300 steps, oracle] {storage}: " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()),
              flush=True)
        assert max(errs.values()) < tol, (storage, errs)


@pytest.mark.parametrize("Pr,gamma,name", (
    (0.71, 1.4, "shock_vortex_2048x1024_oracle_100.npz"),
    (2.0, 5.0 / 3.0, "shock_vortex_2048x1024_Pr2_gamma5-3_oracle_100.npz")), ids=("Pr0.71-g1.4", "Pr2-g5/3"))
def test_shock_vortex_2048x1024_100_steps_against_the_oracle(Pr, gamma, name):
    """The 2048 x 1024 shock-vortex workload (x zero-gradient, y periodic) at
    two (Pr, gamma) pairs, one for each side of Table I (Pr < 1 and Pr > 1),
    over 100 steps against the oracle's own full-size run of the same steps
    (tests/golden/*.npz, written by tests/golden/make_shock_vortex_reference.py
    from the oracle alone, with the time step it used): rho and T on the
    128 x 64 grid of 16 x 16 block averages and at 256 sampled cells, the x
    edges included.  Float64 storage within 1e-12, FP32 and FP32-dev within
    2e-6 (measured at Pr 0.71, gamma 1.4: 2.4e-16 to 5.5e-16, 1.3e-7 to
    2.4e-7 and 3.3e-7 to 7.6e-7; at Pr 2, gamma 5/3: 1.7e-16 to 4.7e-16,
    5.0e-8 to 1.1e-7 and 1.1e-7 to 2.8e-7; at Mach 1.2 the deviations from
    the rest state are as large as the values, so FP32-dev does not gain)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    ref = np.load(path)
    ys, xs = torch.tensor(ref["ys"]), torch.tensor(ref["xs"])
    wl = shock_vortex(2048, 1024, mach_s=1.2, mach_v=0.25, r_frac=0.075, gamma=gamma)
    pool = torch.nn.functional.avg_pool2d
    for storage, tol in (("f64", 1e-12), ("f32", 2e-6), ("f32_dev", 2e-6)):
        s, _ = solver(wl, split=2, storage=storage, Pr=Pr, gamma=gamma, tau_ref=wl.phys["mu"], bc_x="zero_gradient",
                      bc_y="periodic", dt=float(ref["dt"]))
        s.step(int(ref["steps"]))
        m = s.moments(fields=True, sums=False)
        s.close()
        errs = {}
        for k in ("rho", "T"):
            f = m[k]
            errs[k + "_blocks"] = rel(pool(f[None, None], 16)[0, 0].cpu(), torch.tensor(ref[k + "_blocks"]))
            errs[k + "_samples"] = rel(f[ys.to(f.device), xs.to(f.device)].cpu(), torch.tensor(ref[k + "_samples"]))
        print(f"[shock-vortex 2048x1024, Pr {Pr}, gamma {gamma:.3f}, 100 steps, oracle] {storage}: "
              + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()), flush=True)
        assert max(errs.values()) < tol, (storage, errs)


@pytest.mark.parametrize("storage", ("f32", "f32_dev"))
@pytest.mark.parametrize("Pr,gamma", [(Pr, g) for Pr in (0.1, 0.71, 2.0) for g in (1.4, 5.0 / 3.0)])
def test_shock_vortex_2048x1024_sampled(Pr, gamma, storage):
    """The six (Pr, gamma) pairs of the 2048 x 1024 shock-vortex workload, x
    zero-gradient, y periodic: sampled cells of a step against the oracle."""
    wl = shock_vortex(2048, 1024, mach_s=1.2, mach_v=0.25, r_frac=0.075, gamma=gamma)
    s, p = solver(wl, split=2, storage=storage, Pr=Pr, gamma=gamma, tau_ref=wl.phys["mu"], bc_x="zero_gradient",
                  bc_y="periodic")
    s.step(2)
    got, ref, before = sampled_check(s, p)
    check_sampled(got, ref, before, storage, 1e-5, f"shock-vortex Pr {Pr} gamma {gamma:.3f}")


@pytest.mark.parametrize("storage,tol", (("f32", 1e-5), ("f64", 1e-12), ("f32_dev", 1e-5)))
def test_thermal_wave_4096_sampled(storage, tol):
    wl = thermal_wave(4096, seed=0)
    s, p = solver(wl, split=2, storage=storage, Pr=0.5, tau_ref=5e-5)
    s.step(1)
    got, ref, before = sampled_check(s, p, nsamples=64)
    check_sampled(got, ref, before, storage, tol, "thermal wave 4096")


@pytest.mark.parametrize("storage,u", (("bf16_dev", 2.0 ** -8), ("fp16_dev", 2.0 ** -11)))
def test_thermal_wave_4096_sampled_16bit(storage, u):
    """The 4096^2 thermal wave in the 16-bit deviation formats: one step on
    64 sampled cells against the oracle's update of the same (decoded) state.
    The stored value is the format's rounding of the deviation from the rest
    equilibrium, so the difference is bounded by 1.5 units of the format
    times the deviation's size (as on the small grids); measured 0.016 units
    (BF16) and 0.020 (FP16): a step moves most stored deviations by less
    than their rounding unit."""
    wl = thermal_wave(4096, seed=0)
    s, p = solver(wl, split=2, storage=storage, Pr=0.5, tau_ref=5e-5)
    s.step(1)
    got, ref, before = sampled_check(s, p, nsamples=64)
    cfg = oracle_cfg(p)
    fr, gr = O.initial_state(np.ones((1, 1)), np.zeros((1, 1)), np.zeros((1, 1)), np.full((1, 1), p.T_ref), cfg)
    xref = torch.stack([fr[:, 0, 0], gr[:, 0, 0]])[:, :, None]  # rest equilibrium per plane, [2, Q, 1]
    e = float(torch.linalg.vector_norm(got - ref))
    dev = float(torch.linalg.vector_norm(ref - xref))
    print(f"[thermal wave 4096] {storage}: |got - oracle| / |deviation| = {e / dev:.2e} = {e / (u * dev):.3f} u",
          flush=True)
    assert e <= 1.5 * u * dev


def test_largest_grids_sampled():
    """6528 x 6528, split II.  In float32 one distribution takes 3.97 GiB: the
    32-bit buffer offsets are near their 4 GiB limit, and the grid is above the
    column-sweep kernel's 2 GiB, so AUTO takes the per-cell kernel.  In bfloat16
    it takes 1.98 GiB, just below the column-sweep kernel's limit, which AUTO
    then takes."""
    n = 6528
    print(f"[largest grids] {n}x{n}", flush=True)
    wl = smooth_random(n, n, seed=21, amp_T=0.05)
    for storage in ("f32", "bf16_dev"):
        print(f"[largest grids] {storage}", flush=True)
        s, p = solver(wl, split=2, storage=storage, Pr=0.71, tau_ref=5e-5)
        assert s.buffers[0].numel() // 2 == 25 * n * n * (4 if storage == "f32" else 2)
        got, ref, _ = sampled_check(s, p, nsamples=48, seed=5)
        s.close()
        del s
        torch.cuda.empty_cache()
        if storage == "f32":
            assert rel(got, ref) < 1e-5
        else:
            # the rounding of the stored deviation from w_i (f) bounds the error
            w = O.velocity_set(oracle_cfg(p))[1].reshape(-1, 1)
            dev_f = torch.linalg.vector_norm(ref[0] - w)
            assert float(torch.linalg.vector_norm(got[0] - ref[0])) <= 1.5 * 2.0 ** -8 * float(dev_f) + \
                1e-6 * float(torch.linalg.vector_norm(ref[0]))
            assert float(torch.linalg.vector_norm(got[1] - ref[1])) <= 1.5 * 2.0 ** -8 * float(
                torch.linalg.vector_norm(ref[1]))


def test_largest_grid_fp64_sampled():
    """4608 x 4608 in float64: one distribution takes 3.96 GiB, near the 4 GiB
    limit of the 32-bit load offsets; AUTO takes the column sweep, whose stores
    go through one buffer resource per buffer row (the Q planes of one
    distribution at one y)."""
    n = 4608
    print(f"[largest grid fp64] {n}x{n}", flush=True)
    wl = smooth_random(n, n, seed=22, amp_T=0.05)
    s, p = solver(wl, split=2, storage="f64", Pr=0.71, tau_ref=5e-5)
    assert s.buffers[0].numel() // 2 == 25 * n * n * 8
    got, ref, before = sampled_check(s, p, nsamples=48, seed=6)
    assert rel(got, ref) < 1e-12
    assert rel(got - before, ref - before) < 1e-9


# ---------------------------------------------------------------- no-slip walls (thermal Couette flow, Sec. IV)
@pytest.mark.parametrize("split", (1, 2))
@pytest.mark.parametrize("Pr", (0.5, 1.0, 2.0))
@pytest.mark.parametrize("bc_x", ("periodic", "zero_gradient"))
@pytest.mark.parametrize("storage,tol", (("f64", 1e-12), ("f32", 1e-5), ("f32_dev", 1e-5)))
def test_walls_match_oracle(split, Pr, bc_x, storage, tol):
    """Walls in y at temperatures 0.95 and 1.1, the upper one moving at 0.3:
    an off-equilibrium start on 11 x 9 cells (a ragged tile in both
    directions, rows 0, 1 and ny-2, ny-1 next to the walls), 6 steps."""
    wl = smooth_random(11, 9, seed=23, amp_T=0.05)
    s, p = solver(wl, split=split, storage=storage, Pr=Pr, tau_ref=0.02, bc_x=bc_x, bc_y="wall", cfl=0.1,
                  wall_T=(0.95, 1.1), wall_ux=(0.0, 0.3))
    cfg = oracle_cfg(p)
    f0, g0 = oracle_state(s)
    s.step(6)
    f, g = oracle_state(s)
    fo, go = O.run(f0, g0, cfg, s.dt, 6)
    assert rel(f, fo) < tol and rel(g, go) < tol
    if storage == "f64":
        assert rel(f - f0, fo - f0) < 1e-9 and rel(g - g0, go - g0) < 1e-9


@pytest.mark.parametrize("Ma,Ec", ((0.5, 4.0), (1.2, 40.0)))
@pytest.mark.parametrize("split", (2, 1))
@pytest.mark.parametrize("Pr", (0.5, 1.0, 2.0))
def test_thermal_couette_steady_profile(split, Pr, Ma, Ec):
    """Thermal Couette flow at the paper's two parameter sets (Sec. IV:
    Ma = 0.5, Ec = 4 and Ma = 1.2, Ec = 40; Re = 100, T_C = T_ref, linear
    initial profiles), 128 rows as in the paper, CFL 0.2 (the fastest lattice
    velocity, 2.86 sqrt(R T_ref), sets the stable step: CFL 0.5 diverges),
    run for about 8 slowest-mode decay times: the temperature against
    (T - T_C)/(T_H - T_C) = y + Pr Ec/2 y (1 - y), exact for constant mu and
    kappa whatever the density.  Measured at Ma = 0.5: 0.24-0.41 % of the
    profile's peak, split I at Pr = 2 1.9 %; the error does not fall below
    ~0.4 % with resolution (split II, Pr = 1: 32 rows 1.1 %, 64 rows 0.36 %,
    256 rows 0.40 %); split I converges more slowly (Pr = 1: 64 rows 0.97 %,
    128 rows 0.37 %).  At Ma = 1.2, Ec = 40, where viscous heating makes the
    profile ten times the wall difference: 1.0-3.5 %, first order in the row
    spacing and independent of the time step (split II, Pr = 1: 64 / 128 /
    256 rows 5.5 / 2.6 / 1.1 %, the same at CFL 0.1; the wall velocity's slip
    halves likewise, 0.85 / 0.43 / 0.21 % of u_0)."""
    import math
    ny, nx, Re, gamma = 128, 4, 100.0, 1.4
    u0 = Ma * math.sqrt(gamma)
    TC, TH = 1.0, 1.0 + u0 * u0 / (gamma / (gamma - 1) * Ec)
    y = (np.arange(ny) + 0.5) / ny
    Y = np.repeat(y[:, None], nx, 1)
    p = make_params(nx, ny, dx=1.0 / ny, dy=1.0 / ny, split=split, storage="f64", Pr=Pr, gamma=gamma, tau_ref=u0 / Re,
                    cfl=0.2, bc_y="wall", wall_T=(TC, TH), wall_ux=(0.0, u0))
    s = Solver(p, np.ones((ny, nx)), u0 * Y, np.zeros((ny, nx)), TC + (TH - TC) * Y, device=DEV)
    s.step(int(8.0 * max(1.0, Pr) * Re / u0 / math.pi ** 2 / s.dt))
    T = s.moments(fields=True, sums=False)["T"].cpu().numpy()
    s.close()
    th = (T - TC) / (TH - TC)
    ref = (y + Pr * Ec / 2 * y * (1 - y))[:, None]
    err = float(np.abs(th - ref).max()) / float(ref.max())
    print(f"[couette] Ma {Ma} Ec {Ec} split {split} Pr {Pr}: max error {err:.2e} of the peak", flush=True)
    assert np.isfinite(th).all()
    assert np.abs(th - th[:, :1]).max() < 1e-12  # x-independent
    if Ma > 1:
        assert err < 0.05
    else:
        assert err < (0.03 if (split == 1 and Pr == 2.0) else 0.01)


# ---------------------------------------------------------------- Sod shock tube (Sec. IV, conservation)
@pytest.mark.parametrize("split", (1, 2))
@pytest.mark.parametrize("Pr", (0.5, 1.0, 2.0))
def test_sod_tube_matches_oracle(split, Pr):
    """The Sod tube's discontinuities put the limiter on all of its branches:
    128 x 4 cells of the extended periodic domain, 20 steps, FP64."""
    wl = sod_tube(128, 4)
    s, p = solver(wl, split=split, storage="f64", Pr=Pr, tau_ref=5e-4)
    cfg = oracle_cfg(p)
    f0, g0 = oracle_state(s)
    s.step(20)
    f, g = oracle_state(s)
    fo, go = O.run(f0, g0, cfg, s.dt, 20)
    assert rel(f, fo) < 1e-12 and rel(g, go) < 1e-12
    assert rel(f - f0, fo - f0) < 1e-9 and rel(g - g0, go - g0) < 1e-9


@pytest.mark.parametrize("split", (1, 2))
@pytest.mark.parametrize("Pr", (0.5, 1.0, 2.0))
def test_sod_tube_conservation(split, Pr):
    """The paper's conservation case: 1024 x 4 cells of x in [-0.5, 1.5],
    CFL 0.01, mu = 5e-5, FP64 storage, run to t = 0.2.  Total mass and energy
    (float64 sums over the domain) change by rounding only (below 2^-53 per
    step; measured 1e-14 to 5e-13 over 12116 steps), the x momentum stays at
    rounding level, and the density on [0, 1] is within 2 % (relative L1) of
    the exact Riemann solution of the Euler equations."""
    wl = sod_tube(1024, 4)
    s, p = solver(wl, split=split, storage="f64", Pr=Pr, tau_ref=5e-5)
    m0 = s.moments(fields=False, sums=True)["sums"]
    dt = s.dt
    n = int(round(0.2 / dt))
    s.step(n)
    out = s.moments(fields=True, sums=True)
    m1 = out["sums"]
    s.close()
    eps = 2.0 ** -53
    # density on [0, 1] against the exact Riemann solution (Euler level)
    x = (np.arange(1024) + 0.5) * (2.0 / 1024) - 0.5
    sel = (x >= 0.0) & (x <= 1.0)
    rho = out["rho"].cpu().numpy()[0, sel]
    ex = riemann_density(x[sel] - 0.5, n * dt, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4)
    l1 = float(np.abs(rho - ex).mean() / np.abs(ex).mean())
    print(f"[sod] split {split} Pr {Pr}: {n} steps, mass {abs(m1[0] / m0[0] - 1):.2e}, "
          f"energy {abs(m1[3] / m0[3] - 1):.2e}, momentum {abs(m1[1]) / m0[0]:.2e}, density L1 vs Riemann {l1:.2e}",
          flush=True)
    assert abs(m1[0] / m0[0] - 1) < eps * n
    assert abs(m1[3] / m0[3] - 1) < eps * n
    assert abs(m1[1]) < eps * n * m0[0]
    assert l1 < 0.02


# ---------------------------------------------------------------- errors raised from device checks
def test_zero_and_negative_step_counts():
    wl = smooth_random(16, 16, seed=1)
    s, _ = solver(wl, tau_ref=0.02)
    X0 = s.store_populations()
    idx = s.state_index
    s.step(0)
    assert s.state_index == idx and torch.equal(s.store_populations(), X0)
    with pytest.raises(DVBMError) as e:
        s.step(-1)
    assert e.value.code == dvbm.DVBM_EINVAL
    assert torch.equal(s.store_populations(), X0)
    s.close()


def test_nonphysical_initial_state_rejected():
    wl = smooth_random(16, 16, seed=1)
    wl.T[3, 4] = -1.0
    with pytest.raises(DVBMError) as e:
        solver(wl, tau_ref=0.02)
    assert e.value.code == dvbm.DVBM_ENAN


def test_stiff_relaxation_rejected():
    wl = smooth_random(16, 16, seed=1)
    with pytest.raises(DVBMError) as e:
        solver(wl, tau_ref=1e-6, cfl=0.5)
    assert e.value.code == dvbm.DVBM_ESTIFF


@pytest.mark.parametrize("kernel", ("cell", "sweep", "tile"))
@pytest.mark.parametrize("storage", ("f32_dev", "bf16_dev", "fp16_dev"))
@pytest.mark.parametrize("split", (1, 2))
def test_rest_state_stores_zero_deviations(split, storage, kernel):
    """The rest equilibrium (rho = 1, u = 0, T = T_ref) is the deviation
    formats' reference, so its stored deviations (X / w - r, formed in float64
    and rounded once) are zero up to the float64 residue of X / w - r, and stay
    so over 10 steps.  Rounding X to float32 before subtracting would leave
    about 6e-8."""
    wl = uniform(70, 9)
    s, p = solver(wl, split=split, storage=storage, tau_ref=0.02, cfl=0.1, T_ref=1.0, kernel=kernel)
    dt = {"f32_dev": torch.float32, "bf16_dev": torch.bfloat16, "fp16_dev": torch.float16}[storage]
    pitch = dvbm.load_library().dvbm_pitch(ctypes.byref(p))

    def devs():  # buffer rows hold the Q planes of a distribution side by side
        b = s.state_buffer.view(dt).reshape(2, p.ny, s.Q, pitch).transpose(1, 2)
        return b.reshape(2 * s.Q, p.ny, pitch)[:, :, : p.nx].float()

    d0 = devs()
    assert float(d0[: s.Q].abs().max()) == 0.0  # f: X / w = 1 exactly
    assert float(d0.abs().max()) <= 1e-12
    hist = []
    for _ in range(10):
        s.step(1)
        d = devs()
        hist.append((float(d[: s.Q].abs().max()), float(d[s.Q:].abs().max()),
                     int(d[s.Q:].abs().amax(dim=(1, 2)).argmax())))
    print(f"[rest state] split {split} {storage} {kernel}: max |d| per step (f, g, worst g plane) {hist}", flush=True)
    assert max(max(f, g) for f, g, _ in hist) <= 1e-12
    s.close()


@pytest.mark.parametrize("split", (1, 2))
def test_population_buffer_layout(split):
    """The population buffer holds element (d, i, y, x) at ((d ny + y) Q + i) pitch + x, as the header
    states: float64 populations loaded from the dense [2][Q][ny][nx] array are found there bit for bit."""
    wl = smooth_random(70, 9, seed=4)
    s, p = solver(wl, split=split, storage="f64", tau_ref=0.02, cfl=0.1)
    Q = s.Q
    X = torch.tensor(np.random.default_rng(7).standard_normal((2, Q, p.ny, p.nx)))
    s.load_populations(X)
    pitch = dvbm.load_library().dvbm_pitch(ctypes.byref(p))
    raw = s.state_buffer.view(torch.float64).cpu()
    assert raw.numel() == 2 * p.ny * Q * pitch
    d, i, y, x = torch.meshgrid(*(torch.arange(n) for n in (2, Q, p.ny, p.nx)), indexing="ij")
    idx = ((d * p.ny + y) * Q + i) * pitch + x
    assert torch.equal(raw[idx.reshape(-1)].reshape(X.shape), X)
    s.close()


@pytest.mark.parametrize("storage", ("f64", "f32", "bf16_dev", "f32_dev"))
def test_step_from_matches_step(storage):
    """dvbm_step_from(src, dst) computes the same step as dvbm_step and leaves the handle's state alone."""
    wl = smooth_random(70, 37, seed=12)
    s, p = solver(wl, split=2, storage=storage, Pr=0.7, tau_ref=0.02, cfl=0.1)
    s.step(2)
    idx = s.state_index
    src = s.state_buffer.clone()
    dst = torch.empty_like(src)
    s.step_from(src, dst)
    assert s.state_index == idx and torch.equal(s.state_buffer, src)
    s.step(1)
    # compare the cells only (the pitch padding of the two buffers holds unrelated bytes)
    dt = {"f64": torch.float64, "f32": torch.float32, "bf16_dev": torch.int16, "f32_dev": torch.float32}[storage]
    pitch = dvbm.load_library().dvbm_pitch(ctypes.byref(p))

    def cells(buf):  # buffer rows hold the Q planes of a distribution side by side
        return buf.view(dt).reshape(2, p.ny, s.Q, pitch)[..., : p.nx]

    assert torch.equal(cells(s.state_buffer), cells(dst))


@pytest.mark.parametrize("nsteps", (300, 5000))
def test_vortex_1024_fp32_vs_fp64(nsteps):
    """Ma = 1 isentropic vortex on 1024^2 (column-sweep kernel), 300 steps and
    the workload's full 5000: the float32 runs (values and deviations) stay
    within 1e-5 relative L2 of the float64-storage run (itself checked against
    the oracle above) in rho and T, also after 8 x 8 block averaging to 128^2."""
    wl = isentropic_vortex(1024, seed=0, mach_adv=1.0, mach_v=0.3, r_frac=0.05)
    out = {}
    for storage in ("f64", "f32", "f32_dev"):
        s, _ = solver(wl, split=2, storage=storage, Pr=0.71, tau_ref=5e-5)
        s.step(nsteps)
        out[storage] = s.moments(fields=True, sums=False)
        s.close()
    pool = torch.nn.functional.avg_pool2d
    for st in ("f32", "f32_dev"):
        for k in ("rho", "T"):
            a, b = out[st][k], out["f64"][k]
            full, down = rel(a, b), rel(pool(a[None, None], 8), pool(b[None, None], 8))
            print(f"[vortex 1024] {st}, {nsteps} steps, {k}: relative L2 against f64 {full:.2e}, on the 128^2 "
                  f"average {down:.2e}", flush=True)
            assert full < 1e-5 and down < 1e-5, (st, k)


@pytest.mark.parametrize("Pr,gamma", [(Pr, g) for Pr in (0.1, 0.71, 2.0) for g in (1.4, 5.0 / 3.0)])
def test_shock_vortex_2048x1024_fp32_vs_fp64_8000_steps(Pr, gamma):
    """The 2048 x 1024 shock-vortex workload over its 8000 steps, each (Pr,
    gamma) pair: both float32 storages against the float64-storage run (itself
    checked against the oracle on sampled cells), relative L2 of rho and T.
    Measured: f32 rho 6.9e-6 to 1.0e-5, T 1.06e-5 to 2.0e-5; f32_dev rho 7.5e-6
    to 9.5e-6, T 1.04e-5 to 1.37e-5 (8 x 8 block averages within 8 % of these).
    Density meets 1e-5; temperature, the difference of the total and the
    kinetic energy in this Mach 1.2 flow, does not: deviations from the rest
    state are as large as the values here, so f32_dev gains little.  The
    bounds (rho 1.5e-5, T 3e-5 and 2e-5) hold what was measured."""
    wl = shock_vortex(2048, 1024, mach_s=1.2, mach_v=0.25, r_frac=0.075, gamma=gamma)
    out = {}
    for storage in ("f64", "f32", "f32_dev"):
        s, _ = solver(wl, split=2, storage=storage, Pr=Pr, gamma=gamma, tau_ref=wl.phys["mu"],
                      bc_x="zero_gradient", bc_y="periodic")
        s.step(8000)
        m = s.moments(fields=True)
        assert np.isfinite(m["sums"]).all()
        out[storage] = {k: m[k] for k in ("rho", "T")}
        s.close()
    errs = {(st, k): rel(out[st][k], out["f64"][k]) for st in ("f32", "f32_dev") for k in ("rho", "T")}
    print(f"[shock-vortex 2048x1024] Pr {Pr} gamma {gamma:.3f}, 8000 steps: "
          + ", ".join(f"{st} {k} {v:.2e}" for (st, k), v in errs.items()), flush=True)
    assert errs["f32", "rho"] < 1.5e-5 and errs["f32_dev", "rho"] < 1.5e-5
    assert errs["f32", "T"] < 3e-5 and errs["f32_dev", "T"] < 2e-5


def test_thermal_wave_4096_precision_2000_steps():
    """The 4096^2 thermal wave over 2000 steps (CFL 0.01, dt / tau = 0.04):
    a step moves a population by a few float32 ulps in all, so float32 values
    drift from the float64-storage run by 2e-5 (relative L2, growing with the
    step count), while float32 deviations from the rest state, a twentieth of
    the values' size here, stay within 1e-5, in the column sweep and in the
    per-cell kernel alike.

    Conductivity from the same runs: over 4e-3 time units (0.5 % of the
    acoustic time L / c) the density does not move, so the wave's mode decays
    at the isochoric diffusivity kappa / (rho c_v) = gamma nu / Pr, less the
    start-up of the heat flux from the initial equilibrium (about tau_alpha =
    mu / (p Pr)): rate = gamma (nu / Pr)(1 - tau_alpha / t).  The float64 run
    gives it within 1e-3 (measured 5e-4).  The decay is 1.1e-6 in T over the
    run, near what float32 storage resolves: float32 deviations give it within
    5 % (measured +1.5 % and +3.2 % for two rounding orders of the same
    arithmetic, -1.6 % on the per-cell kernel); float32 values, whose drift is
    of the size of the decay, give 2.5 to 3.4 times it and are not checked."""
    wl = thermal_wave(4096, seed=0)
    out, rate = {}, {}
    y = torch.tensor((np.arange(4096) + 0.5) / 4096, device=DEV)
    mode = torch.exp(-2j * math.pi * y)

    def amplitude(T):  # |T_k| of the wave's mode sin(2 pi y), float64 projection of the x-average
        return float(torch.abs(2 * ((T - T.mean()).mean(dim=1) * mode).mean()))

    for storage, kernel in (("f64", "auto"), ("f32", "auto"), ("f32_dev", "auto"), ("f32_dev", "cell")):
        print(f"[thermal 4096] {storage} {kernel}", flush=True)
        s, _ = solver(wl, split=2, storage=storage, Pr=0.5, tau_ref=5e-5, kernel=kernel)
        a0 = amplitude(s.moments(fields=True, sums=False)["T"])
        s.step(2000)
        m = s.moments(fields=True, sums=False)
        key = storage if kernel == "auto" else f"{storage}_{kernel}"
        out[key] = {k: m[k] for k in ("rho", "T")}
        rate[key] = math.log(a0 / amplitude(m["T"])) / ((2 * math.pi) ** 2 * 2000 * s.dt)
        t_run = 2000 * s.dt
        s.close()
        del s, m
        torch.cuda.empty_cache()
    # conductivity: the run lasts 0.5 % of the acoustic time, so the wave decays at the isochoric
    # diffusivity gamma nu / Pr, over the elapsed time less the heat flux's start-up (tau_alpha = 1e-4)
    expected = 1.4 * (5e-5 / 0.5) * (1.0 - 1e-4 / t_run)
    print("[thermal 4096] decay rate / k^2 over gamma (nu/Pr)(1 - tau_alpha/t): "
          + ", ".join(f"{k} {v / expected:.5f}" for k, v in rate.items()), flush=True)
    errs = {(st, k): rel(out[st][k], out["f64"][k]) for st in ("f32", "f32_dev", "f32_dev_cell") for k in ("rho", "T")}
    print("[thermal 4096] relative L2 against f64 after 2000 steps: "
          + ", ".join(f"{st} {k} {v:.2e}" for (st, k), v in errs.items()), flush=True)
    assert errs["f32_dev", "rho"] < 1e-5 and errs["f32_dev", "T"] < 1e-5
    assert errs["f32_dev_cell", "rho"] < 1e-5 and errs["f32_dev_cell", "T"] < 1e-5
    assert errs["f32", "rho"] < 5e-5 and errs["f32", "T"] < 5e-5
    assert abs(rate["f64"] / expected - 1) < 1e-3
    assert abs(rate["f32_dev"] / expected - 1) < 5e-2 and abs(rate["f32_dev_cell"] / expected - 1) < 5e-2


@pytest.mark.parametrize("storage", ("bf16_dev", "fp16_dev"))
def test_adjoint_rejects_16bit_storage(storage):
    wl = smooth_random(16, 16, seed=40)
    s, _ = solver(wl, split=2, storage=storage, tau_ref=0.02)
    lam = s.new_cotangent()
    with pytest.raises(DVBMError) as e:
        s.adjoint_step(s.state_buffer, lam, torch.empty_like(lam), torch.zeros(2, dtype=torch.float64, device=DEV))
    assert e.value.code == dvbm.DVBM_EINVAL
    s.close()


def riemann_density(x, t, left, right, gamma):
    """Exact density of the 1-D Euler Riemann problem for an ideal gas at time
    t, interface at x = 0 (states (rho, u, p)): the star pressure from the
    shock / rarefaction pressure functions by Newton iteration, then the wave
    fan sampled at x / t (textbook construction, e.g. Toro, ch. 4)."""
    rl, ul, pl = left
    rr, ur, pr = right
    g1, g2 = (gamma - 1) / (2 * gamma), (gamma + 1) / (2 * gamma)
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)

    def fk(p, rk, pk, ck):
        if p > pk:  # shock
            a, b = 2 / ((gamma + 1) * rk), (gamma - 1) / (gamma + 1) * pk
            q = math.sqrt(a / (p + b))
            return (p - pk) * q, q * (1 - 0.5 * (p - pk) / (p + b))
        # rarefaction
        return 2 * ck / (gamma - 1) * ((p / pk) ** g1 - 1), (p / pk) ** (-g2) / (rk * ck)

    p = 0.5 * (pl + pr)
    for _ in range(100):
        f1, d1 = fk(p, rl, pl, cl)
        f2, d2 = fk(p, rr, pr, cr)
        step = (f1 + f2 + ur - ul) / (d1 + d2)
        p = max(p - step, 1e-12)
        if abs(step) < 1e-14 * p:
            break
    us = 0.5 * (ul + ur) + 0.5 * (fk(p, rr, pr, cr)[0] - fk(p, rl, pl, cl)[0])
    out = np.empty_like(x)
    for k, xk in enumerate(x):
        s = xk / t
        if s <= us:  # left of the contact
            if p > pl:
                sl = ul - cl * math.sqrt(g2 * p / pl + g1)
                out[k] = rl if s < sl else rl * ((p / pl + (gamma - 1) / (gamma + 1)) /
                                               ((gamma - 1) / (gamma + 1) * p / pl + 1))
            else:
                shl, cs = ul - cl, cl * (p / pl) ** g1
                stl = us - cs
                if s < shl:
                    out[k] = rl
                elif s > stl:
                    out[k] = rl * (p / pl) ** (1 / gamma)
                else:
                    out[k] = rl * (2 / (gamma + 1) + (gamma - 1) / ((gamma + 1) * cl) * (ul - s)) ** (2 / (gamma - 1))
        else:
            if p > pr:
                sr = ur + cr * math.sqrt(g2 * p / pr + g1)
                out[k] = rr if s > sr else rr * ((p / pr + (gamma - 1) / (gamma + 1)) /
                                               ((gamma - 1) / (gamma + 1) * p / pr + 1))
            else:
                shr, cs = ur + cr, cr * (p / pr) ** g1
                str_ = us + cs
                if s > shr:
                    out[k] = rr
                elif s < str_:
                    out[k] = rr * (p / pr) ** (1 / gamma)
                else:
                    out[k] = rr * (2 / (gamma + 1) - (gamma - 1) / ((gamma + 1) * cr) * (ur - s)) ** (2 / (gamma - 1))
    return out


# ---------------------------------------------------------------- dispersion: speed of sound (Sec. IV)
@pytest.mark.parametrize("split", (1, 2))
@pytest.mark.parametrize("theta,mach", ((0.8, 0.0), (1.0, 0.0), (1.25, 0.0), (1.0, 0.5), (1.0, 1.0)))
def test_speed_of_sound(split, theta, mach):
    """Speed of sound from an adiabatic standing wave (amplitude 1e-3, 256
    cells, FP64): the zero crossings of the density mode, with the advective
    phase of the flow removed, against sqrt(gamma R T) at T = theta T_ref,
    on flows up to Mach 1."""
    from synth import acoustic_wave
    n = 256
    wl = acoustic_wave(n, 4, theta=theta, mach=mach)
    s, p = solver(wl, split=split, storage="f64", Pr=0.71, tau_ref=1e-3, cfl=0.2)
    dt = s.dt
    c0 = math.sqrt(1.4 * theta)
    U = mach * c0
    e = np.exp(-2j * math.pi * (np.arange(n) + 0.5) / n)
    times, vals = [], []
    chunk = 10
    for m in range(int(1.3 / (c0 * dt)) // chunk):
        a = 2 * (s.moments(fields=True, sums=False)["rho"].cpu().numpy()[0] * e).mean()
        t = m * chunk * dt
        times.append(t)
        vals.append((a * np.exp(2j * math.pi * U * t)).real)
        s.step(chunk)
    s.close()
    v = np.array(vals)
    tt = np.array(times)
    z = [tt[i] - v[i] * (tt[i + 1] - tt[i]) / (v[i + 1] - v[i]) for i in range(len(v) - 1) if v[i] * v[i + 1] < 0]
    assert len(z) >= 2
    c = 0.5 / np.diff(z).mean()
    print(f"[sound] split {split} theta {theta} Ma {mach}: c / sqrt(gamma R T) - 1 = {c / c0 - 1:.2e}", flush=True)
    assert abs(c / c0 - 1) < 1e-3  # measured 0.8e-4 to 2.8e-4


# ---------------------------------------------------------------- dissipation: thermal diffusivity on a moving background (Sec. IV)
@pytest.mark.parametrize("split,mach", ((1, 0.0), (1, 0.5), (2, 0.0), (2, 0.5), (2, 1.0)))
@pytest.mark.parametrize("Pr", (0.5, 2.0))
def test_thermal_diffusivity_on_a_flow(split, Pr, mach):
    """An isobaric temperature wave T = 1 + 1e-3 sin(2 pi x), rho = 1/T, on a
    uniform flow U: its mode decays as exp(-alpha k^2 t) with alpha = nu / Pr
    (nu = mu / rho) less the anti-diffusion U^2 dt / 2 that forward Euler adds
    to advection (the modified equation of X <- X - dt U X_x).  At CFL 0.2
    that term is 8 % of nu / Pr at Mach 0.5, Pr 2, and it halves with dt.
    256 cells, FP64, mu = 2e-3, one decay time; alpha from a least-squares fit
    of log |T_k(t)|.  Split I (D2Q16) does not carry a Mach-1 flow at CFL 0.2
    (it diverges at Pr 0.5 and is 27 % off at Pr 2) and is run up to Mach 0.5."""
    n = 256
    amp, mu = 1e-3, 2e-3
    x = (np.arange(n) + 0.5) / n
    T = np.repeat((1.0 + amp * np.sin(2 * np.pi * x))[None, :], 4, 0)
    U = mach * math.sqrt(1.4)
    s = Solver(make_params(n, 4, dx=1.0 / n, dy=1.0 / n, split=split, storage="f64", Pr=Pr, tau_ref=mu, cfl=0.2),
               1.0 / T, np.full((4, n), U), np.zeros((4, n)), T, device=DEV)
    dt = s.dt
    k = 2 * math.pi
    e = np.exp(-1j * k * x)
    t_end = Pr / (mu * k * k)
    chunk = max(1, int(t_end / dt) // 200)
    ts, la = [], []
    for m in range(int(t_end / dt) // chunk):
        Tf = s.moments(fields=True, sums=False)["T"].cpu().numpy()[0]
        ts.append(m * chunk * dt)
        la.append(math.log(abs(2 * ((Tf - Tf.mean()) * e).mean())))
        s.step(chunk)
    s.close()
    alpha = -np.polyfit(np.array(ts), np.array(la), 1)[0] / (k * k)
    expected = mu / Pr - 0.5 * U * U * dt
    print(f"[thermal] split {split} Pr {Pr} Ma {mach}: alpha / (nu/Pr - U^2 dt/2) - 1 = {alpha / expected - 1:.2e}"
          f" (forward-Euler term {0.5 * U * U * dt * Pr / mu:.1e} of nu/Pr)", flush=True)
    assert abs(alpha - expected) < 0.01 * mu / Pr  # measured 5e-5 to 1.3e-3; 7.9e-3 for split II, Pr 0.5, Mach 1


# ---------------------------------------------------------------- dissipation: sound attenuation and bulk viscosity (Sec. II C, IV)
@pytest.mark.parametrize("split", (1, 2))
@pytest.mark.parametrize("Pr", (0.5, 2.0))
@pytest.mark.parametrize("gamma,mach", ((1.4, 0.0), (5.0 / 3.0, 0.0), (4.0 / 3.0, 0.0), (1.4, 0.5)))
def test_sound_attenuation(split, Pr, gamma, mach):
    """Decay of an adiabatic standing sound wave (amplitude 1e-3, 256 cells,
    FP64, mu = 2e-3, half a decay time): the right- and left-running waves
    u_k +- p_k / (rho c) (which the entropy mode, carrying no pressure, does
    not enter) each decay as exp(-Gamma k^2 t), less the anti-diffusion
    (U +- c)^2 dt / 2 that forward Euler adds to a wave of that speed."""
    from synth import acoustic_wave
    n, mu = 256, 2e-3
    wl = acoustic_wave(n, 4, gamma=gamma, mach=mach)
    s, p = solver(wl, split=split, storage="f64", Pr=Pr, tau_ref=mu, gamma=gamma, cfl=0.2)
    dt = s.dt
    c = math.sqrt(gamma)
    U = mach * c
    k = 2 * math.pi
    G = sound_decay_rate(split, Pr, gamma, mu)
    e = np.exp(-1j * k * (np.arange(n) + 0.5) / n)
    nsteps = int(0.5 / (G * k * k) / dt)
    chunk = max(1, nsteps // 100)
    ts, lr, ll = [], [], []
    for m in range(nsteps // chunk):
        mo = {q: v.cpu().numpy()[0] for q, v in s.moments(fields=True, sums=False).items()}
        uk = 2 * (mo["ux"] * e).mean()
        pk = 2 * (mo["rho"] * mo["T"] * e).mean()
        ts.append(m * chunk * dt)
        lr.append(math.log(abs(uk + pk / c)))
        ll.append(math.log(abs(uk - pk / c)))
        s.step(chunk)
    s.close()
    worst = 0.0
    for logs, a in ((lr, U + c), (ll, U - c)):
        g = -np.polyfit(np.array(ts), np.array(logs), 1)[0] / (k * k)
        worst = max(worst, abs(g - (G - 0.5 * a * a * dt)) / G)
    print(f"[bulk] split {split} Pr {Pr} gamma {gamma:.3f} Ma {mach}: |Gamma_measured - Gamma| / Gamma = {worst:.2e}"
          f" (forward-Euler term {0.5 * (U + c) ** 2 * dt / G:.2f} of Gamma)", flush=True)
    assert worst < 1e-2  # measured 1.4e-5 to 8.7e-4; 4.7e-3 for split I, Pr 0.5, Mach 0.5


# ---------------------------------------------------------------- shock-vortex sound diagnostics (Sec. IV)
@pytest.mark.parametrize("case,mach_s,mach_v", (("C", 1.2, 0.25), ("G", 1.29, 0.39)))
def test_shock_vortex_sound(case, mach_s, mach_v):
    """Cases C (Ma_s 1.2, Ma_v 0.25) and G (Ma_s 1.29, Ma_v 0.39) of the
    shock-vortex interaction (Re_v 800, Pr 0.75, split II) on the 28 x 24 r_v domain at 60 cells per r_v, shock at
    x = 8, vortex at (6, 12), zero-gradient x boundaries; CFL 0.1 (at CFL 0.2
    the post-shock dt / tau_1 is 1.2 and the run diverges).  Properties that
    hold without the reference DNS data:
    * the vortex centre (its vorticity minimum: it turns clockwise) moves with
      the post-shock flow speed u_r (t* 4 to 10);
    * along the 45 degree ray, the peaks of the precursor and of the second
      sound move outwards at the post-shock sound speed, approached from above
      as the fronts grow (a front centred off the vortex centre runs ahead of
      c_r along the ray by a share that falls as its radius grows): between
      t* = 8 and 10 within -2 % to +5 % of c_r / c_l per unit t*, and slower
      than between t* = 6 and 8 (measured in case C 3.6 % and 0.1 % above,
      in case G 3.2 % above and 0.9 % below: a weak wave of amplitude p'/p
      runs at c (1 + (gamma + 1)/(2 gamma) p'/p), and case G's second sound
      is a rarefaction of about 1 %);
    * ahead of the precursor (r from 9 to 13 r_v at t* = 6) the field is quiet;
    * (case C) float32 and float64 storage give the same vortex centre and sound
      pressure at t* = 6 (8,800 steps), within what 8,800 float32 steps
      through a shock accumulate: relative L2 of the pressure 1.3e-4, largest
      at the shock (a sub-cell shift of it), and 1.2e-4 of p_r along the
      ray (2 % of the precursor's peak).  Float32 deviations do no better
      here (1.5e-4): at Mach 1.2 the deviation from the rest state is as
      large as the value."""
    from paper_2510_04197_amd import diagnostics as Dg
    from synth import shock_vortex
    wl = shock_vortex(1680, 1440, mach_s, mach_v, 1.0 / 24.0, Lx=28.0, Ly=24.0, x_shock=8.0)
    ph = wl.phys
    c_ratio = math.sqrt(ph["T_post"])  # c_r / c_l with T_l = 1
    radii = np.arange(0.0, 13.0, 0.05)
    rays, centres, fields6 = {}, {}, {}
    runs = (("f32", (4.0, 6.0, 8.0, 10.0)), ("f64", (6.0,)), ("f32_dev", (6.0,)))
    for storage, t_stars in runs if case == "C" else runs[:1]:
        print(f"[shock-vortex] case {case}, {storage}", flush=True)
        s, p = solver(wl, split=2, storage=storage, Pr=0.75, gamma=1.4, tau_ref=ph["mu"], bc_x="zero_gradient",
                      bc_y="periodic", cfl=0.1)
        dt, n, c = s.dt, 0, ph["centre"]
        for ts in t_stars:
            target = int(round(ts * ph["rv"] / ph["c_l"] / dt))
            guess = (c[0] + (target - n) * dt * ph["u_post"], c[1])
            s.step(target - n)
            n = target
            m = {k: v.cpu().numpy() for k, v in s.moments(fields=True, sums=False).items()}
            ps = Dg.sound_pressure(m["rho"], m["T"], ph["p_post"])
            assert np.isfinite(ps).all()
            c = Dg.vortex_centre(Dg.vorticity(m["ux"], m["uy"], wl.dx, wl.dy), wl.dx, wl.dy, guess, 1.5)
            centres[storage, ts] = (n * dt, c)
            rays[storage, ts] = Dg.ray(ps, c, 45.0, radii, wl.dx, wl.dy)
            if ts == 6.0:
                fields6[storage] = ps
        s.close()

    (t4, c4), (t10, c10) = centres["f32", 4.0], centres["f32", 10.0]
    speed = (c10[0] - c4[0]) / (t10 - t4)
    print(f"[shock-vortex] case {case}: vortex speed / u_r - 1 = {speed / ph['u_post'] - 1:.2e}", flush=True)
    assert abs(speed / ph["u_post"] - 1) < 5e-3

    def peak(pr, lo, hi, sign):
        idx = np.where((radii >= lo) & (radii <= hi))[0]
        k = idx[np.argmax(sign * pr[idx])]
        a, b, cc = pr[k - 1], pr[k], pr[k + 1]
        return radii[k] + 0.05 * 0.5 * (a - cc) / (a - 2 * b + cc)

    for name, lo, hi, sign in (("precursor", 4.5, 12.5, 1), ("second sound", 2.5, 9.5, -1)):
        r6, r8, r10 = (peak(rays["f32", ts], lo, hi, sign) for ts in (6.0, 8.0, 10.0))
        early, late = (r8 - r6) / 2 / c_ratio, (r10 - r8) / 2 / c_ratio
        amp = float(np.interp(r10, radii, rays["f32", 10.0]) / (1.0 + np.interp(r10, radii, rays["f32", 10.0])))
        print(f"[shock-vortex] case {case}: {name} at r/r_v {r6:.3f} {r8:.3f} {r10:.3f}; speed / c_r: {early:.4f} "
              f"then {late:.4f}; amplitude p'/p at t* 10 {amp:+.2e}", flush=True)
        assert 0.98 <= late < 1.05 and late < early

    pr6 = rays["f32", 6.0]
    front = peak(pr6, 4.5, 12.5, 1)
    ahead = np.abs(pr6[radii >= 9.0]).max()
    print(f"[shock-vortex] case {case}, t* 6: precursor {pr6.max():.2e} at {front:.2f}; max |p_sound| ahead "
          f"{ahead:.1e}", flush=True)
    assert front < 7.5 and ahead < 0.1 * pr6.max()
    if case != "C":
        return

    c64 = centres["f64", 6.0][1]
    shift = math.hypot(c64[0] - centres["f32", 6.0][1][0], c64[1] - centres["f32", 6.0][1][1])
    ray_diff = np.abs(Dg.ray(fields6["f32"], c64, 45.0, radii, wl.dx, wl.dy) - rays["f64", 6.0])
    p32, p64 = fields6["f32"] + 1.0, fields6["f64"] + 1.0
    rel_l2 = float(np.linalg.norm(p32 - p64) / np.linalg.norm(p64))
    print(f"[shock-vortex] f32 vs f64 at t* 6: centre shift {shift:.1e} r_v; along the ray (same centre) max "
          f"{ray_diff.max():.1e}, beyond r = 1: {ray_diff[radii >= 1.0].max():.1e}; pressure rel. L2 {rel_l2:.1e}; "
          f"max |dp/p_r| {np.abs(p32 - p64).max():.1e}", flush=True)
    assert shift < 2e-3 and rel_l2 < 3e-4 and ray_diff.max() < 3e-4  # measured 7.4e-4, 1.3e-4, 1.2e-4
    pd = fields6["f32_dev"] + 1.0
    rel_dev = float(np.linalg.norm(pd - p64) / np.linalg.norm(p64))
    ray_dev = np.abs(Dg.ray(fields6["f32_dev"], c64, 45.0, radii, wl.dx, wl.dy) - rays["f64", 6.0]).max()
    print(f"[shock-vortex] f32_dev vs f64 at t* 6: pressure rel. L2 {rel_dev:.1e}, along the ray {ray_dev:.1e}", flush=True)
    assert rel_dev < 3e-4 and ray_dev < 3e-4


@pytest.mark.parametrize("split,theta,mach,gamma,bound", (
    (1, 0.1, 0.0, 1.4, 5e-3), (1, 10.0, 0.0, 1.4, 1e-3), (1, 100.0, 0.0, 1.4, 1e-3), (1, 1.0, 0.0, 5.0 / 3.0, 1e-3),
    (2, 0.1, 0.0, 1.4, 1e-2), (2, 30.0, 0.0, 1.4, 1e-3), (2, 1.0, 1.5, 1.4, 2e-3), (2, 1.0, 2.0, 1.4, 2e-3),
    (2, 1.0, 2.0, 4.0 / 3.0, 2e-3), (2, 1.0, 0.0, 5.0 / 3.0, 1e-3), (2, 0.5, 2.5, 1.4, 2e-3),
    (2, 0.5, 2.0, 5.0 / 3.0, 2e-3), (1, 0.3, 2.0, 1.4, 2e-3)))
def test_speed_of_sound_ranges(split, theta, mach, gamma, bound):
    """The speed of sound over the temperature and Mach ranges of the paper's
    study (Sec. IV), at its CFL of 0.01 (256 cells, FP64, tau_ref = 1e-3
    sqrt(theta)): split I (D2Q16) from T / T_ref = 0.1 to 100, split II
    (D2Q25) from 0.1 to 30 and up to Mach 2 (gamma 1.4 and 4/3); colder
    flows go further: split II at Mach 2.5 (T / T_ref = 0.5) and Mach 2 with
    gamma 5/3, split I at Mach 2 (T / T_ref = 0.3).  Measured
    (c / sqrt(gamma R T) - 1): 0.24 % (split I) and 0.55 % (split II) at
    T / T_ref = 0.1, at most 2.6e-4 from 0.3 to 100, 3.5e-4 to 8.4e-4 at
    Mach 1.5 to 2.5.  Beyond these the runs diverge or drift at this
    tau_ref: split I below T / T_ref = 0.05 and at Mach 2 at T_ref, split II
    at 100 T_ref, at Mach 2.5 at T_ref for tau_ref from 1e-3 up to 3e-2 and CFL
    down to 0.002, at Mach 3 at every temperature tried (0.2 to 1 T_ref), and
    at any Mach >= 2 at 0.2 T_ref.  The high-Mach limit is set by tau, not by
    the Mach number alone: at tau_ref = 5e-5 both splits stay bounded to
    Mach 3.5 (test_high_mach_bounded_at_small_tau, and the pressure-front
    test below)."""
    from synth import acoustic_wave
    n = 256
    wl = acoustic_wave(n, 4, theta=theta, mach=mach, gamma=gamma)
    s, _ = solver(wl, split=split, storage="f64", Pr=0.71, tau_ref=1e-3 * math.sqrt(theta), gamma=gamma, cfl=0.01)
    dt = s.dt
    c0 = math.sqrt(gamma * theta)
    U = mach * c0
    e = np.exp(-2j * math.pi * (np.arange(n) + 0.5) / n)
    nsteps = int(1.3 / (c0 * dt))
    chunk = max(1, nsteps // 120)
    times, vals = [], []
    for m in range(nsteps // chunk):
        a = 2 * (s.moments(fields=True, sums=False)["rho"].cpu().numpy()[0] * e).mean()
        t = m * chunk * dt
        times.append(t)
        vals.append((a * np.exp(2j * math.pi * U * t)).real)
        s.step(chunk)
    s.close()
    v, tt = np.array(vals), np.array(times)
    assert np.isfinite(v).all()
    z = [tt[i] - v[i] * (tt[i + 1] - tt[i]) / (v[i + 1] - v[i]) for i in range(len(v) - 1) if v[i] * v[i + 1] < 0]
    assert len(z) >= 2
    c = 0.5 / np.diff(z).mean()
    print(f"[sound range] split {split} theta {theta} Ma {mach} gamma {gamma:.3f}: c / sqrt(gamma R T) - 1 = "
          f"{c / c0 - 1:.2e}", flush=True)
    assert abs(c / c0 - 1) < bound


@pytest.mark.parametrize("split", (1, 2))
def test_high_mach_bounded_at_small_tau(split):
    """A Mach-3 sound wave (256 cells, amplitude 1e-3, CFL 0.01, FP64) at
    T_ref: with tau_ref = 5e-5 the density perturbation stays within its
    initial amplitude over 1.3 acoustic crossing times, while at tau_ref =
    1e-3 it grows past 10x within 0.6 of one (measured: growth 0.992 and
    0.997 at 5e-5; at 1e-3, 30x (split I) and 19x (split II) at the first
    check past 10x; the same holds at every amplitude from 1e-6 to 1e-3)."""
    from synth import acoustic_wave
    n, amp, mach, gamma = 256, 1e-3, 3.0, 1.4
    c0 = math.sqrt(gamma)
    growth = {}
    for tau in (5e-5, 1e-3):
        wl = acoustic_wave(n, 4, amp=amp, mach=mach, gamma=gamma)
        s, _ = solver(wl, split=split, storage="f64", Pr=0.71, gamma=gamma, tau_ref=tau, cfl=0.01)
        nsteps = int((1.3 if tau < 1e-4 else 0.6) / (c0 * s.dt))
        chunk = max(1, nsteps // 26)
        g = 0.0
        for _ in range(26):
            s.step(chunk)
            try:
                r = s.moments(fields=True, sums=True)["rho"]  # raises ENAN on a non-finite state
            except DVBMError:
                g = math.inf
                break
            g = max(g, float((r - r.mean()).abs().max()) / amp)
            if g > 10.0:
                break
        s.close()
        growth[tau] = g
    print(f"[high Mach] split {split} Ma 3: growth {growth[5e-5]:.3f} at tau 5e-5, {growth[1e-3]:.3g} at tau 1e-3",
          flush=True)
    assert growth[5e-5] < 1.0 and growth[1e-3] > 10.0


# ---------------------------------------------------------------- dissipation: shear viscosity on a moving background (Sec. IV)
@pytest.mark.parametrize("split,mach", ((1, 0.0), (1, 0.5), (2, 0.0), (2, 0.5), (2, 1.0)))
@pytest.mark.parametrize("Pr", (0.5, 2.0))
def test_shear_viscosity_on_a_flow(split, Pr, mach):
    """A shear wave u_y = 1e-3 sin(2 pi x) on a uniform flow U in x: its mode
    decays as exp(-nu_eff k^2 t) with nu_eff = nu (the shear time, whichever
    of tau_1, tau_2 carries it) less forward Euler's U^2 dt / 2.  256 cells,
    FP64, mu = 2e-3, CFL 0.2, one decay time."""
    n = 256
    amp, mu = 1e-3, 2e-3
    x = (np.arange(n) + 0.5) / n
    U = mach * math.sqrt(1.4)
    uy = np.repeat((amp * np.sin(2 * np.pi * x))[None, :], 4, 0)
    s = Solver(make_params(n, 4, dx=1.0 / n, dy=1.0 / n, split=split, storage="f64", Pr=Pr, tau_ref=mu, cfl=0.2),
               np.ones((4, n)), np.full((4, n), U), uy, np.ones((4, n)), device=DEV)
    dt = s.dt
    k = 2 * math.pi
    e = np.exp(-1j * k * x)
    nsteps = int(1.0 / (mu * k * k) / dt)
    chunk = max(1, nsteps // 200)
    ts, la = [], []
    for m in range(nsteps // chunk):
        v = s.moments(fields=True, sums=False)["uy"].cpu().numpy()[0]
        ts.append(m * chunk * dt)
        la.append(math.log(abs(2 * (v * e).mean())))
        s.step(chunk)
    s.close()
    nu = -np.polyfit(np.array(ts), np.array(la), 1)[0] / (k * k)
    expected = mu - 0.5 * U * U * dt
    print(f"[shear] split {split} Pr {Pr} Ma {mach}: nu / (mu - U^2 dt/2) - 1 = {nu / expected - 1:.2e}"
          f" (forward-Euler term {0.5 * U * U * dt / mu:.1e} of nu)", flush=True)
    assert abs(nu - expected) < 0.01 * mu  # measured 5e-5 to 7.7e-4 of nu


# ---------------------------------------------------------------- the paper's speed-of-sound test (Sec. IV)
def front_crossing(q, xc, level, dx, window=25):
    """Position (unwrapped around xc) where the periodic cell profile q falls
    through `level`, by linear interpolation between cell centres; of the
    downward crossings within `window` cells of xc, the nearest to xc."""
    n = len(q)
    k0 = int(np.floor(xc / dx - 0.5))
    best = float("nan")
    for k in range(k0 - window, k0 + window):
        a, b = q[k % n], q[(k + 1) % n]
        if a >= level > b:
            xk = (k + 0.5 + (a - level) / (a - b)) * dx
            if not abs(xk - xc) >= abs(best - xc):
                best = xk
    return best


def pressure_front_speed(split, theta, mach, gamma, Pr, n=512, amp=1e-6, cfl=0.01, run=0.15):
    """The paper's dispersion test: on a periodic pseudo-1-D line of n cells,
    p = 1 + amp for x <= 1/2 and 1 beyond, uniform T = theta T_ref and
    u = Ma sqrt(gamma R T).  The step at x = 1/2 splits into a right- and a
    left-running acoustic front, both pressure drops of amp / 2, moving at
    u + c and u - c (the entropy part carries no pressure), with a plateau of
    amp / 2 between them.  Each front is located where p - 1 falls through
    its mid level (3 amp / 4 for the left-runner, amp / 4 for the right-runner;
    linear interpolation, the crossing nearest to where the front should be),
    at 1/3 and at the end of the run (t = 0.15 / c, before any front meets
    another), so c = (v_+ - v_-) / 2 and the flow speed (v_+ + v_-) / 2 follow
    from the two front speeds.  mu = max(5e-5, 2 dt p) keeps dt / tau_1 <= 0.5
    (CFL 0.01 gives dt / tau > 2 in cold flows at mu = 5e-5).  Returns
    (c / sqrt(gamma R T) - 1, measured flow speed / u - 1 (at rest: the
    measured flow speed / c), whether the run stayed finite)."""
    ny = 4
    dx = 1.0 / n
    x = (np.arange(n) + 0.5) * dx
    c0 = math.sqrt(gamma * theta)
    U = mach * c0
    p0 = np.where(x <= 0.5, 1.0 + amp, 1.0)
    T = np.full((ny, n), theta)
    rho = np.repeat((p0 / theta)[None, :], ny, 0)
    dt_est = cfl * dx / (abs(U) + c0)
    Pr_eff = Pr if Pr > 1 else 1.0
    mu = max(5e-5, 2.0 * dt_est * (1.0 + amp) * Pr_eff)
    s = Solver(make_params(n, ny, dx=dx, dy=dx, split=split, storage="f64", Pr=Pr, gamma=gamma, tau_ref=mu, cfl=cfl),
               rho, np.full((ny, n), U), np.zeros((ny, n)), T, device=DEV)
    dt = s.dt
    t_end = run / c0
    n_end = int(round(t_end / dt))
    n_mid = n_end // 3
    pos = {}

    def locate(t):
        try:
            m = s.moments(fields=True, sums=True)  # raises ENAN on a non-finite state
        except DVBMError:
            return None
        pr = ((m["rho"] * m["T"]).mean(dim=0).cpu().numpy() - 1.0) / amp  # (p - 1) / amp, R = 1
        return [front_crossing(pr, 0.5 + v * t, level, dx) for v, level in ((U + c0, 0.25), (U - c0, 0.75))]

    s.step(n_mid)
    pos[1] = (n_mid * dt, locate(n_mid * dt))
    ok = pos[1][1] is not None
    if ok:
        s.step(n_end - n_mid)
        pos[2] = (n_end * dt, locate(n_end * dt))
        ok = pos[2][1] is not None
    s.close()
    if not ok:
        return float("nan"), float("nan"), False
    (t1, (r1, l1)), (t2, (r2, l2)) = pos[1], pos[2]
    vr, vl = (r2 - r1) / (t2 - t1), (l2 - l1) / (t2 - t1)
    c = 0.5 * (vr - vl)
    u = 0.5 * (vr + vl)
    return c / c0 - 1.0, (u / U - 1.0) if U else u / c0, True


@pytest.mark.parametrize("Pr", (0.5, 1.0, 2.0))
@pytest.mark.parametrize("gamma", (5.0 / 3.0, 4.0 / 3.0), ids=("5/3", "4/3"))
@pytest.mark.parametrize("split", (1, 2))
def test_pressure_front_speed_paper_ranges(split, gamma, Pr):
    """The paper's speed-of-sound test (Sec. IV, dispersion): a pressure step
    of 1e-6 on 512 cells at CFL 0.01, both fronts tracked (pressure_front_speed).
    Measured over both gamma and the three Pr:
      - at T_ref, Mach 0 to 3: |c / sqrt(gamma R T) - 1| at most 0.29 % to
        Mach 2.5 (split I) and 2 (split II), 0.29 % and 0.82 % at Mach 3
        (finite to Mach 3.5: 0.56 % and 2.0 %); the flow speed within 0.23 %;
      - at rest, split I (D2Q16) from T / T_ref = 0.03 to 300: 1.15 % at 0.03,
        at most 0.30 % from 0.1 to 100, 0.75 % at 300 (5.3 % at 0.01);
        split II (D2Q25) from 0.03 to 30: 1.45 % at 0.03, at most 0.41 % from
        0.1 to 10, 0.87 % at 30 (8.8 % at 0.01), and the run diverges at
        100 T_ref: four and three orders of temperature within about 1 %,
        the ranges the paper reports for the two velocity sets."""
    mach_pts = [(1.0, m, 4e-3) for m in (0.0, 1.0, 2.0)] + [(1.0, 3.0, 1.2e-2)]
    if split == 1:
        temp_pts = [(0.01, 0.0, 8e-2), (0.03, 0.0, 1.6e-2), (0.1, 0.0, 4e-3), (10.0, 0.0, 4e-3),
                    (100.0, 0.0, 4e-3), (300.0, 0.0, 1e-2)]
    else:
        temp_pts = [(0.03, 0.0, 2e-2), (0.1, 0.0, 6e-3), (0.3, 0.0, 4e-3), (10.0, 0.0, 4e-3), (30.0, 0.0, 1.2e-2)]
    for theta, mach, bound in mach_pts + temp_pts:
        e, u, ok = pressure_front_speed(split, theta, mach, gamma, Pr)
        print(f"[pressure front] split {split} gamma {gamma:.3f} Pr {Pr} T/T_ref {theta} Ma {mach}: "
              f"c / sqrt(gamma R T) - 1 = {e:.2e}, flow speed error {u:.1e}", flush=True)
        assert ok and abs(e) < bound, (theta, mach, e)
        assert abs(u) < 5e-3, (theta, mach, u)
    if split == 2:
        assert not pressure_front_speed(split, 100.0, 0.0, gamma, Pr)[2]  # D2Q25's upper temperature limit


