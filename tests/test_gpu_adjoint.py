"""GPU adjoint (dvbm_adjoint_*) against the FP64 oracle's reverse-mode derivative
(PyTorch autograd through the oracle's step) and against central finite
differences of the FP64 forward.

Tolerances: the adjoint arithmetic is float64 for both float64 and float32
storage, so step-level cotangents agree with the oracle to 1e-11 relative L2
(rounding only), and whole rollouts to 1e-10. Central differences are
secants across the flux limiter's kinks, with an error proportional to h
(see test_adjoint_vs_central_differences_256).
"""

import math

import numpy as np
import pytest
import torch

from oracle import dvbm_oracle as O
from paper_2510_04197_amd import Solver, make_params, rollout_temperature
from adjoint_windows import oracle_adjoint_windows
from synth import gaussian_bump, smooth_random, thermal_wave

pytestmark = pytest.mark.gpu
DEV = "cuda"


def oracle_cfg(p) -> O.Config:
    inv_bc = {0: O.PERIODIC, 1: O.ZERO_GRADIENT}
    return O.Config(nx=p.nx, ny=p.ny, split=p.split, bc_x=inv_bc[p.bc_x], bc_y=inv_bc[p.bc_y],
                    visc_mode=O.CONST_MU if p.visc_mode == 0 else O.CONST_TAU, dx=p.dx, dy=p.dy, R=p.R,
                    gamma=p.gamma, Pr=p.Pr, tau_ref=p.tau_ref, p_ref=p.p_ref, T_ref=p.T_ref, beta=p.beta,
                    cfl=p.cfl)


def rel(a, b):
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def step_adjoint_vs_oracle(nx, ny, split, Pr, bc_x, bc_y, storage, seed=11):
    """Relative L2 error of one adjoint step (lam0, d/dtau_ref, d/dPr) against
    reverse mode through the oracle's step, on random lam' and a perturbed state."""
    print(f"[adjoint step] {nx}x{ny} split={split} Pr={Pr} bc=({bc_x},{bc_y}) {storage}", flush=True)
    wl = smooth_random(nx, ny, seed=seed)
    p = make_params(wl.nx, wl.ny, dx=wl.dx, dy=wl.dy, split=split, storage=storage, Pr=Pr, tau_ref=0.02,
                    bc_x=bc_x, bc_y=bc_y, dt=3e-3, R=1.1, T_ref=0.9, gamma=1.3)
    s = Solver(p, wl.rho, wl.ux, wl.uy, wl.T, device=DEV)
    cfg = oracle_cfg(p)
    f0, g0 = O.initial_state(wl.rho, wl.ux, wl.uy, wl.T, cfg)
    rng = np.random.default_rng(0)
    X = torch.stack([f0, g0]) * (1 + 0.01 * torch.tensor(rng.standard_normal((2,) + tuple(f0.shape))))
    s.load_populations(X)
    X = s.store_populations().cpu()  # the state as stored (rounded for f32)
    lam1 = torch.tensor(rng.standard_normal(tuple(X.shape)))
    lam0 = s.new_cotangent()
    dpar = torch.zeros(2, dtype=torch.float64, device=DEV)
    s.adjoint_step(s.state_buffer, lam1.to(DEV), lam0, dpar)
    torch.cuda.synchronize()
    # oracle: reverse mode through the oracle's step
    fr = X[0].clone().requires_grad_()
    gr = X[1].clone().requires_grad_()
    tau = torch.tensor(0.02, dtype=torch.float64, requires_grad=True)
    prt = torch.tensor(Pr, dtype=torch.float64, requires_grad=True)
    fn, gn = O.step(fr, gr, cfg, 3e-3, tau, prt)
    ((lam1[0] * fn).sum() + (lam1[1] * gn).sum()).backward()
    ref = torch.stack([fr.grad, gr.grad])
    d = dpar.cpu()
    s.close()
    return rel(lam0.cpu(), ref), (float(d[0]), float(d[1])), (float(tau.grad), float(prt.grad))


def check_step_adjoint(res):
    e_lam, got, want = res
    assert e_lam < 1e-11
    for g, w in zip(got, want):
        assert abs(g - w) <= 1e-10 * abs(w) + 1e-14


BCS = (("periodic", "periodic"), ("zero_gradient", "periodic"), ("periodic", "zero_gradient"),
       ("zero_gradient", "zero_gradient"))


@pytest.mark.parametrize("split", (1, 2))
@pytest.mark.parametrize("Pr", (0.6, 1.0, 1.7))
@pytest.mark.parametrize("bc", BCS, ids=lambda b: f"{b[0][0]}{b[1][0]}")
@pytest.mark.parametrize("storage", ("f64", "f32", "f32_dev"))
def test_step_adjoint_matches_oracle(split, Pr, bc, storage):
    # 70 x 13: two strips of 58 columns (the second ragged), two row ranges of 8 and 5 rows
    check_step_adjoint(step_adjoint_vs_oracle(70, 13, split, Pr, bc[0], bc[1], storage))


@pytest.mark.parametrize("shape", ((4, 4), (5, 9), (117, 17), (600, 400)), ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("bc", (BCS[0], BCS[3]), ids=lambda b: f"{b[0][0]}{b[1][0]}")
def test_step_adjoint_grid_shapes(shape, bc):
    # the smallest grid (the row walk wraps the whole domain), a last row range of
    # one row, two full strips and a one-column strip, and a grid whose row
    # ranges are longer than the minimum (11 rows, the last one 4)
    check_step_adjoint(step_adjoint_vs_oracle(shape[0], shape[1], 2, 0.71, bc[0], bc[1], "f64", seed=3))


@pytest.mark.parametrize("storage,nx,ny,bc_x", (("f64", 4096, 4096, "periodic"), ("f32_dev", 4099, 2053, "periodic"),
                                                 ("f32", 2048, 1024, "zero_gradient")))
def test_step_adjoint_full_size_sampled(storage, nx, ny, bc_x):
    """One adjoint step on the 4096^2 grid of the precision workload (float64
    storage), on a ragged 4099 x 2053 grid (float32 deviations: 70 strips of
    58 columns and a 39-column tail) and on the 2048 x 1024 shock-vortex grid
    with zero-gradient x (float32), the state perturbed by 1 % noise so the
    limiter takes every branch: lam at 36 sampled cells against the oracle's
    reverse mode on periodic windows (1e-11).  The periodic grids' samples
    include the corners; with zero-gradient x the samples keep 4 cells from
    the x edges, where a periodic window equals the domain (the edges' ghost
    shares are checked element by element on the small grids)."""
    wl = thermal_wave(nx, seed=0) if nx == ny else smooth_random(nx, ny, seed=4)
    p = make_params(wl.nx, wl.ny, dx=wl.dx, dy=wl.dy, split=2, storage=storage, Pr=0.5, tau_ref=2e-3, bc_x=bc_x)
    s = Solver(p, wl.rho, wl.ux, wl.uy, wl.T, device=DEV)
    gen = torch.Generator(device=DEV).manual_seed(3)
    X = s.store_populations()
    X.mul_(1.0 + 0.01 * torch.randn(X.shape, generator=gen, device=DEV, dtype=torch.float64))
    s.load_populations(X)
    X = s.store_populations()  # the state as stored
    lam1 = torch.randn(X.shape, generator=gen, device=DEV, dtype=torch.float64)
    lam0 = s.new_cotangent()
    s.adjoint_step(s.state_buffer, lam1, lam0, None)
    rng = np.random.default_rng(7)
    ys = torch.tensor(np.concatenate([rng.integers(0, ny, 32), [0, ny - 1, 0, ny - 1]]))
    if bc_x == "periodic":
        xs = torch.tensor(np.concatenate([rng.integers(0, nx, 32), [0, nx - 1, nx - 1, 0]]))
    else:
        xs = torch.tensor(np.concatenate([rng.integers(4, nx - 4, 32), [4, nx - 5, nx - 5, 4]]))
    got = lam0[:, :, ys.to(DEV), xs.to(DEV)].cpu()
    ref = oracle_adjoint_windows(X, lam1, ys, xs, oracle_cfg(p), s.dt)
    s.close()
    e = rel(got, ref)
    print(f"[adjoint {nx}x{ny} {storage} {bc_x}] sampled lam against the oracle: {e:.2e}", flush=True)
    assert e < 1e-11


@pytest.mark.parametrize("split", (1, 2))
@pytest.mark.parametrize("storage", ("f64", "f32", "f32_dev"))
@pytest.mark.parametrize("bc", (BCS[0], BCS[3]), ids=lambda b: f"{b[0][0]}{b[1][0]}")
def test_step_adjoint_float32_cotangents(split, storage, bc):
    """dvbm_adjoint_step_f32 equals dvbm_adjoint_step on the same (float32)
    lam': the arithmetic is float64 in both, so lam differs by its final
    rounding to float32 only, and d/dtau_ref, d/dPr by summation order at most."""
    wl = smooth_random(117, 17, seed=5)
    p = make_params(wl.nx, wl.ny, dx=wl.dx, dy=wl.dy, split=split, storage=storage, Pr=0.7, tau_ref=0.02,
                    bc_x=bc[0], bc_y=bc[1], dt=3e-3)
    s = Solver(p, wl.rho, wl.ux, wl.uy, wl.T, device=DEV)
    rng = np.random.default_rng(2)
    lam1 = torch.tensor(rng.standard_normal((2, s.Q, wl.ny, wl.nx)), device=DEV).float()
    out = {}
    for dt_ in (torch.float64, torch.float32):
        lam0 = s.new_cotangent(dt_)
        dpar = torch.zeros(2, dtype=torch.float64, device=DEV)
        s.adjoint_step(s.state_buffer, lam1.to(dt_), lam0, dpar)
        torch.cuda.synchronize()
        out[dt_] = (lam0.cpu(), dpar.cpu())
    s.close()
    l64, d64 = out[torch.float64]
    l32, d32 = out[torch.float32]
    assert l32.dtype == torch.float32
    assert torch.equal(l32, l64.float())  # one rounding of the same float64 value
    assert torch.allclose(d32, d64, rtol=1e-14, atol=0.0)


@pytest.mark.parametrize("split", (1, 2))
def test_readout_and_initial_adjoints(split):
    wl = smooth_random(66, 9, seed=12)
    p = make_params(wl.nx, wl.ny, dx=wl.dx, dy=wl.dy, split=split, storage="f64", tau_ref=0.02, dt=1e-3,
                    gamma=1.3)
    s = Solver(p, wl.rho, wl.ux, wl.uy, wl.T, device=DEV)
    cfg = oracle_cfg(p)
    rng = np.random.default_rng(1)
    Tb = torch.tensor(rng.standard_normal((wl.ny, wl.nx)))
    ub = torch.tensor(rng.standard_normal((wl.ny, wl.nx)))
    lam = s.adjoint_moments(s.state_buffer, d_ux=ub, d_T=Tb)
    fields = [torch.tensor(a).requires_grad_() for a in (wl.rho, wl.ux, wl.uy, wl.T)]
    f, g = O.initial_state(*fields, cfg)
    fr, gr = f.detach().clone().requires_grad_(), g.detach().clone().requires_grad_()
    d = O.diagnostics(fr, gr, cfg)
    ((d["T"] * Tb).sum() + (d["ux"] * ub).sum()).backward()
    assert rel(lam.cpu(), torch.stack([fr.grad, gr.grad])) < 1e-12
    lam0 = torch.tensor(rng.standard_normal((2,) + tuple(f.shape)))
    out = s.adjoint_init(lam0.to(DEV), wl.rho, wl.ux, wl.uy, wl.T, which=("rho", "ux", "uy", "T"))
    ((lam0[0] * f).sum() + (lam0[1] * g).sum()).backward()
    for k, fld in zip(("rho", "ux", "uy", "T"), fields):
        assert rel(out[k].cpu(), fld.grad) < 1e-12, k


def smooth_T0(n, seed=9):
    """1 + a few smooth random-phase periodic modes of amplitude ~0.05.

    Random phases keep neighbouring differences from tying exactly; on a
    symmetric field (say sin x cos y sampled at cell centres) equal
    differences put the limiter exactly on its kinks, where the one-sided
    derivatives differ and any two correct adjoints may pick different
    subgradients."""
    return smooth_random(n, n, seed=seed, amp_rho=0.0, amp_u=0.0, amp_T=0.05, mean_u=(0.0, 0.0)).T


def _loss_problem(n=24, nsteps=12, storage="f64", Pr=0.71, split=2):
    bump = gaussian_bump(n, seed=3, amp=0.1, width=0.15)
    T0 = smooth_T0(n)
    zeros = np.zeros((n, n))
    kw = dict(dx=1.0 / n, dy=1.0 / n, split=split, storage=storage, dt=2e-3, gamma=1.4)
    return bump, T0, zeros, kw, nsteps, Pr


def test_rollout_gradient_matches_oracle():
    bump, T0, zeros, kw, nsteps, Pr = _loss_problem()
    n = T0.shape[0]
    # target from the hidden bump, then the gradient at T0
    tgt = rollout_temperature(torch.tensor(bump.T, device=DEV), torch.tensor(0.01, dtype=torch.float64),
                              torch.tensor(Pr, dtype=torch.float64), np.ones((n, n)), zeros, zeros, nsteps, K=5,
                              **kw).detach()
    T0t = torch.tensor(T0, device=DEV, requires_grad=True)
    tau = torch.tensor(0.01, dtype=torch.float64, requires_grad=True)
    prt = torch.tensor(Pr, dtype=torch.float64, requires_grad=True)
    out = rollout_temperature(T0t, tau, prt, np.ones((n, n)), zeros, zeros, nsteps, K=5, **kw)
    ((out - tgt) ** 2).sum().backward()
    # oracle
    cfg = O.Config(nx=n, ny=n, split=2, dx=1.0 / n, dy=1.0 / n, Pr=Pr, tau_ref=0.01)
    T0o = torch.tensor(T0, requires_grad=True)
    tauo = torch.tensor(0.01, dtype=torch.float64, requires_grad=True)
    pro = torch.tensor(Pr, dtype=torch.float64, requires_grad=True)
    f, g = O.initial_state(np.ones((n, n)), zeros, zeros, T0o, cfg)
    f, g = O.run(f, g, cfg, 2e-3, nsteps, tauo, pro)
    To = O.diagnostics(f, g, cfg)["T"]
    assert rel(out.detach().cpu(), To.detach()) < 1e-13
    ((To - tgt.cpu()) ** 2).sum().backward()
    assert rel(T0t.grad.cpu(), T0o.grad) < 1e-10
    assert abs(float(tau.grad) / float(tauo.grad) - 1) < 1e-10
    assert abs(float(prt.grad) / float(pro.grad) - 1) < 1e-10


def test_rollout_float32_cotangents():
    """Gradients with float32 cotangents (12 steps, K = 5) against float64
    cotangents: within 1e-5 relative for T0, tau_ref and Pr."""
    bump, T0, zeros, kw, nsteps, Pr = _loss_problem()
    n = T0.shape[0]
    grads = {}
    for cot in ("f64", "f32"):
        T0t = torch.tensor(T0, device=DEV, requires_grad=True)
        tau = torch.tensor(0.01, dtype=torch.float64, requires_grad=True)
        prt = torch.tensor(Pr, dtype=torch.float64, requires_grad=True)
        out = rollout_temperature(T0t, tau, prt, np.ones((n, n)), zeros, zeros, nsteps, K=5, cotangent=cot, **kw)
        ((out - torch.tensor(bump.T, device=DEV)) ** 2).sum().backward()
        grads[cot] = (T0t.grad.cpu(), float(tau.grad), float(prt.grad))
    assert rel(grads["f32"][0], grads["f64"][0]) < 1e-5
    assert abs(grads["f32"][1] / grads["f64"][1] - 1) < 1e-5
    assert abs(grads["f32"][2] / grads["f64"][2] - 1) < 1e-5


@pytest.mark.parametrize("K", (1, 5, 12, 20))
def test_rollout_overlap_matches_sequential(K):
    """The recomputation on a second stream gives the same gradient, bit for bit,
    as recomputing after each reverse sweep on one stream (12 steps: segments of
    1, of 5, 5 and 2, one segment of 12, and K beyond nsteps)."""
    bump, T0, zeros, kw, nsteps, Pr = _loss_problem()
    n = T0.shape[0]
    grads = []
    for overlap in (False, True):
        T0t = torch.tensor(T0, device=DEV, requires_grad=True)
        tau = torch.tensor(0.01, dtype=torch.float64, requires_grad=True)
        prt = torch.tensor(Pr, dtype=torch.float64, requires_grad=True)
        out = rollout_temperature(T0t, tau, prt, np.ones((n, n)), zeros, zeros, nsteps, K=K, overlap=overlap, **kw)
        ((out - torch.tensor(bump.T, device=DEV)) ** 2).sum().backward()
        torch.cuda.synchronize()
        grads.append((T0t.grad.cpu(), float(tau.grad), float(prt.grad)))
    assert torch.equal(grads[0][0], grads[1][0])
    assert grads[0][1:] == grads[1][1:]


FD_N, FD_STEPS, FD_PR, FD_TAU = 256, 200, 0.71, 2e-3


def _fd_problem(beta=1.2):
    """The 256^2 periodic gradient workload: target temperature from a hidden
    Gaussian bump (amplitude 0.1, width 0.1 L), gradient at T0 = 1 plus a
    smooth mode of amplitude 0.05, 200 float64 steps at dt = 1e-4."""
    n = FD_N
    bump = gaussian_bump(n, seed=7, amp=0.1, width=0.1)
    T0 = smooth_T0(n, seed=13)
    ones, zeros = np.ones((n, n)), np.zeros((n, n))
    kw = dict(dx=1.0 / n, dy=1.0 / n, split=2, storage="f64", dt=1e-4, beta=beta)

    def run(T, tau=FD_TAU, pr=FD_PR, K=10):
        return rollout_temperature(T, torch.tensor(tau, dtype=torch.float64), torch.tensor(pr, dtype=torch.float64),
                                   ones, zeros, zeros, FD_STEPS, K=K, **kw).detach()

    tgt = run(torch.tensor(bump.T, device=DEV))

    def dloss(a, b):  # L(a) - L(b) without cancelling two large sums
        return float(((a - b) * (a + b - 2 * tgt)).sum())

    return T0, ones, zeros, kw, run, tgt, dloss


def _gradient(T0, ones, zeros, kw, tgt, K):
    T0t = torch.tensor(T0, device=DEV, requires_grad=True)
    taut = torch.tensor(FD_TAU, dtype=torch.float64, requires_grad=True)
    prt = torch.tensor(FD_PR, dtype=torch.float64, requires_grad=True)
    out = rollout_temperature(T0t, taut, prt, ones, zeros, zeros, FD_STEPS, K=K, **kw)
    ((out - tgt) ** 2).sum().backward()
    return T0t.grad, taut.grad, prt.grad


def test_rollout_gradient_matches_oracle_256():
    """The gradient workload as specified (256^2 periodic, the hidden-bump
    target, T0 = 1 plus a smooth mode, 200 steps at dt = 1e-4, FP64 storage),
    checkpoints every 10 and every 50 steps: dL/dT0, dL/dtau_ref and dL/dPr
    against reverse mode through the oracle's 200 steps (taken segment by
    segment, 5 steps each, to bound its memory), within 1e-10."""
    n, nsteps = FD_N, FD_STEPS
    bump = gaussian_bump(n, seed=7, amp=0.1, width=0.1)
    T0 = smooth_T0(n, seed=13)
    ones, zeros = np.ones((n, n)), np.zeros((n, n))
    kw = dict(dx=1.0 / n, dy=1.0 / n, split=2, storage="f64", dt=1e-4)
    tgt = rollout_temperature(torch.tensor(bump.T, device=DEV), torch.tensor(FD_TAU, dtype=torch.float64),
                              torch.tensor(FD_PR, dtype=torch.float64), ones, zeros, zeros, nsteps, K=10, **kw).detach()
    grads = {}
    for K in (10, 50):
        T0t = torch.tensor(T0, device=DEV, requires_grad=True)
        taut = torch.tensor(FD_TAU, dtype=torch.float64, requires_grad=True)
        prt = torch.tensor(FD_PR, dtype=torch.float64, requires_grad=True)
        out = rollout_temperature(T0t, taut, prt, ones, zeros, zeros, nsteps, K=K, **kw)
        ((out - tgt) ** 2).sum().backward()
        grads[K] = (T0t.grad.cpu(), float(taut.grad), float(prt.grad))
    # the oracle's reverse mode, segment by segment: the forward keeps the states
    # at segment boundaries, the reverse recomputes one segment at a time with its
    # graph and pushes the cotangents through it, so at most one segment's graph
    # (5 steps, about 12 GB at this size) is alive
    seg = 5
    cfg = O.Config(nx=n, ny=n, split=2, dx=1.0 / n, dy=1.0 / n, Pr=FD_PR, tau_ref=FD_TAU)
    T0o = torch.tensor(T0, requires_grad=True)
    tauo = torch.tensor(FD_TAU, dtype=torch.float64, requires_grad=True)
    pro = torch.tensor(FD_PR, dtype=torch.float64, requires_grad=True)
    f0, g0 = O.initial_state(ones, zeros, zeros, T0o, cfg)
    states = [(f0.detach(), g0.detach())]
    with torch.no_grad():
        for _ in range(nsteps // seg):
            states.append(O.run(*states[-1], cfg, 1e-4, seg, tauo, pro))
    fL, gL = (x.clone().requires_grad_(True) for x in states[-1])
    ((O.diagnostics(fL, gL, cfg)["T"] - tgt.cpu()) ** 2).sum().backward()
    cf, cg = fL.grad, gL.grad
    for k in reversed(range(nsteps // seg)):
        fi, gi = (x.clone().requires_grad_(True) for x in states[k])
        fo, go = O.run(fi, gi, cfg, 1e-4, seg, tauo, pro)
        torch.autograd.backward([fo, go], [cf, cg])
        cf, cg = fi.grad, gi.grad
        del fo, go, fi, gi
        states[k + 1] = None
    torch.autograd.backward([f0, g0], [cf, cg])
    for K, (gT, gtau, gpr) in grads.items():
        e = (rel(gT, T0o.grad), abs(gtau / float(tauo.grad) - 1), abs(gpr / float(pro.grad) - 1))
        print(f"[rollout 256^2, {nsteps} steps, K {K}] against the oracle: T0 {e[0]:.1e}, tau_ref {e[1]:.1e}, "
              f"Pr {e[2]:.1e}", flush=True)
        assert max(e) < 1e-10, (K, e)


@pytest.mark.parametrize("K", (10, 50))
def test_adjoint_vs_central_differences_256(K):
    """256^2 periodic, 200 steps, loss sum (T - T_target)^2: parameter and
    directional derivatives against central FD in float64.  d/dtau_ref and
    d/dPr agree within 1e-6 at h = 1e-6 (measured ~1e-9), and so do
    directional derivatives along smooth fields (measured <= 7e-8).  Point
    derivatives follow the protocol of test_point_derivatives_32_points.  The
    exact statement, that the adjoint is the reverse-mode derivative of the
    discrete map, is test_rollout_gradient_matches_oracle (1e-10)."""
    n = FD_N
    T0, ones, zeros, kw, run, tgt, dloss = _fd_problem()
    g_T0, g_tau, g_pr = _gradient(T0, ones, zeros, kw, tgt, K)
    T0d = torch.tensor(T0, device=DEV)
    h = 1e-6
    fd_tau = dloss(run(T0d, FD_TAU * (1 + h)), run(T0d, FD_TAU * (1 - h))) / (2 * h * FD_TAU)
    fd_pr = dloss(run(T0d, FD_TAU, FD_PR * (1 + h)), run(T0d, FD_TAU, FD_PR * (1 - h))) / (2 * h * FD_PR)
    print("dL/dtau adjoint %.8e FD %.8e; dL/dPr adjoint %.8e FD %.8e" % (float(g_tau), fd_tau, float(g_pr), fd_pr))
    assert abs(fd_tau - float(g_tau)) <= 1e-6 * abs(fd_tau)
    assert abs(fd_pr - float(g_pr)) <= 1e-6 * abs(fd_pr)
    for seed in (21, 22, 23):
        v = torch.tensor(smooth_random(n, n, seed=seed, amp_rho=0.0, amp_u=0.0, amp_T=1.0, mean_u=(0.0, 0.0)).T - 1.0,
                         device=DEV)
        ad = float((g_T0 * v).sum())
        fd = dloss(run(T0d + h * v), run(T0d - h * v)) / (2 * h)
        print("direction %d: adjoint %.10e FD %.10e" % (seed, ad, fd))
        assert abs(fd - ad) <= 1e-6 * abs(ad)


def _signed_trajectory(p, T0, ones, zeros):
    """Final temperature of a float64 run from the equilibrium of (1, 0, T0),
    and the limiter-branch signature of each of its steps."""
    s = Solver(p, ones, zeros, zeros, T0, device=DEV)
    sig = torch.zeros(FD_STEPS, dtype=torch.int64, device=DEV)
    for k in range(FD_STEPS):
        s.limiter_signature(s.state_buffer, sig[k:k + 1])
        s.step(1)
    T = s.moments(fields=True, sums=False)["T"]
    s.close()
    return T, sig.cpu()


def test_point_derivatives_32_points():
    """dL/dT0 at 32 seeded cells against central differences in float64.

    A central difference is the derivative (to O(h^2)) only while the runs
    from T0 + h and T0 - h take the same limiter branch at every face of every
    step; across a kink of the limiter (r = 0, or a change of the smallest of
    beta r, (1 + r)/2, beta) it is a secant.  Each pair of runs therefore
    records the limiter-branch signature of every step
    (dvbm_limiter_signature).

    At the workload's h = 1e-4 (about a tenth of the neighbour differences at
    this resolution) every point's two runs differ in branch at some face in
    most of the 200 steps (measured at all 32 points; with beta = 2 as well),
    so h = 1e-4 measures secants: their difference from the adjoint is
    reported and bounded by 2e-3 of the largest gradient component (measured
    at most 7e-4).  For each point the step is then divided by 10 until the
    two runs agree in branch at every face of every step (h >= 1e-8); there
    the difference is the derivative's up to O(h^2) and the float64 rounding
    of T(+h) - T(-h), about 1e-8 of the gradient's scale at h = 1e-8: it must
    lie within 1e-6 of the largest gradient component, and within 1e-6 of the
    point's own component where h = 1e-7 already keeps every branch (measured
    1.4e-7 to 3.5e-7; at h = 1e-8 rounding alone gives up to 3e-6 of small
    components).  The gradients with checkpoint intervals 10 and 50 are
    identical."""
    n = FD_N
    T0, ones, zeros, kw, run, tgt, dloss = _fd_problem()
    g10 = _gradient(T0, ones, zeros, kw, tgt, 10)
    g50 = _gradient(T0, ones, zeros, kw, tgt, 50)
    assert torch.equal(g10[0], g50[0]) and torch.equal(g10[1], g50[1]) and torch.equal(g10[2], g50[2])
    grad = g10[0].cpu().numpy()
    gmax = float(np.abs(grad).max())
    p = make_params(n, n, tau_ref=FD_TAU, Pr=FD_PR, **kw)
    rng = np.random.default_rng(5)
    pts = rng.choice(n * n, size=32, replace=False)
    secant, stable, unresolved = [], [], []
    for idx in pts:
        yy, xx = divmod(int(idx), n)
        g = grad[yy, xx]
        for h in (1e-4, 1e-5, 1e-6, 1e-7, 1e-8):
            Tp, Tm = T0.copy(), T0.copy()
            Tp[yy, xx] += h
            Tm[yy, xx] -= h
            Tpl, sp = _signed_trajectory(p, Tp, ones, zeros)
            Tmi, sm = _signed_trajectory(p, Tm, ones, zeros)
            fd = dloss(Tpl, Tmi) / (2 * h)
            err = abs(fd - g) / abs(g)
            flips = int((sp != sm).sum())
            print("point (%3d, %3d) h %.0e: adjoint %+.10e FD %+.10e rel err %.2e, steps with a branch change %d"
                  % (yy, xx, h, g, fd, err, flips), flush=True)
            if h == 1e-4 and flips:
                secant.append(abs(fd - g) / gmax)
            if flips == 0:
                stable.append((h, err, abs(fd - g) / gmax))
                break
        else:
            unresolved.append((yy, xx))
    print("h = 1e-4: %d of 32 points change branch; secant differences / max |gradient|: median %.2e max %.2e"
          % (len(secant), float(np.median(secant)) if secant else 0.0, max(secant, default=0.0)))
    print("branch-stable at some h >= 1e-8: %d points, h used %s, max difference / max |gradient| %.2e, max rel err "
          "%.2e (h = 1e-7: %.2e); unresolved %d"
          % (len(stable), sorted({h for h, _, _ in stable}), max((a for _, _, a in stable), default=0.0),
             max((e for _, e, _ in stable), default=0.0),
             max((e for h, e, _ in stable if h >= 1e-7), default=0.0), len(unresolved)))
    assert all(a <= 2e-3 for a in secant)
    assert all(a <= 1e-6 for _, _, a in stable)
    assert all(e <= 1e-6 for h, e, _ in stable if h >= 1e-7)
    assert len(stable) >= 24


def _mix64(z):
    """SplitMix64 output function on numpy uint64 (wrapping arithmetic)."""
    z = z + np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def _branch_ratio_form(a, b, beta):
    """Branch of phi(r) = max(0, min(beta r, (1 + r)/2, beta)), r = a/b (Sec. III A 2), in
    the paper's ratio form: 0 when phi = 0, else 1, 2, 3 for the smallest of the three."""
    out = np.zeros(a.shape, dtype=np.uint64)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = a / b
    live = (b != 0) & (r > 0)
    c = np.stack([beta * r, (1 + r) / 2, np.full_like(r, beta)])
    out[live] = (np.argmin(c, axis=0)[live] + 1).astype(np.uint64)
    return out


@pytest.mark.parametrize("split", (1, 2))
@pytest.mark.parametrize("bc", (("periodic", "periodic"), ("zero_gradient", "periodic"), ("periodic", "zero_gradient")),
                         ids=lambda b: f"{b[0][0]}{b[1][0]}")
def test_limiter_signature_matches_branch_rule(split, bc):
    """dvbm_limiter_signature equals, bit for bit, the sum over faces of the
    SplitMix64 mix of (face, branch) with the branches taken from the ratio
    form of phi on the host, on a random off-equilibrium state (every branch
    occurs); a second call adds the same value again."""
    wl = smooth_random(13, 9, seed=31)
    p = make_params(wl.nx, wl.ny, dx=wl.dx, dy=wl.dy, split=split, storage="f64", tau_ref=0.02, dt=1e-3,
                    bc_x=bc[0], bc_y=bc[1], beta=1.3)
    s = Solver(p, wl.rho, wl.ux, wl.uy, wl.T, device=DEV)
    rng = np.random.default_rng(split)
    X = s.store_populations().cpu().numpy()
    X = X * (1 + 0.2 * rng.standard_normal(X.shape))
    s.load_populations(torch.tensor(X))
    sig = torch.zeros(1, dtype=torch.int64, device=DEV)
    s.limiter_signature(s.state_buffer, sig)
    torch.cuda.synchronize()
    one = int(sig.item())
    s.limiter_signature(s.state_buffer, sig)
    torch.cuda.synchronize()
    two = int(sig.item())
    s.close()
    v = O.velocity_set(O.Config(nx=wl.nx, ny=wl.ny, split=split))[0].numpy()
    Q, ny, nx = X.shape[1], X.shape[2], X.shape[3]
    n = nx * ny
    total = np.zeros(1, dtype=np.uint64)  # arrays wrap silently modulo 2^64
    counts = np.zeros(4, dtype=np.int64)
    for ax in (0, 1):
        axis = 1 - ax  # of a [ny, nx] plane: x is axis 1, y axis 0
        for pl in range(2 * Q):
            vel = v[pl % Q, ax]
            if vel == 0:
                continue
            P = X[pl // Q, pl % Q]

            def sh(d):  # value at cell + d along the axis under the boundary rule
                m = P.shape[axis]
                idx = np.arange(m) + d
                idx = idx % m if bc[ax] == "periodic" else np.clip(idx, 0, m - 1)
                return np.take(P, idx, axis=axis)

            a = sh(0) - sh(-1) if vel > 0 else sh(1) - sh(2)
            b = sh(1) - sh(0) if vel > 0 else sh(0) - sh(1)
            br = _branch_ratio_form(a, b, 1.3)
            counts += np.bincount(br.ravel().astype(np.int64), minlength=4)
            face = (np.uint64((ax * 2 * Q + pl) * n) + np.arange(n, dtype=np.uint64)).reshape(ny, nx)
            total += _mix64(np.uint64(4) * face + br).sum(dtype=np.uint64)
    assert (counts > 0).all(), counts
    assert one == int(total.view(np.int64)[0])
    assert two == int((total * np.uint64(2)).view(np.int64)[0])


def test_fp32_adjoint_close_to_fp64():
    """Gradient of float32-storage rollouts (f32 and f32_dev) against the float64 one.

    Both adjoints are exact for their own trajectories (the step adjoint at a
    float32 state matches the oracle to 1e-11); they differ because the
    trajectories differ by float32 rounding and, near limiter kinks, that
    rounding can select a different limiter branch, which changes the local
    derivative by O(1) (f32 measured 1.5e-3 relative L2).  The bound 5e-3
    records that sensitivity for both storages."""
    bump, T0, zeros, kw, nsteps, Pr = _loss_problem(n=64, nsteps=40)
    n = T0.shape[0]
    grads = {}
    for st in ("f64", "f32", "f32_dev"):
        kw2 = dict(kw, storage=st)
        tgt = rollout_temperature(torch.tensor(bump.T, device=DEV), torch.tensor(0.01, dtype=torch.float64),
                                  torch.tensor(Pr, dtype=torch.float64), np.ones((n, n)), zeros, zeros, nsteps,
                                  K=10, **kw2).detach()
        T0t = torch.tensor(T0, device=DEV, requires_grad=True)
        out = rollout_temperature(T0t, torch.tensor(0.01, dtype=torch.float64), torch.tensor(Pr, dtype=torch.float64),
                                  np.ones((n, n)), zeros, zeros, nsteps, K=10, **kw2)
        ((out - tgt) ** 2).sum().backward()
        grads[st] = T0t.grad.cpu()
    for st in ("f32", "f32_dev"):
        print("%s storage: gradient relative L2 against float64 storage %.2e" % (st, rel(grads[st], grads["f64"])))
        assert rel(grads[st], grads["f64"]) < 5e-3


@pytest.mark.parametrize("storage", ("f64", "f32_dev"))
def test_binding_refuses_short_or_strided_tensors(storage):
    """The binding checks every tensor before the library sees its pointer: a short population buffer,
    a cotangent of the wrong shape, dtype or layout, and a host tensor are refused, and the refused
    calls leave the state and the good cotangent untouched."""
    print(f"[binding checks] {storage}", flush=True)
    wl = smooth_random(20, 12, seed=3)
    p = make_params(wl.nx, wl.ny, dx=wl.dx, dy=wl.dy, split=2, storage=storage, tau_ref=0.02, dt=3e-3)
    s = Solver(p, wl.rho, wl.ux, wl.uy, wl.T, device=DEV)
    state = s.state_buffer
    before = state.clone()
    good = s.new_cotangent()
    lam1 = torch.ones_like(good)
    with pytest.raises(ValueError, match="fewer"):
        s.step_from(state, torch.empty(state.numel() - 1, dtype=torch.uint8, device=DEV))
    with pytest.raises(ValueError, match="fewer"):
        s.adjoint_step(state[:-8], lam1, good)
    with pytest.raises(ValueError, match="shape"):
        s.adjoint_step(state, lam1[:, :, :-1].contiguous(), good[:, :, :-1].contiguous())
    with pytest.raises(ValueError, match="contiguous"):
        s.adjoint_step(state, lam1, good.transpose(2, 3))
    with pytest.raises(TypeError):
        s.adjoint_step(state, lam1, good, torch.zeros(2, dtype=torch.float32, device=DEV))
    with pytest.raises(ValueError, match="must be on"):
        s.adjoint_step(state, lam1.cpu(), good.cpu())
    with pytest.raises(ValueError, match="shape"):
        s.adjoint_moments(state, d_T=torch.ones(p.ny, p.nx + 1, dtype=torch.float64, device=DEV))
    torch.cuda.synchronize()
    assert torch.equal(state, before)
    assert not torch.any(good)
    s.adjoint_step(state, lam1, good)
    torch.cuda.synchronize()
    assert torch.isfinite(good).all() and torch.any(good)
