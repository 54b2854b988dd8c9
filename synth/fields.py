"""Seeded macroscopic initial conditions for the benchmark workloads.

Every generator returns a :class:`Workload`: cell-centred float64 fields of
shape ``(ny, nx)`` (row ``y``, column ``x``) plus the domain size and the
physical parameters the workload is defined with. Cell ``(j, i)`` has its
centre at ``((i + 1/2) dx, (j + 1/2) dy)``.

Units follow the paper's simulation parameters (Sec. III A 3): ``R = 1``,
lattice reference temperature ``T_ref = 1``, ``gamma = 1.4`` and
``mu = 5e-5`` unless a workload says otherwise.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    T: np.ndarray
    Lx: float
    Ly: float
    phys: dict = field(default_factory=dict)

    @property
    def ny(self) -> int:
        return self.rho.shape[0]

    @property
    def nx(self) -> int:
        return self.rho.shape[1]

    @property
    def dx(self) -> float:
        return self.Lx / self.nx

    @property
    def dy(self) -> float:
        return self.Ly / self.ny


def _centres(n: int, L: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) * (L / n)


def _grid(nx: int, ny: int, Lx: float, Ly: float):
    x = _centres(nx, Lx)
    y = _centres(ny, Ly)
    return np.meshgrid(x, y)  # X[j, i] = x_i, Y[j, i] = y_j


def uniform(nx: int, ny: int, rho=1.0, ux=0.0, uy=0.0, T=1.0, L=1.0) -> Workload:
    """Uniform state (a fixed point of the full update on a periodic grid)."""
    shape = (ny, nx)
    return Workload(
        "uniform",
        np.full(shape, float(rho)),
        np.full(shape, float(ux)),
        np.full(shape, float(uy)),
        np.full(shape, float(T)),
        L,
        L * ny / nx,
    )


def shear_wave(n: int = 64, ny: int | None = None, amp: float = 1e-3, mach: float = 0.1,
               gamma: float = 1.4, R: float = 1.0, T0: float = 1.0, rho0: float = 1.0,
               L: float = 1.0) -> Workload:
    """Plane shear wave of the shear-viscosity test (Sec. III D 1).

    ``u_y = A sin(2 pi x / L)`` on a uniform state moving with
    ``u_x = Ma sqrt(gamma R T0)``.
    """
    ny = n if ny is None else ny
    X, _ = _grid(n, ny, L, L * ny / n)
    rho = np.full_like(X, rho0)
    T = np.full_like(X, T0)
    ux = np.full_like(X, mach * np.sqrt(gamma * R * T0))
    uy = amp * np.sin(2.0 * np.pi * X / L)
    return Workload("shear_wave", rho, ux, uy, T, L, L * ny / n,
                    {"gamma": gamma, "R": R, "amp": amp, "mach": mach})


def thermal_wave_1d(n: int = 64, ny: int = 4, amp: float = 1e-3, mach: float = 0.0,
                    gamma: float = 1.4, R: float = 1.0, T0: float = 1.0, rho0: float = 1.0,
                    L: float = 1.0) -> Workload:
    """Isobaric density/temperature wave of the thermal-diffusivity test (Sec. III D 3)."""
    X, _ = _grid(n, ny, L, L * ny / n)
    rho = rho0 + amp * np.sin(2.0 * np.pi * X / L)
    T = rho0 * T0 / rho
    ux = np.full_like(X, mach * np.sqrt(gamma * R * T0))
    uy = np.zeros_like(X)
    return Workload("thermal_wave_1d", rho, ux, uy, T, L, L * ny / n,
                    {"gamma": gamma, "R": R, "amp": amp, "mach": mach})


def _vortex_perturbation(X, Y, xv, yv, rv, Lx, Ly, periodic_x, periodic_y):
    dx = X - xv
    dy = Y - yv
    if periodic_x:
        dx = dx - Lx * np.round(dx / Lx)
    if periodic_y:
        dy = dy - Ly * np.round(dy / Ly)
    r2 = (dx * dx + dy * dy) / (rv * rv)
    return dx, dy, r2


def isentropic_vortex(n: int = 1024, seed: int = 0, mach_adv: float = 1.0, mach_v: float = 0.3,
                      r_frac: float = 0.05, gamma: float = 1.4, R: float = 1.0,
                      L: float = 1.0) -> Workload:
    """Isentropic vortex (the vortex of Sec. III F) carried by a uniform stream.

    Free stream ``rho = p = 1``, ``u = (Ma_adv c, 0)`` with ``c = sqrt(gamma)``;
    vortex of Mach number ``mach_v`` and radius ``r_frac L`` centred at a
    seeded uniform point, distances taken as minimum images on the periodic
    domain.
    """
    rng = np.random.default_rng(seed)
    xv, yv = rng.uniform(0.0, L, size=2)
    X, Y = _grid(n, n, L, L)
    rho_inf, p_inf = 1.0, 1.0
    c = np.sqrt(gamma * p_inf / rho_inf)
    rv = r_frac * L
    dx, dy, r2 = _vortex_perturbation(X, Y, xv, yv, rv, L, L, True, True)
    e_half = np.exp(0.5 * (1.0 - r2))
    ux = mach_adv * c + c * mach_v * (dy / rv) * e_half
    uy = -c * mach_v * (dx / rv) * e_half
    base = 1.0 - 0.5 * (gamma - 1.0) * mach_v ** 2 * np.exp(1.0 - r2)
    rho = rho_inf * base ** (1.0 / (gamma - 1.0))
    p = p_inf * base ** (gamma / (gamma - 1.0))
    T = p / (rho * R)
    return Workload("isentropic_vortex", rho, ux, uy, T, L, L,
                    {"gamma": gamma, "R": R, "centre": (float(xv), float(yv)), "rv": rv})


def rankine_hugoniot(rho_l: float, p_l: float, mach_s: float, gamma: float):
    """Post-shock state of a stationary normal shock (Sec. III F)."""
    c_l = np.sqrt(gamma * p_l / rho_l)
    u_l = mach_s * c_l
    m2 = mach_s * mach_s
    rho_r = rho_l * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p_r = p_l * (2.0 * gamma * m2 - (gamma - 1.0)) / (gamma + 1.0)
    u_r = u_l * ((gamma - 1.0) * m2 + 2.0) / ((gamma + 1.0) * m2)
    return (rho_l, p_l, u_l), (rho_r, p_r, u_r)


def shock_vortex(nx: int = 2048, ny: int = 1024, mach_s: float = 1.2, mach_v: float = 0.25,
                 r_frac: float = 0.075, gamma: float = 1.4, R: float = 1.0, Re_v: float = 800.0,
                 Lx: float = 2.0, Ly: float = 1.0, x_shock: float | None = None) -> Workload:
    """Stationary normal shock hit by an isentropic vortex (Sec. III F).

    Pre-shock ``rho = p = 1`` for ``x < x_shock`` (default ``Lx/2``),
    Rankine-Hugoniot post-shock state beyond. The vortex of radius
    ``r_frac Ly`` sits upstream at ``(x_shock - 2 r_v, Ly/2)`` (the paper's
    spacing of two radii between the vortex centre and the shock) and
    perturbs both sides. The dynamic viscosity follows from
    ``Re_v = rho_l c_l r_v / mu``. The paper's case C is
    ``shock_vortex(1680, 1440, 1.2, 0.25, 1/24, Lx=28, Ly=24, x_shock=8)``.
    """
    (rho_l, p_l, u_l), (rho_r, p_r, u_r) = rankine_hugoniot(1.0, 1.0, mach_s, gamma)
    X, Y = _grid(nx, ny, Lx, Ly)
    xs = 0.5 * Lx if x_shock is None else float(x_shock)
    left = X < xs
    rho_inf = np.where(left, rho_l, rho_r)
    p_inf = np.where(left, p_l, p_r)
    u_inf = np.where(left, u_l, u_r)
    c_l = np.sqrt(gamma * p_l / rho_l)
    rv = r_frac * Ly
    xv, yv = xs - 2.0 * rv, 0.5 * Ly
    dx, dy, r2 = _vortex_perturbation(X, Y, xv, yv, rv, Lx, Ly, False, True)
    e_half = np.exp(0.5 * (1.0 - r2))
    ux = u_inf + c_l * mach_v * (dy / rv) * e_half
    uy = -c_l * mach_v * (dx / rv) * e_half
    base = 1.0 - 0.5 * (gamma - 1.0) * mach_v ** 2 * np.exp(1.0 - r2)
    rho = rho_inf * base ** (1.0 / (gamma - 1.0))
    p = p_inf * base ** (gamma / (gamma - 1.0))
    T = p / (rho * R)
    mu = rho_l * c_l * rv / Re_v
    return Workload("shock_vortex", rho, ux, uy, T, Lx, Ly,
                    {"gamma": gamma, "R": R, "mu": mu, "rv": rv, "p_post": p_r, "c_l": float(c_l),
                     "T_post": p_r / (rho_r * R), "u_post": u_r, "centre": (xv, yv),
                     "mach_s": mach_s, "mach_v": mach_v})


def thermal_wave(n: int = 4096, seed: int = 0, amp: float = 0.05, sigma: float = 1e-3,
                 n_modes: int = 8, kmax: int = 4, L: float = 1.0) -> Workload:
    """Isobaric thermal wave with a seeded random velocity perturbation.

    ``T = 1 + amp sin(2 pi y / L)``, ``rho = 1 / T``; each velocity component
    is a sum of ``n_modes`` Fourier modes with amplitudes ``N(0, sigma^2)``,
    integer wave-vector components in ``[-kmax, kmax] \\ {0}`` and phases
    ``U[0, 2 pi)``, drawn independently per component.
    """
    rng = np.random.default_rng(seed)
    X, Y = _grid(n, n, L, L)
    T = 1.0 + amp * np.sin(2.0 * np.pi * Y / L)
    rho = 1.0 / T
    nonzero = np.array([k for k in range(-kmax, kmax + 1) if k != 0])
    comps = []
    for _ in range(2):
        u = np.zeros_like(X)
        A = rng.normal(0.0, sigma, size=n_modes)
        kx = rng.choice(nonzero, size=n_modes)
        ky = rng.choice(nonzero, size=n_modes)
        ph = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
        for m in range(n_modes):
            u += A[m] * np.sin(2.0 * np.pi * (kx[m] * X + ky[m] * Y) / L + ph[m])
        comps.append(u)
    return Workload("thermal_wave", rho, comps[0], comps[1], T, L, L, {"amp": amp})


def gaussian_bump(n: int = 256, seed: int = 0, amp: float = 0.1, width: float = 0.1,
                  L: float = 1.0) -> Workload:
    """Gaussian temperature bump at rest on a periodic square (minimum images)."""
    rng = np.random.default_rng(seed)
    xc, yc = rng.uniform(0.0, L, size=2)
    X, Y = _grid(n, n, L, L)
    dx, dy, _ = _vortex_perturbation(X, Y, xc, yc, 1.0, L, L, True, True)
    T = 1.0 + amp * np.exp(-(dx * dx + dy * dy) / (2.0 * (width * L) ** 2))
    rho = np.ones_like(T)
    z = np.zeros_like(T)
    return Workload("gaussian_bump", rho, z.copy(), z.copy(), T, L, L,
                    {"centre": (float(xc), float(yc))})


def smooth_random(nx: int, ny: int, seed: int = 0, amp_rho: float = 0.05, amp_u: float = 0.1,
                  amp_T: float = 0.05, mean_u=(0.1, -0.05), n_modes: int = 3,
                  L: float = 1.0) -> Workload:
    """Random smooth periodic fields (a few low Fourier modes) for parity checks."""
    rng = np.random.default_rng(seed)
    Ly = L * ny / nx
    X, Y = _grid(nx, ny, L, Ly)

    def field_(scale):
        out = np.zeros_like(X)
        for _ in range(n_modes):
            kx, ky = rng.integers(-3, 4, size=2)
            ph = rng.uniform(0, 2 * np.pi)
            out += rng.normal(0.0, scale) * np.sin(2 * np.pi * (kx * X / L + ky * Y / Ly) + ph)
        return out

    rho = 1.0 + field_(amp_rho)
    ux = mean_u[0] + field_(amp_u)
    uy = mean_u[1] + field_(amp_u)
    T = 1.0 + field_(amp_T)
    return Workload("smooth_random", rho, ux, uy, T, L, Ly, {})


def sod_tube(nx: int = 1024, ny: int = 4, R: float = 1.0) -> Workload:
    """Sod shock tube (Sec. IV, conservation): (rho, p, u_x) = (1, 1, 0) for
    0 <= x <= 0.5 and (0.125, 0.1, 0) for 0.5 < x <= 1, on the extended
    periodic domain x in [-0.5, 1.5] (each state continued by 0.5 on its own
    side, so the second interface, at the periodic seam, stays 0.5 away from
    [0, 1]); nx cells over the length 2, T = p / (rho R)."""
    x = _centres(nx, 2.0) - 0.5
    left = x <= 0.5
    rho1 = np.where(left, 1.0, 0.125)
    p1 = np.where(left, 1.0, 0.1)
    rho = np.repeat(rho1[None, :], ny, 0)
    T = np.repeat((p1 / (rho1 * R))[None, :], ny, 0)
    zero = np.zeros((ny, nx))
    return Workload("sod_tube", rho, zero.copy(), zero.copy(), T, 2.0, 2.0 * ny / nx)


def acoustic_wave(n: int = 256, ny: int = 4, amp: float = 1e-3, theta: float = 1.0, mach: float = 0.0,
                  gamma: float = 1.4, R: float = 1.0) -> Workload:
    """Adiabatic standing sound wave on a periodic unit line (pseudo-1-D):
    rho = 1 + amp cos(2 pi x), T = theta (1 + (gamma - 1) amp cos(2 pi x)),
    on a uniform flow u_x = mach sqrt(gamma R theta)."""
    x = _centres(n, 1.0)
    c = np.cos(2 * np.pi * x)
    rho = np.repeat((1.0 + amp * c)[None, :], ny, 0)
    T = np.repeat((theta * (1.0 + (gamma - 1.0) * amp * c))[None, :], ny, 0)
    ux = np.full((ny, n), mach * np.sqrt(gamma * R * theta))
    return Workload("acoustic_wave", rho, ux, np.zeros((ny, n)), T, 1.0, ny / n,
                    {"theta": theta, "mach": mach, "amp": amp})
