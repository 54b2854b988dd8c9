"""Plain FP64 CPU oracle of the double-distribution quasi-equilibrium DVBM step.

TEST INFRASTRUCTURE ONLY. This module is imported by ``tests/``, by the
smoke check of ``__graft_entry__`` and by the CPU-baseline leg of
``bench.py``; the product (the HIP library and its Python binding) never
imports, calls or links it, and it imports nothing from the product.

It computes, in float64 with plain PyTorch CPU tensor operations, one time
step of Eq. (finalDiscretePDE) of Strassle, Hosseini & Karlin (arXiv
2510.04197): the two-time quasi-equilibrium BGK relaxation of the mass /
momentum distribution ``f`` and the energy distribution ``g`` towards
Grad-Hermite equilibria and quasi-equilibria, plus the finite-volume NND
flux with the generalised van Leer limiter, integrated with forward Euler.

Everything is written the long way, the way the paper states it:

* moments are full symmetric tensors ``M_n = sum_i v_i (x) ... (x) v_i X_i``;
* equilibrium moment sets are the Maxwell-Boltzmann moments of App. A;
* quasi-equilibrium moment sets are the rows of Table I (SummaryOfPopulations);
* Hermite coefficients come from the recursion of App. D, Hermite tensors
  from the explicit polynomials of App. D, and populations from the full
  tensor contraction of Eq. (Grad-Hermite-expansion-static);
* the face values follow the NND + limiter formulas of Sec. III A 2.

Readings taken where the paper is silent or garbled (each is listed in the
design notes):

* D2Q25 weights: the printed factors ``7 +- 2 sqrt 10`` need the ``1/60``
  normalisation of the 5-point Gauss-Hermite rule (App. G, Table III).
* The third-order QE moment ``2 u (x) A`` (Table I, split II) is taken as the
  symmetric tensor ``S(u, A) = [u A]_cyc - tr(A)/(D+2) [u delta]_cyc``,
  whose contraction ``S_abb = 2 (A u)_a`` is what the heat-flux constraints
  Eqs. (QE_Pr<1_quasiconserved) / (QE_Pr>1_conserved) require.
* Every QE population is a new Grad expansion of its full moment set
  (Sec. II D 4), so a changed second moment also changes ``a_4``.
* ``Pr == 1`` has no quasi-conserved field (Table I: ``f* = f^eq``,
  ``g* = g^eq``); the relaxation times use the ``Pr <= 1`` assignment, and
  both assignments coincide there.
* The limiter term ``(b/2) phi(a, b)`` is zero when ``b == 0``; ``v = 0``
  takes the ``v >= 0`` face formula (its flux is zero either way).
* ``dt`` is evaluated once from the initial fields (Sec. III A 3).
* Zero-gradient ("von Neumann") boundaries copy the nearest interior
  populations into two ghost layers.
* ``CONST_MU`` (the paper's fixed dynamic viscosity, Sec. III A 3) gives a
  per-node ``tau_nu = mu / p``; ``CONST_TAU`` keeps ``tau_nu`` fixed.
* No-slip walls (the thermal Couette case, Sec. IV): the wall lies on the
  face below row 0 (above row ny-1); the two ghost rows mirror the first two
  interior rows, ghost ``k`` (k = 1, 2 away from the wall) taking the fields
  ``rho_G = rho_B, u_G = 2 u_W - u_B, T_G = 2 T_W - T_B`` of interior row
  ``k`` and the populations ``X^eq(G) + (X_B - X^eq(B))``.
* Split II with ``Pr > 1``: the QE pressure tensor of f* is taken as printed
  in the discrete form (Sec. II D), with the trace of ``P_f - P_eq`` removed
  for energy conservation.  The trace then relaxes in the first stage, so the
  bulk viscosity follows ``tau_1`` (the thermal time), not the ``tau_2`` that
  the Chapman-Enskog result (Eq. visc_bluk_2) names.  Split I keeps the trace
  in f* and follows ``tau_2``.  The sound-attenuation pins measure this.
"""

from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import torch

DT = torch.float64
D = 2  # physical dimension

PERIODIC = "periodic"
ZERO_GRADIENT = "zero_gradient"
WALL = "wall"  # y only: no-slip wall with a given temperature and x velocity
CONST_MU = "const_mu"
CONST_TAU = "const_tau"


# --------------------------------------------------------------------------
# Configuration
# --------------------------------------------------------------------------
@dataclass
class Config:
    """Parameters of one simulation (names follow Sec. III A 3)."""

    nx: int
    ny: int
    split: int = 2            # 1: total-energy split (D2Q16); 2: internal non-translational (D2Q25)
    bc_x: str = PERIODIC
    bc_y: str = PERIODIC
    visc_mode: str = CONST_MU
    dx: float = 1.0
    dy: float = 1.0
    R: float = 1.0
    gamma: float = 1.4
    Pr: float = 0.71
    tau_ref: float = 5e-5     # CONST_TAU: tau_nu; CONST_MU: mu = tau_ref * p_ref
    p_ref: float = 1.0
    T_ref: float = 1.0
    beta: float = 1.2
    cfl: float = 0.01
    dt: float = 0.0           # > 0: a fixed time step in place of the CFL rule
    wall_T: tuple = (1.0, 1.0)    # bc_y == WALL: temperatures of the lower and upper wall
    wall_ux: tuple = (0.0, 0.0)   # bc_y == WALL: x velocities of the lower and upper wall

    @property
    def Cv(self) -> float:
        return self.R / (self.gamma - 1.0)

    @property
    def N_f(self) -> int:
        """Grad expansion order of f (Sec. II D 3 and App. E)."""
        return 3 if self.split == 1 else 4

    @property
    def q1d(self) -> int:
        """Gauss-Hermite points per direction (Sec. II D 3: D2Q16 for I, D2Q25 for II)."""
        return 4 if self.split == 1 else 5


N_G = 2  # Grad expansion order of g, both splits (Sec. II D 3 and App. E)


# --------------------------------------------------------------------------
# Velocity sets: App. G (Tables II and III)
# --------------------------------------------------------------------------
def gauss_hermite_1d(n_points: int):
    """Probabilists' Gauss-Hermite nodes and weights (App. G), ascending nodes."""
    if n_points == 4:
        s6 = math.sqrt(6.0)
        a, b = math.sqrt(3.0 - s6), math.sqrt(3.0 + s6)
        wa, wb = (3.0 + s6) / 12.0, (3.0 - s6) / 12.0
        xi = [-b, -a, a, b]
        w = [wb, wa, wa, wb]
    elif n_points == 5:
        s10 = math.sqrt(10.0)
        a, b = math.sqrt(5.0 - s10), math.sqrt(5.0 + s10)
        wa, wb = (7.0 + 2.0 * s10) / 60.0, (7.0 - 2.0 * s10) / 60.0
        xi = [-b, -a, 0.0, a, b]
        w = [wb, wa, 8.0 / 15.0, wa, wb]
    else:
        raise ValueError("only the 4- and 5-point rules of App. G are defined")
    return torch.tensor(xi, dtype=DT), torch.tensor(w, dtype=DT)


def velocity_set(cfg: Config):
    """Tensor-product D2Q16 / D2Q25 set; population ``i = a * q1d + b``.

    ``v_i = sqrt(R T_ref) (xi_a, xi_b)`` and ``w_i = w_a w_b`` (App. G).
    Returns ``v`` of shape ``[Q, 2]`` and ``w`` of shape ``[Q]``.
    """
    xi, w1 = gauss_hermite_1d(cfg.q1d)
    c = math.sqrt(cfg.R * cfg.T_ref)
    vx = xi.repeat_interleave(len(xi))
    vy = xi.repeat(len(xi))
    wx = w1.repeat_interleave(len(xi))
    wy = w1.repeat(len(xi))
    return c * torch.stack([vx, vy], dim=1), wx * wy


# --------------------------------------------------------------------------
# Symmetric tensor helpers (index notation of App. A / App. D)
# --------------------------------------------------------------------------
_LET = "abcdefgh"


def delta() -> torch.Tensor:
    return torch.eye(D, dtype=DT)


def outer_power(v: torch.Tensor, n: int) -> torch.Tensor:
    """``v (x) ... (x) v`` (n factors) over trailing dim of ``v`` ([..., D])."""
    out = torch.ones(v.shape[:-1], dtype=v.dtype)
    for k in range(n):
        out = out[..., None] * v.reshape(v.shape[:-1] + (1,) * k + (D,))
    return out


def sym_delta(T: torch.Tensor, k: int) -> torch.Tensor:
    """``[T delta]_cyc``: distinct placements of one Kronecker delta.

    ``T`` is a symmetric rank-``k`` tensor over the trailing ``k`` dims; the
    result has rank ``k + 2`` and is the sum over the ``C(k+2, 2)`` choices of
    the two index positions carried by the delta (3 terms for ``[u delta]``,
    6 for ``[u u delta]`` and ``[a_2 delta]``).
    """
    n = k + 2
    eye = delta()
    out = None
    for p, q in itertools.combinations(range(n), 2):
        rest = [i for i in range(n) if i not in (p, q)]
        spec = "..." + "".join(_LET[i] for i in rest) + "," + _LET[p] + _LET[q] + "->..." + _LET[:n]
        term = torch.einsum(spec, T, eye)
        out = term if out is None else out + term
    return out


def delta_delta() -> torch.Tensor:
    """``[delta delta]_cyc``: the three pairings of four indices."""
    e = delta()
    return (torch.einsum("ab,cd->abcd", e, e) + torch.einsum("ac,bd->abcd", e, e)
            + torch.einsum("ad,bc->abcd", e, e))


def sym_vec_mat(u: torch.Tensor, A: torch.Tensor) -> torch.Tensor:
    """``[u_a A_bc]_cyc = u_a A_bc + u_b A_ac + u_c A_ab`` (A symmetric)."""
    return (torch.einsum("...a,...bc->...abc", u, A) + torch.einsum("...b,...ac->...abc", u, A)
            + torch.einsum("...c,...ab->...abc", u, A))


def trace2(A: torch.Tensor) -> torch.Tensor:
    return torch.einsum("...aa->...", A)


def S_third(u: torch.Tensor, A: torch.Tensor) -> torch.Tensor:
    """Symmetric reading of ``2 u (x) A`` in Table I: contraction ``S_abb = 2 (A u)_a``."""
    return sym_vec_mat(u, A) - (trace2(A) / (D + 2))[..., None, None, None] * sym_delta(u, 1)


# --------------------------------------------------------------------------
# Hermite polynomial tensors and coefficients: App. D
# --------------------------------------------------------------------------
def hermite_tensors(v: torch.Tensor, RT_ref: float, N: int):
    """``H_0 .. H_N`` of Eq. (Hermitepolynomials-0-4) at velocities ``v`` ([Q, D])."""
    s = RT_ref
    H = [torch.ones(v.shape[0], dtype=DT), v.clone()]
    if N >= 2:
        H.append(outer_power(v, 2) - s * delta())
    if N >= 3:
        H.append(outer_power(v, 3) - s * sym_delta(v, 1))
    if N >= 4:
        H.append(outer_power(v, 4) - s * sym_delta(outer_power(v, 2), 2) + s * s * delta_delta())
    return H[: N + 1]


def coefficients_from_moments(M, RT_ref: float):
    """Hermite coefficients of Eq. (Hermitecoefficients-static-regform) from raw moments.

    ``M`` is a list ``[M_0, M_1, ...]`` of per-cell tensors with batch dims in
    front; the returned list has the same length.
    """
    s = RT_ref
    N = len(M) - 1
    a = [M[0], M[1]]
    if N >= 2:
        a.append(M[2] - s * M[0][..., None, None] * delta())
    if N >= 3:
        a.append(M[3] - s * sym_delta(a[1], 1))
    if N >= 4:
        a.append(M[4] - s * sym_delta(a[2], 2) - s * s * M[0][..., None, None, None, None] * delta_delta())
    return a[: N + 1]


def grad_expansion(a, w: torch.Tensor, H, RT_ref: float) -> torch.Tensor:
    """Populations of Eq. (Grad-Hermite-expansion-static) by full contraction.

    ``a[n]`` has shape ``batch + (D,)*n``; ``H[n]`` has shape ``(Q,) + (D,)*n``.
    Returns ``[Q, *batch]``.
    """
    batch = a[0].shape
    Q = w.shape[0]
    X = torch.zeros((Q,) + tuple(batch), dtype=DT)
    for n in range(len(a)):
        an = a[n].reshape(tuple(batch) + (-1,))
        Hn = H[n].reshape(Q, -1)
        contraction = torch.einsum("...k,qk->q...", an, Hn)
        X = X + contraction / (math.factorial(n) * RT_ref ** n)
    return w.reshape((Q,) + (1,) * len(batch)) * X


def discrete_moments(X: torch.Tensor, v: torch.Tensor, N: int):
    """``M_n(X) = sum_i v_i (x) ... (x) v_i X_i`` for ``n = 0..N`` (Sec. II D 5 notation)."""
    out = []
    for n in range(N + 1):
        Vn = outer_power(v, n).reshape(v.shape[0], -1)  # [Q, D^n]
        Mn = torch.einsum("q...,qk->...k", X, Vn)
        out.append(Mn.reshape(Mn.shape[:-1] + (D,) * n))
    return out


# --------------------------------------------------------------------------
# Macroscopic fields: Eqs. (eq_quadratur1-3), (eq:Total_energy_MB)
# --------------------------------------------------------------------------
def macroscopic(f: torch.Tensor, g: torch.Tensor, v: torch.Tensor, cfg: Config):
    """Density, velocity, total energy and temperature from the populations."""
    rho = f.sum(0)
    j = torch.einsum("q...,qa->...a", f, v)
    u = j / rho[..., None]
    if cfg.split == 1:
        E = g.sum(0)
    else:
        v2 = (v * v).sum(1)
        E = g.sum(0) + torch.einsum("q...,q->...", f, 0.5 * v2)
    T = (E / rho - 0.5 * (u * u).sum(-1)) / cfg.Cv
    return rho, u, E, T


# --------------------------------------------------------------------------
# Equilibrium moment sets: App. A
# --------------------------------------------------------------------------
def mb_moments_f(rho, u, T, R: float, N: int):
    """Maxwell-Boltzmann moments of ``f^eq`` up to order ``N`` (Eq. f-equilibria-moments-MB)."""
    p = rho * R * T
    RT = R * T
    M = [rho, rho[..., None] * u]
    M.append(rho[..., None, None] * outer_power(u, 2) + p[..., None, None] * delta())
    M.append(rho[..., None, None, None] * outer_power(u, 3) + p[..., None, None, None] * sym_delta(u, 1))
    M.append(rho[..., None, None, None, None] * outer_power(u, 4)
             + p[..., None, None, None, None] * sym_delta(outer_power(u, 2), 2)
             + (rho * RT * RT)[..., None, None, None, None] * delta_delta())
    return M[: N + 1]


def mb_moments_g(rho, u, T, E, cfg: Config):
    """Moments ``G_0, G_1, G_2`` of ``g^eq`` (App. A, Eqs. Relevantmoments_E/q/R and split II)."""
    R = cfg.R
    RT = R * T
    p = rho * RT
    uu = outer_power(u, 2)
    if cfg.split == 1:
        G0 = E
        G1 = u * (E + p)[..., None]
        G2 = p[..., None, None] * uu + (E + p)[..., None, None] * (uu + RT[..., None, None] * delta())
    else:
        G0 = rho * (cfg.Cv * T - RT * D / 2.0)
        G1 = G0[..., None] * u
        G2 = G0[..., None, None] * (uu + RT[..., None, None] * delta())
    return [G0, G1, G2]


# --------------------------------------------------------------------------
# Quasi-equilibrium moment sets: Table I (SummaryOfPopulations)
# --------------------------------------------------------------------------
def qe_moment_sets(f, g, v, rho, u, T, E, cfg: Config, Pr):
    """Moment sets of ``f*`` and ``g*`` for the current populations.

    Returns ``(Mf_eq, Mg_eq, Mf_star, Mg_star)``.
    """
    Nf = cfg.N_f
    Mf_eq = mb_moments_f(rho, u, T, cfg.R, Nf)
    Mg_eq = mb_moments_g(rho, u, T, E, cfg)
    Mf = discrete_moments(f, v, Nf)
    Mg1 = discrete_moments(g, v, 1)[1]
    dP = Mf[2] - Mf_eq[2]
    Mf_star = list(Mf_eq)
    Mg_star = list(Mg_eq)
    if bool(Pr == 1.0):  # no quasi-conserved fields: f* = f^eq, g* = g^eq
        return Mf_eq, Mg_eq, Mf_star, Mg_star
    pr_le_1 = bool(Pr < 1.0)
    if cfg.split == 1:
        uP = torch.einsum("...a,...ab->...b", u, dP)
        if pr_le_1:
            Mg_star[1] = Mg1 - uP
        else:
            Mf_star[2] = Mf[2]
            Mg_star[1] = Mg_eq[1] + uP
    else:
        if pr_le_1:
            Mf_star[3] = Mf[3] - S_third(u, dP)
            Mg_star[1] = Mg1
        else:
            tr = trace2(dP)
            dP_dev = dP - (tr / D)[..., None, None] * delta()
            Mf_star[2] = Mf[2] - (tr / D)[..., None, None] * delta()
            Mf_star[3] = Mf_eq[3] + S_third(u, dP_dev)
    return Mf_eq, Mg_eq, Mf_star, Mg_star


# --------------------------------------------------------------------------
# Relaxation times: Sec. II C, Eqs. (visc_shear_1) .. (eq:Pr_times_cases)
# --------------------------------------------------------------------------
def relaxation_times(rho, T, cfg: Config, tau_ref, Pr):
    """``(tau_1, tau_2)`` with ``tau_1 <= tau_2`` for the shear time ``tau_nu`` and Pr."""
    p = rho * cfg.R * T
    if cfg.visc_mode == CONST_MU:
        mu = tau_ref * cfg.p_ref
        tau_nu = mu / p
    else:
        tau_nu = tau_ref * torch.ones_like(p)
    tau_alpha = tau_nu / Pr
    if bool(Pr <= 1.0):
        return tau_nu, tau_alpha
    return tau_alpha, tau_nu


# --------------------------------------------------------------------------
# Equilibria, quasi-equilibria and collision
# --------------------------------------------------------------------------
def equilibria(rho, u, T, E, cfg: Config):
    """``f^eq, g^eq`` as Grad expansions of the App. A moment sets (Sec. II D 2)."""
    v, w = velocity_set(cfg)
    s = cfg.R * cfg.T_ref
    Hf = hermite_tensors(v, s, cfg.N_f)
    Hg = hermite_tensors(v, s, N_G)
    feq = grad_expansion(coefficients_from_moments(mb_moments_f(rho, u, T, cfg.R, cfg.N_f), s), w, Hf, s)
    geq = grad_expansion(coefficients_from_moments(mb_moments_g(rho, u, T, E, cfg), s), w, Hg, s)
    return feq, geq


def total_energy(rho, u, T, cfg: Config):
    """``E = rho Cv T + rho u^2 / 2`` (Eq. Total_energy_MB)."""
    return rho * cfg.Cv * T + 0.5 * rho * (u * u).sum(-1)


def populations(f, g, cfg: Config, Pr):
    """``(f^eq, g^eq, f*, g*)`` for the current populations (Sec. II D 2 and II D 4)."""
    v, w = velocity_set(cfg)
    s = cfg.R * cfg.T_ref
    rho, u, E, T = macroscopic(f, g, v, cfg)
    Mf_eq, Mg_eq, Mf_star, Mg_star = qe_moment_sets(f, g, v, rho, u, T, E, cfg, Pr)
    Hf = hermite_tensors(v, s, cfg.N_f)
    Hg = hermite_tensors(v, s, N_G)
    feq = grad_expansion(coefficients_from_moments(Mf_eq, s), w, Hf, s)
    geq = grad_expansion(coefficients_from_moments(Mg_eq, s), w, Hg, s)
    fst = grad_expansion(coefficients_from_moments(Mf_star, s), w, Hf, s)
    gst = grad_expansion(coefficients_from_moments(Mg_star, s), w, Hg, s)
    return feq, geq, fst, gst, (rho, u, E, T)


def collision(f, g, cfg: Config, dt, tau_ref=None, Pr=None):
    """``-dt/tau_1 (X - X*) - dt/tau_2 (X* - X^eq)`` of Eq. (finalDiscretePDE) for f and g."""
    tau_ref = cfg.tau_ref if tau_ref is None else tau_ref
    Pr = cfg.Pr if Pr is None else Pr
    feq, geq, fst, gst, (rho, u, E, T) = populations(f, g, cfg, Pr)
    tau1, tau2 = relaxation_times(rho, T, cfg, tau_ref, Pr)
    w1 = dt / tau1
    w2 = dt / tau2
    cf = -w1 * (f - fst) - w2 * (fst - feq)
    cg = -w1 * (g - gst) - w2 * (gst - geq)
    return cf, cg


# --------------------------------------------------------------------------
# Flux reconstruction: Sec. III A 2
# --------------------------------------------------------------------------
def limiter_phi(a, b, beta):
    """Generalised van Leer limiter ``phi(a, b) = max(0, min(beta r, (1 + r)/2, beta))``, ``r = a/b``."""
    nz = b != 0
    r = torch.where(nz, a / torch.where(nz, b, torch.ones_like(b)), torch.zeros_like(a))
    phi = torch.clamp(torch.minimum(torch.minimum(beta * r, 0.5 * (1.0 + r)), torch.full_like(r, beta)), min=0.0)
    return phi


def limited_increment(a, b, beta):
    """``(b/2) phi(a, b)``, zero when ``b == 0``."""
    return torch.where(b != 0, 0.5 * b * limiter_phi(a, b, beta), torch.zeros_like(b))


def neighbour(n: int, idx: torch.Tensor, bc: str) -> torch.Tensor:
    """Cell index of ``idx`` (may lie outside ``0..n-1``) under the boundary rule."""
    if bc == PERIODIC:
        return torch.remainder(idx, n)
    if bc == ZERO_GRADIENT:
        return torch.clamp(idx, 0, n - 1)
    raise ValueError(bc)


def face_values(X: torch.Tensor, vel: torch.Tensor, axis: int, bc: str, beta: float, ghosts=None) -> torch.Tensor:
    """NND face values ``X_{k - 1/2}`` for ``k = 0 .. n`` along ``axis`` of ``X`` ([Q, ny, nx]).

    Population ``i`` uses the upwind formula of its own velocity component
    ``vel[i]`` (``>= 0``: left-biased; ``< 0``: right-biased).  With
    ``ghosts = (below, above)`` (two layers each, outermost first below,
    innermost first above) the cells outside ``0 .. n-1`` are those layers.
    """
    n = X.shape[axis]
    k = torch.arange(n + 1)

    if ghosts is not None:
        Xe = torch.cat([ghosts[0], X, ghosts[1]], axis)  # cell c sits at c + 2

        def at(off):
            return Xe.index_select(axis, k + off + 2)
    else:
        def at(off):
            return X.index_select(axis, neighbour(n, k + off, bc))

    Xm2, Xm1, X0, Xp1 = at(-2), at(-1), at(0), at(1)
    pos = Xm1 + limited_increment(Xm1 - Xm2, X0 - Xm1, beta)
    neg = X0 + limited_increment(X0 - Xp1, Xm1 - X0, beta)
    mask = (vel >= 0).reshape((-1,) + (1,) * (X.dim() - 1))
    return torch.where(mask, pos, neg)


def advection(X: torch.Tensor, v: torch.Tensor, cfg: Config, dt, ghosts_y=None) -> torch.Tensor:
    """``-(dt/dV) sum_sigma v_i . n X_i(sigma) dA`` on the uniform Cartesian grid (Sec. III A 1-2).

    ``ghosts_y``: the two ghost rows below and above (walls, see ``wall_ghosts``)."""
    fx = face_values(X, v[:, 0], 2, cfg.bc_x, cfg.beta)  # [Q, ny, nx+1]
    fy = face_values(X, v[:, 1], 1, cfg.bc_y, cfg.beta, ghosts_y)  # [Q, ny+1, nx]
    vx = v[:, 0].reshape(-1, 1, 1)
    vy = v[:, 1].reshape(-1, 1, 1)
    div = (vx * (fx[:, :, 1:] - fx[:, :, :-1]) / cfg.dx
           + vy * (fy[:, 1:, :] - fy[:, :-1, :]) / cfg.dy)
    return -dt * div


# --------------------------------------------------------------------------
# Time step, initial state, one update, diagnostics
# --------------------------------------------------------------------------
def time_step(rho, u, T, cfg: Config) -> float:
    """``dt = CFL min(dx, dy) / max(|u| + c_s)`` over the initial fields (Sec. III A 3),
    with the adiabatic sound speed ``c_s = sqrt(gamma R T)``; a given ``cfg.dt > 0``
    is used as it stands."""
    if cfg.dt > 0:
        return float(cfg.dt)
    rho, u, T = (torch.as_tensor(x, dtype=DT) for x in (rho, u, T))
    speed = torch.sqrt((u * u).sum(-1)) + torch.sqrt(cfg.gamma * cfg.R * T)
    return float(cfg.cfl * min(cfg.dx, cfg.dy) / speed.max())


def max_relaxation_rate(rho, T, cfg: Config, dt) -> float:
    """Largest ``dt / tau_1`` over the fields (relaxation times of Sec. II C).

    The collision term of Eq. (finalDiscretePDE) is integrated with forward
    Euler (Sec. III A); on the relaxation alone one step multiplies
    ``X - X*`` by ``1 - dt/tau_1``, which stays bounded only while
    ``dt / tau_1 <= 2``."""
    rho, T = (torch.as_tensor(x, dtype=DT) for x in (rho, T))
    tau1, _ = relaxation_times(rho, T, cfg, cfg.tau_ref, cfg.Pr)
    return float((dt / tau1).max())


def initial_state(rho, ux, uy, T, cfg: Config):
    """Equilibrium populations of the initial fields (Sec. III A 3)."""
    rho = torch.as_tensor(rho, dtype=DT)
    T = torch.as_tensor(T, dtype=DT)
    u = torch.stack([torch.as_tensor(ux, dtype=DT), torch.as_tensor(uy, dtype=DT)], -1)
    E = total_energy(rho, u, T, cfg)
    return equilibria(rho, u, T, E, cfg)


def wall_ghosts(f, g, cfg: Config):
    """Ghost rows of no-slip walls below row 0 and above row ny-1 (thermal
    Couette flow, Sec. IV): ghost k (k = 1, 2 rows away from the wall) takes
    the fields of interior row k, reflected through the wall values,
    ``rho_G = rho_B``, ``u_G = 2 u_W - u_B``, ``T_G = 2 T_W - T_B``, and the
    populations ``X^eq(rho_G, u_G, T_G) + (X_B - X^eq(rho_B, u_B, T_B))``.
    Returns ``((f_below, f_above), (g_below, g_above))``, each [Q, 2, nx]
    (below: the outer row first; above: the inner row first)."""
    v, _ = velocity_set(cfg)
    rho, u, E, T = macroscopic(f, g, v, cfg)
    feq, geq = equilibria(rho, u, T, E, cfg)

    def ghost(row, wall):
        uW = torch.tensor([cfg.wall_ux[wall], 0.0], dtype=DT)
        rG, uG, TG = rho[row], 2.0 * uW - u[row], 2.0 * cfg.wall_T[wall] - T[row]
        fG, gG = equilibria(rG, uG, TG, total_energy(rG, uG, TG, cfg), cfg)
        return fG + (f[:, row] - feq[:, row]), gG + (g[:, row] - geq[:, row])

    ny = f.shape[1]
    b2, b1 = ghost(1, 0), ghost(0, 0)            # rows -2, -1
    a1, a2 = ghost(ny - 1, 1), ghost(ny - 2, 1)  # rows ny, ny+1
    fb = torch.stack([b2[0], b1[0]], 1)
    gb = torch.stack([b2[1], b1[1]], 1)
    fa = torch.stack([a1[0], a2[0]], 1)
    ga = torch.stack([a1[1], a2[1]], 1)
    return (fb, fa), (gb, ga)


def step(f, g, cfg: Config, dt, tau_ref=None, Pr=None):
    """One forward-Euler update of Eq. (finalDiscretePDE) for both distributions."""
    v, _ = velocity_set(cfg)
    cf, cg = collision(f, g, cfg, dt, tau_ref, Pr)
    gf = gg = None
    if cfg.bc_y == WALL:
        gf, gg = wall_ghosts(f, g, cfg)
    f_new = f + advection(f, v, cfg, dt, gf) + cf
    g_new = g + advection(g, v, cfg, dt, gg) + cg
    return f_new, g_new


def run(f, g, cfg: Config, dt, nsteps: int, tau_ref=None, Pr=None):
    for _ in range(nsteps):
        f, g = step(f, g, cfg, dt, tau_ref, Pr)
    return f, g


def diagnostics(f, g, cfg: Config):
    """Fields ``rho, u, T`` and global sums of mass, momentum and total energy."""
    v, _ = velocity_set(cfg)
    rho, u, E, T = macroscopic(f, g, v, cfg)
    sums = torch.stack([rho.sum(), (rho[..., None] * u)[..., 0].sum(),
                        (rho[..., None] * u)[..., 1].sum(), E.sum()])
    return {"rho": rho, "ux": u[..., 0], "uy": u[..., 1], "T": T, "sums": sums}


# --------------------------------------------------------------------------
# Single-cell updates on sampled cells (for checks at sizes the full oracle
# cannot run): the update of a cell needs only a cross of radius 2.
# --------------------------------------------------------------------------
def window_indices(cfg: Config, ys, xs):
    """Row and column indices ``[S, 5]`` of the radius-2 windows around cells ``(ys, xs)``."""
    off = torch.arange(-2, 3)
    yi = neighbour(cfg.ny, torch.as_tensor(ys)[:, None] + off[None, :], cfg.bc_y)
    xi = neighbour(cfg.nx, torch.as_tensor(xs)[:, None] + off[None, :], cfg.bc_x)
    return yi, xi


def gather_windows(X: torch.Tensor, yi: torch.Tensor, xi: torch.Tensor) -> torch.Tensor:
    """``[Q, S, 5, 5]`` windows of ``X`` ([Q, ny, nx]) at the given index sets."""
    return X[:, yi[:, :, None], xi[:, None, :]]


def window_step(fw, gw, cfg: Config, dt, tau_ref=None, Pr=None):
    """Update of the centre cell of each 5x5 window ``[Q, S, 5, 5]``.

    The update of a cell needs only a cross of radius 2 around it, so the
    windows are laid side by side in one periodic 5 x 5S strip; each centre
    reads only its own window. Returns ``(f_new, g_new)`` of shape ``[Q, S]``.
    """
    Q, S = fw.shape[:2]

    def strip(W):
        return W.permute(0, 2, 1, 3).reshape(Q, 5, 5 * S)

    wcfg = Config(**{**cfg.__dict__, "nx": 5 * S, "ny": 5, "bc_x": PERIODIC, "bc_y": PERIODIC})
    fn, gn = step(strip(fw), strip(gw), wcfg, dt, tau_ref, Pr)
    centre = torch.arange(S) * 5 + 2
    return fn[:, 2, centre], gn[:, 2, centre]


def sampled_step(f, g, cfg: Config, dt, ys, xs, tau_ref=None, Pr=None):
    """One update of the cells ``(ys[k], xs[k])`` of a full state ``[Q, ny, nx]``.

    Zero-gradient neighbours are taken as clamped indices when the windows
    are cut out, so the window update equals the full update under either
    boundary rule.
    """
    yi, xi = window_indices(cfg, ys, xs)
    return window_step(gather_windows(f, yi, xi), gather_windows(g, yi, xi), cfg, dt, tau_ref, Pr)
