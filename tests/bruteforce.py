"""A second, deliberately different and slow implementation of one update.

Used only to pin the oracle on tiny grids. It shares nothing with the oracle
but the seeded input fields:

* moments are kept as scalar components ``M[(p, q)] = sum_i vx^p vy^q X_i``
  instead of symmetric tensors;
* Maxwell-Boltzmann moments are products of 1-D Gaussian raw moments, and the
  energy-distribution moments are taken directly from the continuous
  definition of ``g^eq`` in Eq. (energy_eq_1) rather than from App. A;
* (quasi-)equilibrium populations are found by solving the moment-matching
  linear system for a polynomial of total degree <= N times the weights,
  instead of Hermite coefficients (the two agree because the lattice
  integrates every product of two such polynomials exactly);
* the QE corrections of Table I are written component by component;
* fluxes are explicit per-face loops in plain Python floats.
"""

from __future__ import annotations

import math

import numpy as np


def gh_1d(n):
    x, w = np.polynomial.hermite_e.hermegauss(n)
    return x, w / math.sqrt(2.0 * math.pi)


def lattice(split, R=1.0, T_ref=1.0):
    n = 4 if split == 1 else 5
    x, w = gh_1d(n)
    c = math.sqrt(R * T_ref)
    vx = np.repeat(x, n) * c
    vy = np.tile(x, n) * c
    wt = np.repeat(w, n) * np.tile(w, n)
    return vx, vy, wt


def gauss_raw_moment(k, mean, var):
    """E[X^k] for X ~ N(mean, var): sum_j C(k, 2j) (2j-1)!! var^j mean^(k-2j)."""
    s = 0.0
    for j in range(k // 2 + 1):
        dfact = 1.0
        for t in range(1, 2 * j, 2):
            dfact *= t
        s += math.comb(k, 2 * j) * dfact * var ** j * mean ** (k - 2 * j)
    return s


def index_set(N):
    return [(p, q) for p in range(N + 1) for q in range(N + 1 - p)]


def fit_populations(M, N, vx, vy, w):
    """Populations ``w_i P(v_i)`` with ``deg P <= N`` whose moments ``(p, q), p + q <= N`` equal ``M``."""
    idx = index_set(N)
    A = np.empty((len(idx), len(idx)))
    for r, (p1, q1) in enumerate(idx):
        for c, (p2, q2) in enumerate(idx):
            A[r, c] = np.sum(w * vx ** (p1 + p2) * vy ** (q1 + q2))
    rhs = np.array([M[k] for k in idx])
    coef = np.linalg.solve(A, rhs)
    P = sum(coef[c] * vx ** p * vy ** q for c, (p, q) in enumerate(idx))
    return w * P


def moments(X, vx, vy, N):
    return {(p, q): float(np.sum(vx ** p * vy ** q * X)) for (p, q) in index_set(N)}


def cell_update_collision(f, g, vx, vy, w, split, R, gamma, Pr, tau_ref, p_ref, visc_mode, dt):
    Cv = R / (gamma - 1.0)
    Nf = 3 if split == 1 else 4
    Mf = moments(f, vx, vy, Nf)
    rho = Mf[(0, 0)]
    ux, uy = Mf[(1, 0)] / rho, Mf[(0, 1)] / rho
    if split == 1:
        E = float(np.sum(g))
    else:
        E = float(np.sum(g)) + 0.5 * (Mf[(2, 0)] + Mf[(0, 2)])
    T = (E / rho - 0.5 * (ux * ux + uy * uy)) / Cv
    RT = R * T
    # Maxwell-Boltzmann moments of f
    Mfeq = {(p, q): rho * gauss_raw_moment(p, ux, RT) * gauss_raw_moment(q, uy, RT)
            for (p, q) in index_set(Nf)}
    # moments of the continuous g^eq of Eq. (energy_eq_1)
    def gm(p, q):
        mp, mq = gauss_raw_moment(p, ux, RT), gauss_raw_moment(q, uy, RT)
        if split == 2:
            return rho * (Cv * T - RT) * mp * mq
        return rho * ((Cv * T - RT) * mp * mq
                      + 0.5 * (gauss_raw_moment(p + 2, ux, RT) * mq + mp * gauss_raw_moment(q + 2, uy, RT)))
    Mgeq = {(p, q): gm(p, q) for (p, q) in index_set(2)}
    Mg = moments(g, vx, vy, 1)
    dxx = Mf[(2, 0)] - Mfeq[(2, 0)]
    dxy = Mf[(1, 1)] - Mfeq[(1, 1)]
    dyy = Mf[(0, 2)] - Mfeq[(0, 2)]
    Mfs = dict(Mfeq)
    Mgs = dict(Mgeq)
    low = Pr <= 1.0
    if split == 1:
        upx = ux * dxx + uy * dxy
        upy = ux * dxy + uy * dyy
        if low:
            Mgs[(1, 0)] = Mg[(1, 0)] - upx
            Mgs[(0, 1)] = Mg[(0, 1)] - upy
        else:
            Mfs[(2, 0)], Mfs[(1, 1)], Mfs[(0, 2)] = Mf[(2, 0)], Mf[(1, 1)], Mf[(0, 2)]
            Mgs[(1, 0)] = Mgeq[(1, 0)] + upx
            Mgs[(0, 1)] = Mgeq[(0, 1)] + upy
    else:
        def S(axx, axy, ayy):
            tr = axx + ayy
            return {(3, 0): 3 * ux * axx - 3 * tr * ux / 4,
                    (2, 1): 2 * ux * axy + uy * axx - tr * uy / 4,
                    (1, 2): 2 * uy * axy + ux * ayy - tr * ux / 4,
                    (0, 3): 3 * uy * ayy - 3 * tr * uy / 4}
        if low:
            s = S(dxx, dxy, dyy)
            for k in s:
                Mfs[k] = Mf[k] - s[k]
            Mgs[(1, 0)], Mgs[(0, 1)] = Mg[(1, 0)], Mg[(0, 1)]
        else:
            h = 0.5 * (dxx + dyy)
            Mfs[(2, 0)] = Mf[(2, 0)] - h
            Mfs[(1, 1)] = Mf[(1, 1)]
            Mfs[(0, 2)] = Mf[(0, 2)] - h
            s = S(dxx - h, dxy, dyy - h)
            for k in s:
                Mfs[k] = Mfeq[k] + s[k]
    feq = fit_populations(Mfeq, Nf, vx, vy, w)
    fst = fit_populations(Mfs, Nf, vx, vy, w)
    geq = fit_populations(Mgeq, 2, vx, vy, w)
    gst = fit_populations(Mgs, 2, vx, vy, w)
    p = rho * RT
    tau_nu = tau_ref * p_ref / p if visc_mode == "const_mu" else tau_ref
    tau_a = tau_nu / Pr
    t1, t2 = (tau_nu, tau_a) if low else (tau_a, tau_nu)
    cf = -(dt / t1) * (f - fst) - (dt / t2) * (fst - feq)
    cg = -(dt / t1) * (g - gst) - (dt / t2) * (gst - geq)
    return cf, cg


def phi(a, b, beta):
    if b == 0.0:
        return 0.0
    r = a / b
    return max(0.0, min(beta * r, 0.5 * (1.0 + r), beta))


def face(Xline, k, vsign_pos, beta, wrap):
    """Face value between cells k-1 and k of one population line."""
    X = lambda j: Xline[wrap(j)]  # noqa: E731
    if vsign_pos:
        a = X(k - 1) - X(k - 2)
        b = X(k) - X(k - 1)
        return X(k - 1) + 0.5 * b * phi(a, b, beta)
    a = X(k) - X(k + 1)
    b = X(k - 1) - X(k)
    return X(k) + 0.5 * b * phi(a, b, beta)


def step(f, g, split, dx, dy, dt, R=1.0, gamma=1.4, Pr=0.71, tau_ref=1e-2, p_ref=1.0,
         visc_mode="const_mu", beta=1.2, bc_x="periodic", bc_y="periodic"):
    """One update of ``f, g`` (arrays ``[Q, ny, nx]``) by explicit loops."""
    vx, vy, w = lattice(split, R)
    Q, ny, nx = f.shape

    def wrapper(n, bc):
        if bc == "periodic":
            return lambda j: j % n
        return lambda j: min(max(j, 0), n - 1)

    wx, wy = wrapper(nx, bc_x), wrapper(ny, bc_y)
    fn = f.copy()
    gn = g.copy()
    for y in range(ny):
        for x in range(nx):
            cf, cg = cell_update_collision(f[:, y, x], g[:, y, x], vx, vy, w, split, R, gamma, Pr,
                                           tau_ref, p_ref, visc_mode, dt)
            fn[:, y, x] += cf
            gn[:, y, x] += cg
    for X, Xn in ((f, fn), (g, gn)):
        for i in range(Q):
            for y in range(ny):
                line = X[i, y, :]
                for x in range(nx):
                    fl = face(line, x, vx[i] >= 0, beta, wx)
                    fr = face(line, x + 1, vx[i] >= 0, beta, wx)
                    Xn[i, y, x] -= dt / dx * vx[i] * (fr - fl)
            for x in range(nx):
                col = X[i, :, x]
                for y in range(ny):
                    fl = face(col, y, vy[i] >= 0, beta, wy)
                    fr = face(col, y + 1, vy[i] >= 0, beta, wy)
                    Xn[i, y, x] -= dt / dy * vy[i] * (fr - fl)
    return fn, gn
