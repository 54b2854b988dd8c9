"""Sound diagnostics of the shock-vortex interaction (Sec. IV).

Analysis of macroscopic fields that :meth:`Solver.moments` returns (moved to
the host as numpy arrays): none of the solver's arithmetic is here.

* ``sound_pressure``: ``p / p_r - 1`` with ``p_r`` the initial post-shock
  pressure;
* ``t_star``: the non-dimensional time ``t c_l / r_v`` (pre-shock sound speed
  ``c_l``, vortex radius ``r_v``);
* ``vorticity``: ``d u_y / dx - d u_x / dy`` by central differences;
* ``vortex_centre``: the minimum of a field (the vorticity of a clockwise
  vortex) near a guess, refined to sub-cell position by a parabola through
  the neighbours in x and in y;
* ``ray`` and ``circle``: bilinear samples of a cell-centred field along a
  ray from the vortex centre (angle counter-clockwise from +x, the paper's
  45 degree profile) and around a circle (the circumferential profiles at
  ``r / r_v = 8.8`` and ``10.8``);
* ``sound_amplitude``: ``p_Sound,2 - p_Sound,1``, the second sound at one
  radius minus the precursor at another, per angle.

Grids are cell-centred, ``field[y, x]`` with cell ``(i, j)`` at
``((i + 1/2) dx, (j + 1/2) dy)``; samples wrap periodically in y and clamp to
the first and last cell in x.
"""

from __future__ import annotations

import numpy as np


def sound_pressure(rho: np.ndarray, T: np.ndarray, p_post: float, R: float = 1.0) -> np.ndarray:
    """``p / p_r - 1`` with the ideal-gas pressure ``p = rho R T``."""
    return np.asarray(rho) * R * np.asarray(T) / p_post - 1.0


def t_star(t: float, c_l: float, r_v: float) -> float:
    """Non-dimensional time ``t c_l / r_v``."""
    return t * c_l / r_v


def sample(field: np.ndarray, x, y, dx: float, dy: float) -> np.ndarray:
    """Bilinear interpolation of a cell-centred field at points ``(x, y)``."""
    ny, nx = field.shape
    fx = np.clip(np.asarray(x, dtype=np.float64) / dx - 0.5, 0.0, nx - 1.0)
    fy = np.asarray(y, dtype=np.float64) / dy - 0.5
    i0 = np.minimum(np.floor(fx).astype(np.int64), nx - 2)
    j0 = np.floor(fy).astype(np.int64)
    ax, ay = fx - i0, fy - j0
    j0 %= ny
    j1 = (j0 + 1) % ny
    return ((1 - ay) * ((1 - ax) * field[j0, i0] + ax * field[j0, i0 + 1])
            + ay * ((1 - ax) * field[j1, i0] + ax * field[j1, i0 + 1]))


def vorticity(ux: np.ndarray, uy: np.ndarray, dx: float, dy: float) -> np.ndarray:
    """``d u_y / dx - d u_x / dy``: central differences, periodic in y and
    one-sided at the first and last column."""
    return (np.gradient(uy, dx, axis=1)
            - (np.roll(ux, -1, axis=0) - np.roll(ux, 1, axis=0)) / (2.0 * dy))


def vortex_centre(field: np.ndarray, dx: float, dy: float, guess, search: float) -> tuple[float, float]:
    """Position of the minimum of ``field`` within ``search`` of ``guess``
    (for a clockwise vortex, ``field`` is its vorticity)."""
    p = field
    ny, nx = p.shape
    gx, gy = guess
    i_lo, i_hi = max(int((gx - search) / dx), 1), min(int((gx + search) / dx) + 1, nx - 1)
    rows = np.arange(int((gy - search) / dy), int((gy + search) / dy) + 1)
    win = p[rows % ny][:, i_lo:i_hi]
    jr, ir = np.unravel_index(np.argmin(win), win.shape)
    i, j = i_lo + ir, int(rows[jr]) % ny

    def vertex(a, b, c):  # offset of the minimum of the parabola through (-1, a), (0, b), (1, c)
        d = a - 2 * b + c
        return 0.5 * (a - c) / d if d > 0 else 0.0

    ox = vertex(p[j, i - 1], p[j, i], p[j, i + 1])
    oy = vertex(p[(j - 1) % ny, i], p[j, i], p[(j + 1) % ny, i])
    return (i + 0.5 + ox) * dx, (j + 0.5 + oy) * dy


def ray(field: np.ndarray, centre, angle_deg: float, radii, dx: float, dy: float) -> np.ndarray:
    """Samples along the ray from ``centre`` at ``angle_deg``, at distances ``radii``."""
    a = np.deg2rad(angle_deg)
    r = np.asarray(radii, dtype=np.float64)
    return sample(field, centre[0] + r * np.cos(a), centre[1] + r * np.sin(a), dx, dy)


def circle(field: np.ndarray, centre, radius: float, angles_deg, dx: float, dy: float) -> np.ndarray:
    """Samples on the circle of ``radius`` around ``centre`` at ``angles_deg``."""
    a = np.deg2rad(np.asarray(angles_deg, dtype=np.float64))
    return sample(field, centre[0] + radius * np.cos(a), centre[1] + radius * np.sin(a), dx, dy)


def sound_amplitude(p_sound: np.ndarray, centre, r_second: float, r_precursor: float, angles_deg,
                    dx: float, dy: float) -> np.ndarray:
    """``p_Sound,2 - p_Sound,1`` per angle: the sound pressure at ``r_second``
    minus that at ``r_precursor``."""
    return (circle(p_sound, centre, r_second, angles_deg, dx, dy)
            - circle(p_sound, centre, r_precursor, angles_deg, dx, dy))
