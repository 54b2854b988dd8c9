"""Reverse mode through the oracle's step on small windows around sampled
cells: the exact cotangent of those cells on a grid of any size (test
infrastructure; used by the full-size adjoint tests and pinned on the CPU
against the full-grid reverse mode)."""

import torch

from oracle import dvbm_oracle as O


def oracle_adjoint_windows(X, lam1, ys, xs, cfg, dt, r=4):
    """lam at the cells (ys[k], xs[k]) of a periodic grid, from reverse mode
    through the oracle's step on (2r + 1)^2 windows around them.

    lam(c) = sum_j lam'_j dX'_j/dX_c over the cells j whose update reads X_c:
    the cross of radius 2 around c (the flux stencil is radius 2 along each
    axis, the relaxation is local).  Their stencils stay within radius 4 of c,
    so with r = 4 a window laid out periodically in a strip of windows gives
    each centre its exact cotangent.  X and lam1 are [2, Q, ny, nx] (any device);
    returns [2, Q, S] (CPU)."""
    n, S, Q = 2 * r + 1, len(ys), X.shape[1]
    off = torch.arange(-r, r + 1)
    yi = ((ys[:, None] + off[None, :]) % cfg.ny).to(X.device)
    xi = ((xs[:, None] + off[None, :]) % cfg.nx).to(X.device)

    def strip(A):  # [2, Q, S, n, n] -> [2, Q, n, n S]
        return A.permute(0, 1, 3, 2, 4).reshape(2, Q, n, n * S)

    Xs = strip(X[:, :, yi[:, :, None], xi[:, None, :]].cpu()).clone().requires_grad_(True)
    Ls = strip(lam1[:, :, yi[:, :, None], xi[:, None, :]].cpu())
    wcfg = O.Config(**{**cfg.__dict__, "nx": n * S, "ny": n, "bc_x": O.PERIODIC, "bc_y": O.PERIODIC})
    fn, gn = O.step(Xs[0], Xs[1], wcfg, dt)
    mask = torch.zeros(n, n * S, dtype=torch.float64)
    for k in range(S):
        cx = k * n + r
        mask[r, cx - 2:cx + 3] = 1.0
        mask[r - 2:r + 3, cx] = 1.0
    ((Ls[0] * fn + Ls[1] * gn) * mask).sum().backward()
    return Xs.grad[:, :, r, torch.arange(S) * n + r]
