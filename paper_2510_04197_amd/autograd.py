"""Differentiable DVBM rollouts: ``torch.autograd.Function`` over the HIP adjoint.

``rollout_temperature(T0, tau_ref, Pr, ...)`` runs ``nsteps`` steps of the
DDF-QE DVBM from the equilibrium of ``(rho0, u0, T0)`` and returns the final
temperature field; its backward pass is the discrete adjoint of the library
(``dvbm_adjoint_*``), with checkpoints every ``K`` steps and recomputation of
each segment's states during the reverse sweep. The time step is held fixed
(it must be given explicitly), so the gradient is that of the fixed-dt map.

Argument marshalling only: forward and reverse sweeps run in the HIP kernels.
"""

from __future__ import annotations

import torch

from .dvbm import Solver, make_params


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, T0, tau_ref, Pr, rho0, ux0, uy0, nsteps, K, params_kw):
        if not params_kw.get("dt", 0.0) > 0.0:
            raise ValueError("rollout_temperature needs an explicit dt > 0")
        ny, nx = T0.shape
        p = make_params(nx, ny, tau_ref=float(tau_ref), Pr=float(Pr), **params_kw)
        s = Solver(p, rho0, ux0, uy0, T0.detach(), device=T0.device)
        ckpts = []
        n = 0
        while n < nsteps:
            ckpts.append(s.state_buffer.clone())
            k = min(K, nsteps - n)
            s.step(k)
            n += k
        out = s.moments(fields=True, sums=False)["T"]
        ctx.solver = s
        ctx.ckpts = ckpts
        ctx.final = s.state_buffer.clone()
        ctx.nsteps, ctx.K = nsteps, K
        ctx.fields0 = (rho0, ux0, uy0, T0.detach())
        ctx.pdev = (tau_ref.device if torch.is_tensor(tau_ref) else None,
                    Pr.device if torch.is_tensor(Pr) else None)
        return out

    @staticmethod
    def backward(ctx, gT):
        s: Solver = ctx.solver
        lam = s.adjoint_moments(ctx.final, d_T=gT.contiguous())
        lam_tmp = torch.empty_like(lam)
        dparams = torch.zeros(2, dtype=torch.float64, device=lam.device)
        nsteps, K = ctx.nsteps, ctx.K
        # room for the recomputed states of one segment (the checkpoint is the first)
        seg_states = torch.empty((max(K - 1, 1), s.buffers[0].numel()), dtype=torch.uint8, device=lam.device)
        for seg in reversed(range(len(ctx.ckpts))):
            n0 = seg * K
            n1 = min(n0 + K, nsteps)
            # recompute the states n0 .. n1-1 of this segment from its checkpoint
            states = [ctx.ckpts[seg]]
            for j in range(n1 - n0 - 1):
                s.step_from(states[-1], seg_states[j])
                states.append(seg_states[j])
            for st in reversed(states):
                s.adjoint_step(st, lam, lam_tmp, dparams)
                lam, lam_tmp = lam_tmp, lam
        g = s.adjoint_init(lam, *ctx.fields0, which=("T",))["T"]
        s.close()
        dtau = dparams[0].to(ctx.pdev[0]) if ctx.pdev[0] is not None else None
        dpr = dparams[1].to(ctx.pdev[1]) if ctx.pdev[1] is not None else None
        return g, dtau, dpr, None, None, None, None, None, None


def rollout_temperature(T0: torch.Tensor, tau_ref: torch.Tensor, Pr: torch.Tensor, rho0, ux0, uy0,
                        nsteps: int, K: int = 10, **params_kw) -> torch.Tensor:
    """Final temperature after ``nsteps`` steps; differentiable in ``T0``, ``tau_ref`` and ``Pr``.

    ``T0`` is a float64 CUDA tensor of shape ``(ny, nx)``; ``tau_ref`` and
    ``Pr`` are 0-dim tensors; ``params_kw`` are the remaining solver
    parameters of :func:`make_params` (``dx``, ``dy``, ``split``, ``storage``,
    boundaries, ``gamma`` ... and an explicit ``dt``).
    """
    return _Rollout.apply(T0, tau_ref, Pr, rho0, ux0, uy0, int(nsteps), int(K), dict(params_kw))
