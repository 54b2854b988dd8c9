"""Differentiable DVBM rollouts: ``torch.autograd.Function`` over the HIP adjoint.

``rollout_temperature(T0, tau_ref, Pr, ...)`` runs ``nsteps`` steps of the
DDF-QE DVBM from the equilibrium of ``(rho0, u0, T0)`` and returns the final
temperature field; its backward pass is the discrete adjoint of the library
(``dvbm_adjoint_*``), with checkpoints every ``K`` steps and recomputation of
each segment's states during the reverse sweep (optionally on a second stream,
one segment ahead of the sweep); the last segment's states are kept by the
forward pass, which steps through them anyway. The time step is held fixed
(it must be given explicitly), so the gradient is that of the fixed-dt map.

Argument marshalling only: forward and reverse sweeps run in the HIP kernels.
"""

from __future__ import annotations

import torch

from .dvbm import Solver, make_params


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, T0, tau_ref, Pr, rho0, ux0, uy0, nsteps, K, overlap, cotangent, params_kw):
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
            if n + k < nsteps:
                s.step(k)
            else:
                # the last segment steps through a buffer of its k - 1 intermediate states, which the
                # reverse sweep then reads as they are instead of recomputing them (same kernel, same
                # results), and afterwards reuses for recomputing the segments before it (so it holds
                # K - 1 states when there are such segments); the final step lands in the solver's
                # other buffer, made current
                rows = max((K if n > 0 else k) - 1, 1)
                last = torch.empty((rows, s.buffers[0].numel()), dtype=torch.uint8, device=T0.device)
                ctx.last_buf = last
                prev = ckpts[-1]
                for j in range(k - 1):
                    s.step_from(prev, last[j])
                    prev = last[j]
                other = 1 - s.state_index
                s.step_from(prev, s.buffers[other])
                s.set_state_index(other)
                ctx.last = [ckpts[-1]] + [last[j] for j in range(k - 1)]
            n += k
        out = s.moments(fields=True, sums=False)["T"]
        ctx.solver = s
        ctx.ckpts = ckpts
        ctx.final = s.state_buffer.clone()
        ctx.nsteps, ctx.K, ctx.overlap = nsteps, K, overlap
        ctx.lam_dtype = {"f64": torch.float64, "f32": torch.float32}[cotangent]
        ctx.fields0 = (rho0, ux0, uy0, T0.detach())
        ctx.pdev = (tau_ref.device if torch.is_tensor(tau_ref) else None,
                    Pr.device if torch.is_tensor(Pr) else None)
        return out

    @staticmethod
    def backward(ctx, gT):
        s: Solver = ctx.solver
        dev = gT.device
        lam = s.adjoint_moments(ctx.final, d_T=gT.contiguous()).to(ctx.lam_dtype)
        lam_tmp = torch.empty_like(lam)
        dparams = torch.zeros(2, dtype=torch.float64, device=dev)
        nsteps, K = ctx.nsteps, ctx.K
        nseg = len(ctx.ckpts)
        # With overlap, the states of segment j-1 are recomputed from its
        # checkpoint on a side stream, by a second handle, while the main stream
        # runs the reverse sweep over segment j: two buffers of K-1 states take
        # turns.  Without, one buffer and one stream, recomputing after each sweep.
        main = s.stream
        nb = s.buffers[0].numel()
        # the forward pass's last-segment buffer is one of them: segment nseg - 1 is read from it,
        # and the segments of the same parity are recomputed into it afterwards
        if ctx.overlap:
            side = torch.cuda.Stream(device=dev)
            side.wait_stream(main)  # the checkpoints and the forward state are ready
            r = Solver(s.params, *ctx.fields0, device=dev, stream=side)
            bufs = [None, None]
            bufs[(nseg - 1) % 2] = ctx.last_buf
            bufs[nseg % 2] = torch.empty((max(K - 1, 1), nb), dtype=torch.uint8, device=dev) if nseg > 1 else None
            # memory the side stream uses is not handed out again before its work is done
            for tns in [b for b in bufs if b is not None] + ctx.ckpts + r.buffers + [r.workspace] + list(r._fields0):
                tns.record_stream(side)
        else:
            side, r = main, s
            bufs = [ctx.last_buf] * 2
        ready = [torch.cuda.Event() for _ in range(nseg)]
        free = [None, None]  # event on main after the last reverse sweep that read bufs[k]

        def seg_range(seg):
            n0 = seg * K
            return n0, min(n0 + K, nsteps)

        def recompute(seg):
            n0, n1 = seg_range(seg)
            buf = bufs[seg % 2]
            if free[seg % 2] is not None:
                side.wait_event(free[seg % 2])
            states = [ctx.ckpts[seg]]
            for j in range(n1 - n0 - 1):
                r.step_from(states[-1], buf[j])
                states.append(buf[j])
            ready[seg].record(side)
            return states

        # the last segment's states were kept by the forward pass
        ready[nseg - 1].record(main)
        pending = {nseg - 1: ctx.last}
        for seg in reversed(range(nseg)):
            states = pending.pop(seg)
            if ctx.overlap and seg > 0:
                pending[seg - 1] = recompute(seg - 1)
            main.wait_event(ready[seg])
            for st in reversed(states):
                s.adjoint_step(st, lam, lam_tmp, dparams)
                lam, lam_tmp = lam_tmp, lam
            ev = torch.cuda.Event()
            ev.record(main)
            free[seg % 2] = ev
            if not ctx.overlap and seg > 0:
                pending[seg - 1] = recompute(seg - 1)
        if ctx.overlap:
            main.wait_stream(side)
            r.close()
        g = s.adjoint_init(lam.to(torch.float64), *ctx.fields0, which=("T",))["T"]
        s.close()
        dtau = dparams[0].to(ctx.pdev[0]) if ctx.pdev[0] is not None else None
        dpr = dparams[1].to(ctx.pdev[1]) if ctx.pdev[1] is not None else None
        return g, dtau, dpr, None, None, None, None, None, None, None, None


def rollout_temperature(T0: torch.Tensor, tau_ref: torch.Tensor, Pr: torch.Tensor, rho0, ux0, uy0,
                        nsteps: int, K: int = 10, overlap: bool = False, cotangent: str = "f64",
                        **params_kw) -> torch.Tensor:
    """Final temperature after ``nsteps`` steps; differentiable in ``T0``, ``tau_ref`` and ``Pr``.

    ``T0`` is a float64 CUDA tensor of shape ``(ny, nx)``; ``tau_ref`` and
    ``Pr`` are 0-dim tensors; ``params_kw`` are the remaining solver
    parameters of :func:`make_params` (``dx``, ``dy``, ``split``, ``storage``,
    boundaries, ``gamma`` ... and an explicit ``dt``).  ``overlap`` recomputes
    the next segment on a second stream during each reverse sweep, at the cost
    of a second buffer of ``K - 1`` states and a second handle; the gradient is
    the same bit for bit (on a 256 x 256 grid it saves about a tenth of a
    forward run: the reverse sweep's kernels leave little room on the SIMDs).
    ``cotangent="f32"`` stores the cotangents of the reverse
    sweep in float32 (``dvbm_adjoint_step_f32``; the arithmetic stays float64),
    which halves their memory traffic at one float32 rounding per value and step.
    """
    if cotangent not in ("f64", "f32"):
        raise ValueError("cotangent must be 'f64' or 'f32'")
    if int(nsteps) < 1 or int(K) < 1:
        raise ValueError("rollout_temperature needs nsteps >= 1 and a checkpoint interval K >= 1")
    return _Rollout.apply(T0, tau_ref, Pr, rho0, ux0, uy0, int(nsteps), int(K), bool(overlap), cotangent,
                          dict(params_kw))
