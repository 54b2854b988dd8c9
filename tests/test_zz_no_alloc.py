"""dvbm_adjoint_step_noalloc (the adjoint step for callers that cannot
allocate: work rows and reduction partials in the library's fixed per-device
scratch) against dvbm_adjoint_step with a caller work array.

Both run the same kernels on the same inputs and their reductions are summed
in a fixed order, so lam_n and the parameter derivatives must agree bit for
bit.  Two calls in a row share the scratch, the second on a smaller grid, so
stale work rows or a counter left set by the first would show; grids whose
work rows exceed the scratch are rejected.
"""

import numpy as np
import pytest
import torch

from paper_2510_04197_amd import DVBMError, Solver, dvbm, make_params
from synth import smooth_random

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _case(nx, ny, split, Pr, bc, storage, seed):
    print(f"[noalloc] {nx}x{ny} split={split} Pr={Pr} bc={bc} {storage}", flush=True)
    wl = smooth_random(nx, ny, seed=seed)
    p = make_params(wl.nx, wl.ny, dx=wl.dx, dy=wl.dy, split=split, storage=storage, Pr=Pr, tau_ref=0.02,
                    bc_x=bc, bc_y=bc, dt=3e-3)
    s = Solver(p, wl.rho, wl.ux, wl.uy, wl.T, device=DEV)
    s.step(3)
    rng = np.random.default_rng(seed)
    lam1 = torch.tensor(rng.standard_normal((2, s.Q, ny, nx)), device=DEV)
    return s, lam1


def _both(s, lam1):
    ref, got = s.new_cotangent(), s.new_cotangent()
    dref = torch.zeros(2, dtype=torch.float64, device=DEV)
    dgot = torch.zeros(2, dtype=torch.float64, device=DEV)
    s.adjoint_step(s.state_buffer, lam1, ref, dref)
    s.adjoint_step_noalloc(s.state_buffer, lam1, got, dgot)
    torch.cuda.synchronize()
    return ref, got, dref, dgot


@pytest.mark.parametrize("storage", ("f64", "f32"))
def test_noalloc_matches_adjoint_step_two_calls(storage):
    """256^2 (the gradient workload's grid), then 117 x 17 (a ragged strip,
    fewer blocks than the first call): lam_n and d/dtau_ref, d/dPr equal
    dvbm_adjoint_step's bit for bit on both, and again on a repeat of the
    second call."""
    cases = [(256, 256, 2, 0.71, "periodic", 5), (117, 17, 1, 1.7, "zero_gradient", 6)]
    for nx, ny, split, Pr, bc, seed in cases:
        s, lam1 = _case(nx, ny, split, Pr, bc, storage, seed)
        for _ in range(2 if nx == 117 else 1):
            ref, got, dref, dgot = _both(s, lam1)
            assert torch.isfinite(ref).all() and float(ref.abs().max()) > 0
            assert torch.equal(got, ref)
            assert torch.equal(dgot, dref) and float(dref.abs().min()) > 0
        s.close()


def test_noalloc_without_dparams_and_pr_one():
    """dparams = NULL (no reduction) and Pr = 1 (no quasi-equilibrium) on the
    same scratch after a call that used it."""
    s, lam1 = _case(70, 13, 2, 1.0, "periodic", "f64", 7)
    ref, got = s.new_cotangent(), s.new_cotangent()
    s.adjoint_step(s.state_buffer, lam1, ref, None)
    s.adjoint_step_noalloc(s.state_buffer, lam1, got, None)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    s.close()


def test_noalloc_rejects_grids_beyond_the_scratch():
    """512^2 needs 29 MiB of work rows, beyond the 16 MiB scratch: EINVAL
    with a message naming the limit, before any launch."""
    s, lam1 = _case(512, 512, 2, 0.71, "periodic", "f32", 8)
    lam = s.new_cotangent()
    with pytest.raises(DVBMError) as e:
        s.adjoint_step_noalloc(s.state_buffer, lam1, lam, None)
    assert e.value.code == dvbm.DVBM_EINVAL and "149211 cells" in str(e.value)
    s.close()
