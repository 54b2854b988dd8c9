"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and its host-only entry points behave (no GPU needed)."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dvbm.h")
LIB = os.path.join(ROOT, "paper_2510_04197_amd", "libdvbm.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libdvbm.so not built")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dvbm_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    names = declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_binding_declares_every_symbol():
    from paper_2510_04197_amd import dvbm
    assert set(declared_symbols()) == set(dvbm.SIGNATURES)


@pytest.mark.parametrize("split,n1", ((1, 4), (2, 5)))
def test_library_velocity_set_matches_numpy_quadrature(split, n1):
    from paper_2510_04197_amd import velocity_set
    v, w = velocity_set(split, R=1.3, T_ref=0.7)
    x, wx = np.polynomial.hermite_e.hermegauss(n1)
    wx = wx / math.sqrt(2 * math.pi)
    c = math.sqrt(1.3 * 0.7)
    np.testing.assert_allclose(v[:, 0], c * np.repeat(x, n1), atol=1e-14)
    np.testing.assert_allclose(v[:, 1], c * np.tile(x, n1), atol=1e-14)
    np.testing.assert_allclose(w, np.repeat(wx, n1) * np.tile(wx, n1), rtol=1e-13)


def test_sizes_and_defaults():
    from paper_2510_04197_amd import dvbm
    lib = dvbm.load_library()
    p = dvbm.make_params(100, 30, split=2, storage="f32")
    assert lib.dvbm_pitch(ctypes.byref(p)) == 128
    assert lib.dvbm_buffer_bytes(ctypes.byref(p)) == 2 * 25 * 30 * 128 * 4
    p16 = dvbm.make_params(100, 30, split=1, storage="bf16_dev")
    assert lib.dvbm_buffer_bytes(ctypes.byref(p16)) == 2 * 16 * 30 * 128 * 2
    d = dvbm.Params()
    lib.dvbm_params_default(ctypes.byref(d))
    assert (d.split, d.gamma, d.Pr, d.beta, d.cfl, d.tau_ref) == (2, 1.4, 0.71, 1.2, 0.01, 5e-5)
    assert lib.dvbm_num_populations(1) == 16 and lib.dvbm_num_populations(2) == 25
    assert lib.dvbm_num_populations(3) == dvbm.DVBM_EINVAL


@pytest.mark.parametrize("field,value", [("nx", 3), ("nx", 0), ("ny", 0), ("ny", -5), ("split", 3), ("gamma", 2.5),
                                         ("beta", 0.9), ("Pr", 0.0), ("storage", 7), ("tau_ref", -1.0),
                                         ("kernel", 4), ("kernel", -1), ("dx", 0.0), ("bc_x", 2), ("visc_mode", 2),
                                         ("ny", 1 << 28)])
def test_invalid_parameters_rejected_before_any_device_work(field, value):
    from paper_2510_04197_amd import dvbm
    lib = dvbm.load_library()
    p = dvbm.make_params(16, 16)
    setattr(p, field, value)
    assert lib.dvbm_buffer_bytes(ctypes.byref(p)) == 0
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(256)
    rc = lib.dvbm_init(ctypes.byref(p), dummy, dummy, dummy, dummy, dummy, ctypes.c_void_p(512), dummy, None,
                       ctypes.byref(h))
    assert rc == dvbm.DVBM_EINVAL
    assert lib.dvbm_last_error().decode().startswith("dvbm_init:")


def test_null_handle_calls_fail_cleanly():
    from paper_2510_04197_amd import dvbm
    lib = dvbm.load_library()
    assert lib.dvbm_step(None, 1) == dvbm.DVBM_EINVAL
    assert lib.dvbm_moments(None, None, None, None, None, None) == dvbm.DVBM_EINVAL
    assert lib.dvbm_set_state_index(None, 0) == dvbm.DVBM_EINVAL
    lib.dvbm_destroy(None)


def test_sweep_kernel_distribution_limit():
    from paper_2510_04197_amd import dvbm
    lib = dvbm.load_library()
    for storage in ("f64", "f32", "bf16_dev", "fp16_dev", "f32_dev"):
        p = dvbm.make_params(16, 16, storage=storage, kernel="sweep")
        assert lib.dvbm_buffer_bytes(ctypes.byref(p)) > 0, storage
    # float32 deviations take float32's bytes
    sizes = [lib.dvbm_buffer_bytes(ctypes.byref(dvbm.make_params(100, 30, storage=st))) for st in ("f32", "f32_dev")]
    assert sizes[0] == sizes[1]
    # a float32 distribution above 2 GiB: 25 planes x 5120 x 4224 cells x 4 B
    p = dvbm.make_params(5120, 4224, storage="f32", kernel="sweep")
    assert lib.dvbm_buffer_bytes(ctypes.byref(p)) == 0
    # a float64 distribution of 2.05 GiB: its stores go through one buffer resource per plane
    p = dvbm.make_params(3584, 3072, storage="f64", kernel="sweep")
    assert lib.dvbm_buffer_bytes(ctypes.byref(p)) > 0
    p = dvbm.make_params(5120, 4224, storage="f32", kernel="cell")
    assert lib.dvbm_buffer_bytes(ctypes.byref(p)) > 0


def test_bench_refuses_more_than_one_gpu():
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU only" in line["error"]


def test_step_kernel_name_follows_the_auto_rule():
    """bench.py names the kernel the library's AUTO rule launches (for the roofline line)."""
    import sys
    from types import SimpleNamespace
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import bench
    big, small, huge = SimpleNamespace(nx=4096, ny=4096), SimpleNamespace(nx=512, ny=512), SimpleNamespace(nx=6528, ny=6528)
    assert bench.step_kernel_name("f32", big) == "k_collide_advect_sweep"
    assert bench.step_kernel_name("f64", big) == "k_collide_advect_sweep"
    assert bench.step_kernel_name("f64", small) == "k_collide_advect_lds"
    assert bench.step_kernel_name("f32", small) == "k_collide_advect"
    assert bench.step_kernel_name("f32", huge) == "k_collide_advect"  # distribution above 2 GiB
    assert bench.step_kernel_name("bf16_dev", huge) == "k_collide_advect_sweep"


def test_stream_probe_rejects_bad_arguments_on_the_host():
    """dvbm_stream_probe validates mode, width, size, pointers and alignment
    before any launch (EINVAL, no GPU needed)."""
    from paper_2510_04197_amd import dvbm
    lib = dvbm.load_library()
    buf = ctypes.c_void_p(4096)  # never dereferenced: every call below fails its checks first
    for mode, width, nbytes in ((3, 16, 64), (7, 16, 64), (-1, 16, 64), (0, 8, 64), (0, 16, 0), (0, 16, 24),
                                (0, 4, 6)):
        assert lib.dvbm_stream_probe(buf, buf, nbytes, mode, width, None) == dvbm.DVBM_EINVAL
    assert lib.dvbm_stream_probe(None, buf, 64, 0, 16, None) == dvbm.DVBM_EINVAL
    assert lib.dvbm_stream_probe(buf, None, 64, 2, 16, None) == dvbm.DVBM_EINVAL
    assert lib.dvbm_stream_probe(ctypes.c_void_p(4100), buf, 64, 0, 16, None) == dvbm.DVBM_EINVAL
    assert b"dvbm_stream_probe" in lib.dvbm_last_error()


def test_new_entry_points_reject_null_handles():
    from paper_2510_04197_amd import dvbm
    lib = dvbm.load_library()
    p = ctypes.c_void_p(4096)
    assert lib.dvbm_limiter_signature(None, p, p) == dvbm.DVBM_EINVAL
    assert lib.dvbm_adjoint_step_noalloc(None, p, p, p, None) == dvbm.DVBM_EINVAL


def test_rollout_rejects_bad_step_counts():
    """rollout_temperature refuses nsteps < 1 and a checkpoint interval K < 1
    (K = 0 would never advance) before it touches a device."""
    import torch

    from paper_2510_04197_amd import rollout_temperature

    T0 = torch.ones((4, 4), dtype=torch.float64)
    one = torch.tensor(1.0, dtype=torch.float64)
    for nsteps, K in ((0, 10), (10, 0), (5, -1)):
        with pytest.raises(ValueError, match="nsteps >= 1 and a checkpoint interval K >= 1"):
            rollout_temperature(T0, one, one, None, None, None, nsteps, K=K, dt=1e-3)


def test_binding_checks_every_tensor_before_the_call():
    """Pointers reach the library without sizes of their own, so the binding refuses a tensor on another
    device, a strided view, a wrong dtype or shape, and a buffer shorter than the call needs."""
    import torch

    from paper_2510_04197_amd import dvbm
    cpu = torch.device("cpu")
    t = torch.zeros((2, 5, 3, 4), dtype=torch.float64)
    assert dvbm._need(t, "t", cpu, nbytes=t.numel() * 8, dtype=torch.float64, shape=(2, 5, 3, 4)) is t
    with pytest.raises(TypeError):
        dvbm._need(np.zeros(4), "t", cpu)
    with pytest.raises(ValueError, match="must be on"):
        dvbm._need(t, "t", torch.device("cuda"))
    with pytest.raises(ValueError, match="contiguous"):
        dvbm._need(t.transpose(2, 3), "t", cpu)
    with pytest.raises(TypeError, match="float32"):
        dvbm._need(t, "t", cpu, dtype=torch.float32)
    with pytest.raises(ValueError, match="shape"):
        dvbm._need(t, "t", cpu, shape=(2, 5, 4, 3))
    with pytest.raises(ValueError, match="fewer"):
        dvbm._need(t, "t", cpu, nbytes=t.numel() * 8 + 1)
