"""Build the gfx950 shared library ``libdvbm.so`` in-tree with hipcc.

Usage: ``python -m paper_2510_04197_amd.build`` (or ``build()`` from Python).
"""

from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libdvbm.so")

HIPCC_FLAGS = [
    "-O3",
    "--offload-arch=gfx950",
    "-std=c++17",
    "-fPIC",
    # never emit packed FP32 VALU instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]

# csrc/dvbm.hip is compiled once as the main unit (C ABI, small kernels) and
# once per split x storage as a kernel unit holding that pair's step and
# adjoint kernels, so that the units compile in parallel.
STORES = ("dvbm::StoreF64", "dvbm::StoreF32", "dvbm::StoreBF16", "dvbm::StoreF16", "dvbm::StoreF32Dev")
PARTS = [(len(STORES) * (split - 1) + k + 1, STORES[k]) for split in (1, 2) for k in range(len(STORES))]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the ROCm toolchain is required to build libdvbm.so")
    return exe


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with exit code {res.returncode}: {' '.join(cmd)}")


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile ``csrc/dvbm.hip`` for gfx950 into ``libdvbm.so``; returns the path."""
    src = os.path.join(CSRC, "dvbm.hip")
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    units = [("main", [])] + [(f"part{n}", [f"-DDVBM_PART={n}", f"-DDVBM_PART_STORE={st}"]) for n, st in PARTS]
    cmds, objs = [], []
    for name, defs in units:
        obj = os.path.join(objdir, f"dvbm_{name}.o")
        objs.append(obj)
        cmds.append([hipcc(), *HIPCC_FLAGS, *defs, "-c", "-o", obj, src])
    workers = jobs or min(len(cmds), max(1, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([hipcc(), "--offload-arch=gfx950", "-fPIC", "-shared", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
