"""Build libdiffreach.so for gfx950 with hipcc (in-tree, into ``_lib/``).

The chain kernels are instantiated per chain type and tile count in separate
translation units (``csrc/instances.hip`` compiled once per instance set), which are
compiled in parallel with the host side (``csrc/diffreach.hip``) and linked into one
shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "_lib", "libdiffreach.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
INSTANCES = [(t, nt) for t in ("float", "double") for nt in (2, 4, 6, 8, 16)]
# Up to 128 neurons (and in the host unit's kernels: the flowpipes, the contraction) the
# matrix products keep their results in the architectural registers: the VALU work between
# two products then reads them without accumulator-register moves (measured: 1.5-2% faster
# bound, joint, reach-gradient and held-input flowpipe kernels, fewer registers, no spills).
# The 256-wide units keep the compiler's default (the option does not build them).
MFMA_VGPR_FORM = ["-mllvm", "-amdgpu-mfma-vgpr-form"]
MFMA_VGPR_FORM_NT = (2, 4, 6, 8)
HEADERS = ["kernels.hpp", "bound_kernels.hpp", "aux_kernels.hpp", "joint_kernels.hpp", "grad_kernels.hpp", "ct_flow.hpp", "ct_kernels.hpp",
           "instances.h"]


def _units():
    """(object path, source, extra flags) of every translation unit."""
    units = [(os.path.join(OBJ, "diffreach.o"), os.path.join(CSRC, "diffreach.hip"), list(MFMA_VGPR_FORM))]
    for t, nt in INSTANCES:
        units.append((os.path.join(OBJ, f"inst_{t}_{nt}.o"), os.path.join(CSRC, "instances.hip"),
                      [f"-DDR_T={t}", f"-DDR_NT={nt}"] + (MFMA_VGPR_FORM if nt in MFMA_VGPR_FORM_NT else [])))
    return units


def _stale(obj, src):
    if not os.path.exists(obj):
        return True
    deps = [src] + [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(ROOT, "include", "diffreach.h")]
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, incremental: bool = False, jobs: int = 0) -> str:
    """Compile every translation unit (all of them unless ``incremental``) and link."""
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    os.makedirs(OBJ, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    todo = [u for u in _units() if not incremental or _stale(u[0], u[1])]

    def compile_one(u):
        obj, src, extra = u
        cmd = [hipcc, *HIPCC_FLAGS, *inc, *extra, "-c", "-o", obj + ".tmp", src]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode == 0:
            os.replace(obj + ".tmp", obj)
        return u, res

    jobs = jobs or min(len(todo), os.cpu_count() or 4, 16) or 1
    failed = []
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for (obj, _, _), res in ex.map(compile_one, todo):
            if res.returncode != 0:
                failed.append((obj, res.stdout + res.stderr))
    if failed:
        for obj, msg in failed:
            sys.stderr.write(f"--- {obj}\n{msg}\n")
        raise RuntimeError("hipcc failed to compile libdiffreach.so")
    tmp = OUT + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [u[0] for u in _units()]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to link libdiffreach.so")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT, f"({len(todo)} translation units compiled)")
    return OUT


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
