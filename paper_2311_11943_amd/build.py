"""Build libcqr.so (HIP kernels + C ABI) for gfx950 in the package folder.

    python -m paper_2311_11943_amd.build

Always recompiles.  Every HIP source gets the packed-FP32 code-generation
feature switched off (hipcc prints a harmless warning about it for the host
pass).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libcqr.so")

SOURCES = ["cqr_gemm.hip", "cqr_code.hip", "cqr_solve.hip", "cqr_adjoint.hip", "cqr_api.cpp"]
ARCH = os.environ.get("CQR_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          f"-I{INCLUDE}", f"-I{CSRC}"]
HIP_ONLY = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-munsafe-fp-atomics",
            # MFMA accumulators in VGPRs: avoids per-iteration AGPR copies of
            # loop-carried accumulators
            "-mllvm", "-amdgpu-mfma-vgpr-form=1"]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    with tempfile.TemporaryDirectory(prefix="cqr_build_") as tmp:
        objs = []
        for src in SOURCES:
            path = os.path.join(CSRC, src)
            obj = os.path.join(tmp, src + ".o")
            if src.endswith(".hip"):
                cmd = [hipcc, "-c", "-x", "hip", path, "-o", obj] + COMMON + HIP_ONLY
            else:
                cmd = [hipcc, "-c", path, "-o", obj] + COMMON + ["-D__HIP_PLATFORM_AMD__"]
            if verbose:
                print(" ".join(cmd), flush=True)
            res = subprocess.run(cmd, capture_output=True, text=True)
            err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
            if res.returncode != 0:
                raise RuntimeError(f"compiling {src} failed:\n{err}")
            if err.strip() and verbose:
                print(err, file=sys.stderr)
            objs.append(obj)
        tmp_lib = LIB + ".tmp"
        cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp_lib] + objs
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"linking failed:\n{res.stderr}")
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
