"""Build libnsp.so, the gfx950 HIP library behind the C ABI in include/nsp.h."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libnsp.so")
SOURCES = [os.path.join(CSRC, f) for f in ("nsp_kernels.hip", "nsp_adjoint.hip", "nsp_api.hip")]
HEADERS = [os.path.join(CSRC, "nsp_internal.h"), os.path.join(ROOT, "include", "nsp.h")]

# -packed-fp32-ops: keep the compiler from emitting packed FP32 arithmetic.
# -ffp-contract=off: no multiply-add is fused behind the code's back, so every
# instantiation of a kernel (store modes, tile depths, batch sizes) computes
# the same bits from the same values; batched and single runs stay bitwise
# equal.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libnsp.so (always recompiles)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc] + FLAGS + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libnsp.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
