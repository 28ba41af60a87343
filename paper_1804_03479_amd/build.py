"""Build libmhd.so for gfx950 in place with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmhd.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # no packed-FP32 instructions in generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # float division and square root as reciprocal / v_sqrt (a few ulp)
         # instead of the correctly rounded multi-instruction sequences: the
         # float stage kernels are bound by VALU issue; double is unaffected
         "-fno-hip-fp32-correctly-rounded-divide-sqrt",
         # float denormals flush to zero (double keeps them): the fast
         # reciprocal and square root then need no frexp / ldexp range
         # scaling, 8-10 % fewer VALU instructions in the flux stages; no
         # float value of the update comes near 1e-38
         "-fgpu-flush-denormals-to-zero",
         "-Wno-unused-result", "-Wno-unused-value",
         "-I" + os.path.join(ROOT, "include")]
SOURCES = ["mhd_api.hip"]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + srcs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libmhd.so")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
