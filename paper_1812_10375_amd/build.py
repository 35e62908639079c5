"""Builds the gfx950 HIP library ``liblbm_hip.so`` in-tree with hipcc.

Three translation units: the host entry points, the FP32 kernels, and the FP64
kernels.  The FP64 unit is compiled without floating-point contraction so that the
parity path rounds every operation as written.
"""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm_hip.so")

COMMON = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]
UNITS = [
    ("lbm_api.hip", []),
    # FP32 divide and square root at hardware rate (about 1 ulp) in the FP32 path
    ("lbm_f32.hip", ["-fno-hip-fp32-correctly-rounded-divide-sqrt"]),
    ("lbm_f64.hip", ["-ffp-contract=off"]),
    # the surrogate's BF16 matrix-core kernels
    ("mlp.hip", []),
]


def build_library(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    with tempfile.TemporaryDirectory() as tmpd:
        objs = []
        for src, extra in UNITS:
            obj = os.path.join(tmpd, src.replace(".hip", ".o"))
            cmd = [hipcc] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
            subprocess.check_call(cmd, stderr=None if verbose else subprocess.DEVNULL)
            objs.append(obj)
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
        os.replace(tmp, LIB)
    return LIB
