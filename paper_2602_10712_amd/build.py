"""Builds libsrp.so in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsrp.so")
OBJDIR = os.path.join(HERE, "_build")
VALU_RATES = os.path.join(HERE, "valu_rates")

SOURCES = ["srp_api.cpp", "bvh_build.cpp", "ray_stats.cpp", "trace_kernels.hip", "adjoint_kernels.hip", "surface_kernels.hip", "bvh_gpu.hip", "mlp_api.cpp", "mlp_kernels.hip", "mlp_infer.hip",
           "orbit.cpp", "attitude_kernels.hip", "attitude_api.cpp", "noalloc.hip", "ensemble.hip", "edge_kernels.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          "-I", os.path.join(HERE, "..", "include")]
# gfx950 only; packed-FP32 instructions are disabled for all device code
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]
# per-source device options: the fused MLP keeps its MFMA accumulators in architectural VGPRs (the
# SiLU epilogue then reads them without AGPR moves; activations may live in AGPRs as B operands)
EXTRA = {"mlp_infer.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _compile(src: str, obj: str) -> None:
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip", *DEVICE, *EXTRA.get(src, []), *COMMON, "-c", path, "-o", obj]
    else:
        cmd = [HIPCC, "--offload-arch=gfx950", *COMMON, "-D__HIP_PLATFORM_AMD__", "-c", path, "-o", obj]
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(OBJDIR, exist_ok=True)
    objs = [os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o") for src in SOURCES]
    if verbose:
        print("hipcc", " ".join(SOURCES), file=sys.stderr)
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        for f in [pool.submit(_compile, src, obj) for src, obj in zip(SOURCES, objs)]:
            f.result()
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, "-shared", "--offload-arch=gfx950", "-fPIC", "-o", tmp, *objs], check=True)
    os.replace(tmp, LIB)
    # stand-alone measurement of the vector ALU's issue rates (the ALU roofline's ceilings)
    subprocess.run([HIPCC, "-x", "hip", *DEVICE, "-O3", "-std=c++17", os.path.join(CSRC, "valu_rates.hip"), "-o",
                    VALU_RATES], check=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
