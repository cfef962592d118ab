"""Build libfsb.so (HIP kernels + C ABI) for gfx950, in-tree.

    python -m paper_2507_20173_amd.build

Floating-point flags are part of the contract: every binary32 operation is
rounded on its own (-ffp-contract=off), sqrtf and division are correctly
rounded, and denormals are kept.  Packed-FP32 instructions are disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBRARY = os.path.join(PKG, "libfsb.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I", INCLUDE, "-I", CSRC]
DEVICE = [f"--offload-arch={ARCH}", "-ffp-contract=off",
          "-fhip-fp32-correctly-rounded-divide-sqrt",
          "-fno-gpu-flush-denormals-to-zero", "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
SOURCES = ["fsb_kernels.hip", "fsb_batch.hip", "fsb_probe.hip", "fsb_api.cpp", "fsb_batch_api.cpp"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(output: str = LIBRARY, extra: list[str] | None = None) -> str:
    """Compile every source (in parallel) and link the shared library (always
    rebuilds)."""
    from concurrent.futures import ThreadPoolExecutor

    build_dir = os.path.join(PKG, "_build")
    os.makedirs(build_dir, exist_ok=True)
    jobs = []
    for src in SOURCES:
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        jobs.append(([HIPCC, *COMMON, *DEVICE, *(extra or []), *lang, "-c",
                      os.path.join(CSRC, src), "-o", obj], obj))
    with ThreadPoolExecutor(max_workers=len(jobs)) as pool:
        list(pool.map(_run, [cmd for cmd, _ in jobs]))
    objs = [obj for _, obj in jobs]
    tmp = output + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, output)
    return output


def assembly(source: str = "fsb_kernels.hip") -> str:
    """AMD GCN assembly of one of this library's own sources (for checking
    that the float path has no fused multiply-adds)."""
    out = os.path.join(PKG, "_build", os.path.splitext(source)[0] + ".s")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    _run([HIPCC, *COMMON, *DEVICE, "-x", "hip", "--cuda-device-only", "-S",
          os.path.join(CSRC, source), "-o", out])
    return out


if __name__ == "__main__":
    build()
    if "--asm" in sys.argv:
        print(assembly())
