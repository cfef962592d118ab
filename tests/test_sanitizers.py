"""The CPU-side code under the address and undefined-behaviour sanitizers:
the oracle (every entry point on small schools, tests/oracle_sanitize.c) and
the library's pure host code (configuration, column and workspace checks,
layouts, the mapping of refused persistent launches, the batch's school and
tuning checks, tile and chunk tables, autotuner cache lines;
tests/host_checks.cpp).  Built with gcc/g++ on the host; no GPU code is
involved."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ROCM = "/opt/rocm"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
    return r


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    _run(["gcc", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", *SAN,
          "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "fsb_oracle.c"),
          os.path.join(HERE, "oracle_sanitize.c"), "-o", exe, "-lm"])
    r = _run([exe], env=ENV)
    assert "oracle checks ok" in r.stdout
    assert "runtime error" not in r.stderr


@pytest.mark.skipif(not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime_api.h")),
                    reason="HIP headers not installed")
def test_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_checks")
    csrc = os.path.join(ROOT, "paper_2507_20173_amd", "csrc")
    _run([shutil.which("g++") or "g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", *SAN,
          "-I", os.path.join(ROOT, "include"), "-I", csrc, "-I", os.path.join(ROCM, "include"),
          os.path.join(HERE, "host_checks.cpp"), "-o", exe,
          "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    r = _run([exe], env=ENV)
    assert "host checks ok" in r.stdout
    assert "runtime error" not in r.stderr
