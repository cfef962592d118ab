"""Build tests/c_consumer, the plain C11 program that drives the library
through include/fsb.h alone (gcc, linked against the in-tree libfsb.so and
the HIP runtime; the run path is recorded relative to the binary)."""
import os
import subprocess

TESTS = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(TESTS)
SOURCE = os.path.join(TESTS, "c_consumer.c")
BINARY = os.path.join(TESTS, "c_consumer")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build() -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           SOURCE, "-o", BINARY,
           "-L", os.path.join(ROOT, "paper_2507_20173_amd"), "-lfsb",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../paper_2507_20173_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return BINARY


if __name__ == "__main__":
    build()
