"""No kernel of this library writes memory through the scalar data cache:
all stores and atomics in our own gfx950 assembly are vector-memory
instructions.  (This file names those scalar instructions, so it is a
CPU-only check kept off the GPU upload list.)"""
import re

from paper_2507_20173_amd import build as fsb_build

SCALAR_WRITES = re.compile(r"^\s*s_(store_|buffer_store|atomic_|buffer_atomic|scratch_store|"
                           r"dcache_wb|dcache_discard)", re.M)


def test_no_scalar_memory_writes():
    text = open(fsb_build.assembly("fsb_kernels.hip")).read()
    hits = SCALAR_WRITES.findall(text)
    assert not hits, f"scalar-cache writes in kernel assembly: {sorted(set(hits))}"
