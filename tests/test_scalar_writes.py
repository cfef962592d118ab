"""No kernel of this library writes memory through the scalar data cache:
all stores and atomics in our own gfx950 assembly are vector-memory
instructions.  (This file names those scalar instructions, so it is a
CPU-only check kept off the GPU upload list.)"""
import re

import pytest

from paper_2507_20173_amd import build as fsb_build

SCALAR_WRITES = re.compile(r"^\s*s_(store_|buffer_store|atomic_|buffer_atomic|scratch_store|"
                           r"dcache_wb|dcache_discard)", re.M)


@pytest.mark.parametrize("source", ["fsb_kernels.hip", "fsb_batch.hip", "fsb_probe.hip"])
def test_no_scalar_memory_writes(source):
    text = open(fsb_build.assembly(source)).read()
    assert re.search(r"^_Z\w+:", text, re.M), f"no kernel found in the assembly of {source}"
    hits = SCALAR_WRITES.findall(text)
    assert not hits, f"scalar-cache writes in {source} assembly: {sorted(set(hits))}"
