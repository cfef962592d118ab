"""Seeded synthetic workloads (inputs only; none of the method's arithmetic).

The paper draws its school from random number generators (Sec. 2.1.1) and
names no dataset; every workload here is synthetic and fully determined by
its seeds.  Shared by the tests and the benchmark.
"""
from __future__ import annotations

import numpy as np


def log_uniform_school_sizes(n_schools: int, lo: int = 1_000, hi: int = 1_000_000,
                             meta_seed: int = 20250727) -> np.ndarray:
    """School sizes round(exp(ln lo + u (ln hi - ln lo))), u ~ U[0, 1) from
    numpy's PCG64 seeded with `meta_seed`."""
    u = np.random.default_rng(meta_seed).random(n_schools)
    sizes = np.rint(np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))).astype(np.uint64)
    return np.maximum(sizes, 1)


def packed_starts(sizes, align: int = 64) -> np.ndarray:
    """Start of each school in packed columns: consecutive, each rounded up
    to a multiple of `align` fish (64 fish = 256 bytes by default, so a
    wavefront's float4 row never straddles an extra cache line; any multiple
    of 4 is accepted by the library)."""
    sizes = np.asarray(sizes, np.uint64)
    a = np.uint64(align)
    padded = (sizes + a - np.uint64(1)) // a * a
    starts = np.zeros(sizes.size, np.uint64)
    if sizes.size > 1:
        starts[1:] = np.cumsum(padded)[:-1]
    return starts


def school_seeds(n_schools: int, base: int = 0) -> np.ndarray:
    """Per-school Philox keys: school s uses seed base + s."""
    return np.arange(base, base + n_schools, dtype=np.uint64)
