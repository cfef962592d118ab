"""ctypes view of the plain C FSB oracle (``fsb_oracle.c``).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the tests, the smoke check and
the benchmark's CPU-baseline leg import this module.  It shares nothing with
the GPU library; see ``fsb_oracle.h`` for what the oracle computes and for the
readings of the paper (arXiv 2507.20173) it takes.

The school is a numpy structured array with the paper's Fish fields
(Sec. 2.1.1): ``x, y, weight, prevObjective, currentObjective``.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "fsb_oracle.c")
LIBRARY = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-fPIC", "-shared"]

FISH = np.dtype([("x", "<f4"), ("y", "<f4"), ("weight", "<f4"),
                 ("prevObjective", "<f4"), ("currentObjective", "<f4")])
FISH_F64 = np.dtype([("x", "<f8"), ("y", "<f8"), ("weight", "<f8"),
                     ("prevObjective", "<f8"), ("currentObjective", "<f8")])

DOMAIN_SWIM = 0
DOMAIN_INIT = 1


def build(source: str = SOURCE, output: str = LIBRARY) -> str:
    """Compile the oracle with gcc (binary32 SSE arithmetic, no contraction)."""
    cmd = ["gcc", *CFLAGS, "-I", HERE, "-o", output + ".tmp", source, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(output + ".tmp", output)
    return output


class _Config(ctypes.Structure):
    _fields_ = [("numFish", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("pondHalf", ctypes.c_float), ("swimStep", ctypes.c_float),
                ("initWeightLo", ctypes.c_float), ("initWeightHi", ctypes.c_float),
                ("weightMin", ctypes.c_float), ("weightMax", ctypes.c_float),
                ("swimRule", ctypes.c_uint32)]


# Swim rules (flags; 0 = the plain random swim)
SWIM_GREEDY = 1    # keep a move only if it brings the fish closer to the centre
SWIM_WEIGHTED = 2  # step scaled by weightMin / weight


@dataclasses.dataclass
class Config:
    """Simulation fields of the paper's Config structure (Sec. 2.1.3)."""
    numFish: int
    seed: int = 0
    pondHalf: float = 100.0      # 200x200 pond (Sec. 2.1.2), centred at 0
    swimStep: float = 0.1
    initWeightLo: float = 1.0
    initWeightHi: float = 2.0
    weightMin: float = 1.0
    weightMax: float = 4.0
    swimRule: int = 0            # SWIM_* flags

    def c(self) -> _Config:
        return _Config(self.numFish, self.seed, self.pondHalf, self.swimStep,
                       self.initWeightLo, self.initWeightHi, self.weightMin,
                       self.weightMax, self.swimRule)


_P = ctypes.c_void_p


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """One loaded copy of the oracle library (a path lets tests load a copy
    built from a deliberately altered source)."""

    def __init__(self, path: str | None = None):
        if path is None:
            path = LIBRARY
            if not os.path.exists(path):
                build()
        self.path = path
        lib = ctypes.CDLL(path)
        self._lib = lib
        u32, u64 = ctypes.c_uint32, ctypes.c_uint64
        lib.oracle_philox_many.argtypes = [u64, _P, _P, _P]
        lib.oracle_unit_many.argtypes = [u64, _P, _P, _P]
        lib.oracle_unit.argtypes = [u32]
        lib.oracle_unit.restype = ctypes.c_float
        lib.oracle_signed_unit.argtypes = [u32]
        lib.oracle_signed_unit.restype = ctypes.c_float
        lib.oracle_fish_words.argtypes = [u64, u64, u32, u32, _P, _P]
        lib.oracle_init.argtypes = [_P, _P]
        lib.oracle_step.argtypes = [_P, _P, u64, _P, _P, _P]
        lib.oracle_step_displaced.argtypes = [_P, _P, _P, _P, _P, _P, _P]
        lib.oracle_run.argtypes = [_P, _P, u64, u64, _P, _P, _P]
        lib.oracle_follow_fish.argtypes = [_P, u64, u64, u64, _P]
        lib.oracle_follow_fish.restype = ctypes.c_int
        lib.oracle_follow_fish_fed.argtypes = [_P, u64, u64, u64, _P, _P]
        lib.oracle_follow_fish_fed.restype = ctypes.c_int
        lib.oracle_barycentre_sums.argtypes = [_P, u64, _P, _P]
        lib.oracle_init_f64.argtypes = [_P, _P]
        lib.oracle_step_f64.argtypes = [_P, _P, u64, _P, _P]
        lib.oracle_step_displaced_f64.argtypes = [_P, _P, _P, _P, _P, _P]
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int

    # ---- random numbers --------------------------------------------------
    def philox(self, counters, keys) -> np.ndarray:
        """Philox4x32-10 of each (counter[4], key[2]) row; returns (n, 4)."""
        c = np.ascontiguousarray(np.asarray(counters, dtype=np.uint32).reshape(-1, 4))
        k = np.ascontiguousarray(np.asarray(keys, dtype=np.uint32).reshape(-1, 2))
        assert c.shape[0] == k.shape[0]
        out = np.empty_like(c)
        self._lib.oracle_philox_many(c.shape[0], _ptr(c), _ptr(k), _ptr(out))
        return out

    def units(self, words) -> tuple[np.ndarray, np.ndarray]:
        r = np.ascontiguousarray(np.asarray(words, dtype=np.uint32).ravel())
        u = np.empty(r.shape, np.float32)
        v = np.empty(r.shape, np.float32)
        self._lib.oracle_unit_many(r.size, _ptr(r), _ptr(u), _ptr(v))
        return u, v

    def fish_words(self, seed: int, fish: int, sub: int, domain: int):
        a, b = ctypes.c_uint32(), ctypes.c_uint32()
        self._lib.oracle_fish_words(seed, fish, sub, domain, ctypes.byref(a),
                                    ctypes.byref(b))
        return a.value, b.value

    # ---- binary32 school ---------------------------------------------------
    def init(self, cfg: Config) -> np.ndarray:
        school = np.zeros(cfg.numFish, FISH)
        c = cfg.c()
        self._lib.oracle_init(ctypes.byref(c), _ptr(school))
        return school

    def step(self, cfg: Config, school: np.ndarray, t: int):
        """One iteration in place; returns (maxDiff, sums[3], absSums[3])."""
        assert school.dtype == FISH and school.flags.c_contiguous
        assert school.size == cfg.numFish
        m = np.zeros(1, np.float32)
        s = np.zeros(3, np.float64)
        a = np.zeros(3, np.float64)
        c = cfg.c()
        self._lib.oracle_step(ctypes.byref(c), _ptr(school), t, _ptr(m),
                              _ptr(s), _ptr(a))
        return m[0], s, a

    def step_displaced(self, cfg: Config, school: np.ndarray, dx, dy):
        assert school.dtype == FISH and school.size == cfg.numFish
        dx = np.ascontiguousarray(dx, np.float32)
        dy = np.ascontiguousarray(dy, np.float32)
        m = np.zeros(1, np.float32)
        s = np.zeros(3, np.float64)
        a = np.zeros(3, np.float64)
        c = cfg.c()
        self._lib.oracle_step_displaced(ctypes.byref(c), _ptr(school), _ptr(dx),
                                        _ptr(dy), _ptr(m), _ptr(s), _ptr(a))
        return m[0], s, a

    def run(self, cfg: Config, school: np.ndarray, t0: int, n_steps: int,
            with_sums: bool = True):
        """Iterations t0..t0+n_steps-1 in place; per-step maxDiff, sums,
        absSums (the latter two None without ``with_sums``)."""
        assert school.dtype == FISH and school.size == cfg.numFish
        m = np.zeros(n_steps, np.float32)
        s = np.zeros((n_steps, 3), np.float64) if with_sums else None
        a = np.zeros((n_steps, 3), np.float64) if with_sums else None
        c = cfg.c()
        self._lib.oracle_run(ctypes.byref(c), _ptr(school), t0, n_steps, _ptr(m),
                             _ptr(s) if with_sums else None,
                             _ptr(a) if with_sums else None)
        return m, s, a

    def follow_fish(self, cfg: Config, fish: int, t0: int, t1: int,
                    state: np.ndarray) -> np.ndarray:
        """Positions/objectives of one fish after iterations t0..t1-1, from
        its record ``state`` (a FISH scalar or 1-element array) at t0."""
        f = np.array(state, dtype=FISH).reshape(1).copy()
        c = cfg.c()
        if self._lib.oracle_follow_fish(ctypes.byref(c), fish, t0, t1, _ptr(f)) != 0:
            raise ValueError("under the weighted swim rule a fish cannot be followed alone")
        return f[0]

    def follow_fish_fed(self, cfg: Config, fish: int, t0: int, t1: int, state: np.ndarray,
                        max_diff) -> np.ndarray:
        """One fish's whole record after iterations t0..t1-1, its weight fed
        with the given school maxima max_diff[t1 - t0] (eat(), Sec. 2.3.2)."""
        f = np.array(state, dtype=FISH).reshape(1).copy()
        m = np.ascontiguousarray(max_diff, dtype=np.float32)
        if m.size != t1 - t0:
            raise ValueError("one maximum per iteration")
        c = cfg.c()
        if self._lib.oracle_follow_fish_fed(ctypes.byref(c), fish, t0, t1, _ptr(m), _ptr(f)) != 0:
            raise ValueError("under the weighted swim rule a fish cannot be followed alone")
        return f[0]

    def barycentre_sums(self, school: np.ndarray):
        s = np.zeros(3, np.float64)
        a = np.zeros(3, np.float64)
        self._lib.oracle_barycentre_sums(_ptr(school), school.size, _ptr(s), _ptr(a))
        return s, a

    # ---- binary64 drift variant -----------------------------------------
    def init_f64(self, cfg: Config) -> np.ndarray:
        school = np.zeros(cfg.numFish, FISH_F64)
        c = cfg.c()
        self._lib.oracle_init_f64(ctypes.byref(c), _ptr(school))
        return school

    def step_f64(self, cfg: Config, school: np.ndarray, t: int):
        m = np.zeros(1, np.float64)
        s = np.zeros(3, np.float64)
        c = cfg.c()
        self._lib.oracle_step_f64(ctypes.byref(c), _ptr(school), t, _ptr(m), _ptr(s))
        return m[0], s

    def step_displaced_f64(self, cfg: Config, school: np.ndarray, dx, dy):
        dx = np.ascontiguousarray(dx, np.float64)
        dy = np.ascontiguousarray(dy, np.float64)
        m = np.zeros(1, np.float64)
        s = np.zeros(3, np.float64)
        c = cfg.c()
        self._lib.oracle_step_displaced_f64(ctypes.byref(c), _ptr(school), _ptr(dx),
                                            _ptr(dy), _ptr(m), _ptr(s))
        return m[0], s

    # ---- threads -----------------------------------------------------------
    def set_threads(self, n: int) -> None:
        self._lib.oracle_set_threads(n)

    def max_threads(self) -> int:
        return self._lib.oracle_max_threads()


_DEFAULT: Oracle | None = None


def default() -> Oracle:
    """The oracle built from the committed source (built on first use)."""
    global _DEFAULT
    if _DEFAULT is None:
        _DEFAULT = Oracle()
    return _DEFAULT
