"""Benchmark of the FSB hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: one school of N = 2^24 fish (x, y uniform in the 200x200 pond,
weights in [1, 2], seed 0), advanced by per-iteration launches
(FSB_RUN_PLAIN: the swim pass of the first iteration, then one pipelined pass
per iteration that feeds the previous iteration and swims this one, then the
closing feed pass).  A "step" is one FSB iteration over the whole school:
swim, objective, max |diff|, feeding and barycentre sums.
`value` is fish-updates/s = N * K / wall time of K iterations, with the
school resident in HBM.  Prints ONE JSON line on stdout.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per fish of each plain kernel (float32 columns).
BYTES_PER_FISH = {
    "swim_eval": 8 + 16,   # reads x, y; writes x, y, prev, cur
    "feed_bary": 16 + 4,   # reads prev, w, x, y; writes w (+4: cur, closing a pipelined run)
    "feed_swim": 16 + 16,  # reads x, y, w, prev; writes x, y, w, prev
}
SPLIT_BYTES_PER_FISH_STEP = BYTES_PER_FISH["swim_eval"] + BYTES_PER_FISH["feed_bary"]


def plain_launches(steps: int, split: bool) -> dict:
    """Launches of each plain kernel in a run of `steps` iterations."""
    if split or steps < 2:
        return {"swim_eval": steps, "feed_bary": steps}
    return {"swim_eval": 1, "feed_swim": steps - 1, "feed_bary": 1}


def plain_kernel_bytes(kernel: str, split: bool) -> int:
    """Bytes per fish of one launch of a plain kernel (the feed pass that
    closes a pipelined run also writes cur)."""
    return BYTES_PER_FISH[kernel] + (4 if kernel == "feed_bary" and not split else 0)


def plain_bytes(n: int, steps: int, split: bool = False) -> int:
    """Algorithmic bytes of a plain run of `steps` iterations: 44 B per
    fish-iteration in two passes, or pipelined 24 B (first swim) + 32 B per
    further iteration + 24 B (closing feed, cur included)."""
    split = split or steps < 2
    return n * sum(c * plain_kernel_bytes(k, split)
                   for k, c in plain_launches(steps, split).items())
# Every PROFILE_EVERY-th launch of each kernel is timed by HIP events inside
# the timed region (the plain passes' launches record them themselves; the
# persistent launches are bracketed by them).
PROFILE_EVERY = 8
KERNEL_SOURCE = os.path.join(ROOT, "paper_2507_20173_amd", "csrc", "fsb_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_plain_n16777216.json")
# Vector-ALU instructions per fish-iteration of the deep kernels, from a
# committed SQ_INSTS_VALU counter summary (like the traffic above).
VALU_FILE = os.path.join(ROOT, "profiles", "valu_deep_forms.json")
# Nominal vector-ALU issue rate of MI355X in lane instructions per second:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, i.e. one wave64 instruction per SIMD
# every four cycles (dual issue can exceed it).
VALU_LANE_PEAK = 256 * 4 * 16 * 2.4e9
# The deep kernels a counter run of the persistent forms launches, by school:
# `bench.py --forms fused,registers --fused-steps F` runs each school's timed
# launch of F iterations in one of these instances.
DEEP_COUNTER_KERNELS = {
    "fused_deep_n67108864": ("fused_deep_kernel<4, true, 0u>", 1 << 26),
    "fused_deep_n16777216": ("fused_deep_kernel<4, false, 0u>", 1 << 24),
    "fused_deep_n2097152": ("fused_deep_kernel<8, false, 0u>", 1 << 21),
}
BATCH_DEEP_COUNTER_KERNEL = "batch_deep_kernel<256, 4, true, 8, 0u>"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def valu_digest() -> str:
    """Digest of the code the deep kernels are built from."""
    return code_digest(_csrc("fsb_kernels.hip", "fsb_batch.hip", "fsb_device.hpp",
                             "fsb_sweep.hpp", "fsb_internal.hpp"))


# Plain-VALU ceilings measured by the probe kernels at the start of the run
# (None until then, or when there is no GPU).
MEASURED_VALU = None


def valu_ceiling(waves_per_simd: int = 8, reps: int = 3) -> dict:
    """Measured plain-VALU ceilings: fsb_valu_probe's independent chains of
    v_fma_f32, of Philox4x32-10 calls (v_mad_u64_u32 + v_bitop3_b32) and of
    both mixed, on every SIMD, `waves_per_simd` waves each; the best of `reps`
    launches."""
    import torch

    import paper_2507_20173_amd as fsb

    blocks = 256 * waves_per_simd
    buf = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    out = {"unit": "T lane-instructions/s", "waves_per_simd": waves_per_simd,
           "nominal": VALU_LANE_PEAK / 1e12}
    for name, kind, iters in (("fma", fsb.FSB_PROBE_FMA, 4096),
                              ("philox", fsb.FSB_PROBE_PHILOX, 512),
                              ("mixed", fsb.FSB_PROBE_MIXED, 512)):
        fsb.fsb_valu_probe(kind, blocks, 64, buf)
        best = 0.0
        for _ in range(reps):
            ms, lanes = fsb.fsb_valu_probe(kind, blocks, iters, buf)
            best = max(best, lanes / (ms / 1e3))
        out[name] = best / 1e12
    out["ceiling"] = max(out["fma"], out["philox"], out["mixed"])
    out["note"] = ("single-issue chains of one instruction kind; under such load the clock "
                   "runs near 2.0-2.1 GHz, not 2.4 (GRBM_GUI_ACTIVE cycles per ns), and "
                   "kernels mixing kinds can exceed it by dual issue")
    del buf
    return out


def sweep_ceiling(n: int, reps: int = 3) -> dict:
    """The copy rate of the plain kernels' access pattern on a school of n
    fish: fsb_sweep_probe reads and writes four columns of n floats in place
    once (32 B per fish, the pipelined pass's traffic, without its arithmetic)
    on the plain passes' grid, cached or streamed as the library's footprint
    rule would take them; the best of `reps` launches."""
    import torch

    import paper_2507_20173_amd as fsb

    cols = [torch.zeros(n, dtype=torch.float32, device="cuda") for _ in range(4)]
    streamed = 16 * n > INFINITY_CACHE_MIB << 20
    fsb.fsb_sweep_probe(cols, 0, streamed)
    best = min(fsb.fsb_sweep_probe(cols, 0, streamed) for _ in range(reps))
    del cols
    torch.cuda.empty_cache()
    return {"achieved_GBs": 32 * n / (best / 1e3) / 1e9, "n_fish": n, "streamed": streamed,
            "note": "in-place read and write of four float32 columns, 512 blocks of 256 "
                    "threads, one float4 group per thread per round: the pipelined pass's "
                    "access pattern without its arithmetic"}


def valu_roofline(key: str, fish_iterations: float, kernel_s: float, path: str = VALU_FILE):
    """The "alu" roofline of a deep form: its lane instructions (the committed
    count per fish-iteration, if taken from the current sources) over its
    event-timed kernel time, against the nominal issue rate."""
    try:
        with open(path) as fh:
            v = json.load(fh)
    except OSError:
        return None
    lane = v.get("lane_instructions_per_fish_iteration", {}).get(key)
    if v.get("source_digest") != valu_digest() or lane is None or kernel_s <= 0:
        return None
    achieved = lane * fish_iterations / kernel_s
    measured = MEASURED_VALU["ceiling"] * 1e12 if MEASURED_VALU else None
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_LANE_PEAK / 1e12,
            "unit": "T lane-instructions/s", "frac": achieved / VALU_LANE_PEAK,
            "measured_ceiling": measured / 1e12 if measured else None,
            "frac_of_measured_ceiling": achieved / measured if measured else None,
            "lane_instructions_per_fish_iteration": lane,
            "note": "SQ_INSTS_VALU per fish-iteration from " + os.path.relpath(path, ROOT) +
                    "; peak = 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one wave64 VALU issue "
                    "per SIMD per 4 cycles; dual issue can exceed it)"}


def code_digest(paths) -> str:
    """Digest of the code in the given source files: comments, trailing blanks
    and blank lines are left out, so that rewording a comment does not void
    figures measured on the code."""
    h = hashlib.sha256()
    for path in paths:
        with open(path) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip()).encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


def _csrc(*names):
    return [os.path.join(ROOT, "paper_2507_20173_amd", "csrc", n) for n in names]


def source_digest() -> str:
    """Digest of the code the plain kernels are built from."""
    return code_digest(_csrc("fsb_kernels.hip", "fsb_device.hpp", "fsb_sweep.hpp",
                             "fsb_internal.hpp"))


def measured_traffic(kernel: str, n_fish: int, path: str = TRAFFIC_FILE):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    if it was taken from the current kernel sources."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("source_digest") != source_digest() or t.get("n_fish") != n_fish:
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def plain_run(n: int, steps: int, warmup: int, split: bool = False):
    """Wall time of `steps` plain iterations (FSB_RUN_PLAIN, or fsb_step's two
    passes with split), and each kernel's event-timed duration and rate."""
    import torch

    import paper_2507_20173_amd as fsb

    mode = fsb.FSB_RUN_PLAIN_SPLIT if split else fsb.FSB_RUN_PLAIN
    cfg = fsb.FsbConfig(n_fish=n, seed=0, history_len=1)
    sch = fsb.School(cfg)
    sch.run(warmup, mode)
    sch.sync()
    fsb.fsb_profile_enable(sch.h, PROFILE_EVERY)
    fsb.fsb_kernel_times(sch.h)  # reset counters
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sch.run(steps, mode)
    sch.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    counts, ms = fsb.fsb_kernel_times(sch.h)
    xy, sums = sch.barycentre()
    sch.close()
    kinds = {"swim_eval": fsb.FSB_KERNEL_SWIM_EVAL, "feed_bary": fsb.FSB_KERNEL_FEED_BARY,
             "feed_swim": fsb.FSB_KERNEL_FEED_SWIM}
    kernels = {}
    for name, launches in plain_launches(steps, split).items():
        c = int(counts[kinds[name]])
        avg_s = ms[kinds[name]] / 1e3 / max(c, 1)
        nbytes = plain_kernel_bytes(name, split or steps < 2) * n
        kernels[name] = {"launches": launches, "timed_launches": c, "avg_us": avg_s * 1e6,
                         "share_of_kernel_time": avg_s * launches,
                         "algorithmic_bytes_per_launch": nbytes,
                         "achieved_GBs": nbytes / avg_s / 1e9}
    total = sum(k["share_of_kernel_time"] for k in kernels.values())
    for k in kernels.values():
        k["share_of_kernel_time"] /= total
    return wall, kernels, xy


def dominant(kernels: dict) -> str:
    """The kernel that takes most of a run's kernel time."""
    return max(kernels, key=lambda k: kernels[k]["share_of_kernel_time"])


def run_form(n: int, steps: int, mode: int, warmup: int = 2, swim_rule: int = 0):
    """Wall time of `steps` iterations of one school in the given mode, plus
    the kernels' event-timed durations."""
    import torch

    import paper_2507_20173_amd as fsb

    cfg = fsb.FsbConfig(n_fish=n, seed=0, history_len=1, swim_rule=swim_rule)
    sch = fsb.School(cfg)
    sch.run(warmup, mode)
    sch.sync()
    fsb.fsb_profile_enable(sch.h, 1 if mode == fsb.FSB_RUN_FUSED else PROFILE_EVERY)
    fsb.fsb_kernel_times(sch.h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sch.run(steps, mode)
    sch.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    counts, ms = fsb.fsb_kernel_times(sch.h)
    sch.close()
    del sch
    torch.cuda.empty_cache()
    return wall, counts, ms


# Largest school the register-resident kernel holds on MI355X: 256 blocks of
# 512 threads, four groups of four fish each, plus up to three tail fish.
REGS_MAX_FISH = 4 * 4 * 512 * 256 + 3


DEEP_WIDE_FISH = 5 << 20  # above this the single-school deep kernel runs four iterations per barrier
BATCH_DEEP_DEPTH = 8  # iterations per grid barrier of the batched deep kernel


def deep_depth(n: int) -> int:
    """Iterations per grid barrier of the single-school deep kernel for a
    school of n fish, as the library picks them (include/fsb.h)."""
    forced = os.environ.get("FSB_DEEP_DEPTH", "")
    if forced in ("2", "4", "8"):
        return int(forced)
    return 4 if n > DEEP_WIDE_FISH else 8


def fused_variant(n: int, deep_ok: bool = True) -> str:
    """The variant FSB_RUN_FUSED runs for a school of n fish (deep_ok: the
    compensated sums and no weighted rule, the default configuration)."""
    if deep_ok:
        return "deep"
    if n <= REGS_MAX_FISH:
        return "regs"
    # lean once the 16 B/fish of the 32-byte variant's live columns reach the
    # 256 MiB last-level cache
    return "lean" if n * 16 >= (256 << 20) else "prev"


def persistent_bytes(variant: str, n: int, steps: int) -> int:
    """Algorithmic bytes of one persistent launch of `steps` iterations."""
    if variant == "regs":  # x, y, w read once, all five columns written once
        return n * (12 + 20)
    if variant == "deep":  # prologue reads x, y; 32 B per superstep (x, y, w, cur read and
        # written; the first forms cur instead of reading it, the last also writes prev)
        return n * (8 + 32 * -(-steps // deep_depth(n)))
    if variant == "lean":  # prologue reads x, y; sweeps 24 B; the last also writes prev, cur
        return n * (8 + 24 * steps + 8)
    return n * (20 + 32 * (steps - 1) + 24)  # prologue 20 B, sweeps 32 B, last sweep 24 B


INFINITY_CACHE_MIB = 256
# A school whose five columns (1.25 GiB) and reused columns (1 GiB) are far
# above the Infinity Cache: the plain passes stream it from HBM.
HBM_RESIDENT_FISH = 1 << 26


def cache_residency(n: int) -> dict:
    """How the school's columns compare with the 256 MiB last-level cache
    (MI355X's Infinity Cache): the five columns, and the three (x, y, w) a
    sweep of the persistent kernels keeps live."""
    five, three = 5 * 4 * n / 2**20, 3 * 4 * n / 2**20
    return {"cache_MiB": INFINITY_CACHE_MIB, "columns_MiB": five, "live_columns_MiB": three,
            "columns_fit": five <= INFINITY_CACHE_MIB,
            "live_columns_fit": three <= INFINITY_CACHE_MIB}


def batch_bytes(variant: str, fish: int, steps: int, per_launch: int, launches: int) -> int:
    """Algorithmic bytes of a batched run of `steps` iterations in launches of
    `per_launch` (the last one shorter if it does not divide)."""
    if variant == "lean":  # prologue reads x, y; 24 B per iteration; the last sweep writes prev, cur
        return fish * (16 * launches + 24 * steps)
    if variant == "deep":  # per launch as a single school's: prologue 8 B, 32 B per superstep
        full, rest = divmod(steps, per_launch)
        supersteps = full * -(-per_launch // BATCH_DEEP_DEPTH) + -(-rest // BATCH_DEEP_DEPTH)
        return fish * (8 * launches + 32 * supersteps)
    return fish * (44 * launches + 32 * (steps - launches))  # prologue 20 B, last sweep 24 B


def fused_vs_plain(n: int, steps: int, label: str):
    """The persistent form (every variant, and the one FSB_RUN_FUSED picks)
    against per-iteration launches on the same school."""
    import paper_2507_20173_amd as fsb

    out = {"workload": label, "n_fish": n, "iterations": steps,
           "infinity_cache": cache_residency(n)}
    probe = fsb.School(fsb.FsbConfig(n_fish=n, seed=0, history_len=1))
    us, _ = fsb.fsb_barrier_probe(probe.h, 0, 2000)
    probe.close()
    del probe
    out["barrier_us"] = us
    forms = [("fused", fsb.FSB_RUN_FUSED), ("fused_prev", fsb.FSB_RUN_FUSED_PREV),
             ("fused_lean", fsb.FSB_RUN_FUSED_LEAN)]
    if n <= REGS_MAX_FISH:
        forms.append(("fused_regs", fsb.FSB_RUN_FUSED_REGS))
    for key, mode in forms:
        wall, counts, ms = run_form(n, steps, mode)
        variant = {"fused_prev": "prev", "fused_lean": "lean", "fused_regs": "regs"}.get(
            key, fused_variant(n))
        kernel_s = ms[fsb.FSB_KERNEL_FUSED] / 1e3
        nbytes = persistent_bytes(variant, n, steps)
        per_step = {"lean": 24, "prev": 32, "regs": 32 / steps, "deep": 32 / deep_depth(n)}[variant]
        barriers_per_step = 1.0 / deep_depth(n) if variant == "deep" else 1.0
        out[key] = {"variant": variant, "value": n * steps / wall, "ms_per_step": wall / steps * 1e3,
                    "launches": int(counts[fsb.FSB_KERNEL_FUSED]),
                    "algorithmic_bytes_per_fish_step": per_step,
                    "kernel_achieved_GBs": nbytes / kernel_s / 1e9,
                    "kernel_hbm_frac": nbytes / kernel_s / 1e9 / HBM_PEAK_GBS,
                    "barrier_share": us * barriers_per_step * 1e-3 / (wall / steps * 1e3)}
        if variant == "deep":
            out[key]["iterations_per_barrier"] = deep_depth(n)
            out[key]["lane_sums"] = ("binary64 accumulation of pairwise float32 group totals "
                                     "(not the compensated float32 lanes of the plain path)")
            out[key]["roofline_alu"] = valu_roofline(f"fused_deep_n{n}", n * steps, kernel_s)
        if key == "fused" and steps >= 4:
            # per-iteration cost as the slope between a launch of steps/2 and one
            # of steps iterations (the launch and its prologue drop out)
            half, _, _ = run_form(n, steps // 2, mode)
            out[key]["slope_ms_per_step"] = (wall - half) / (steps - steps // 2) * 1e3
    for key, split in (("plain", False), ("plain_split", True)):
        wp, _, _ = run_form(n, steps, fsb.FSB_RUN_PLAIN_SPLIT if split else fsb.FSB_RUN_PLAIN)
        nb = plain_bytes(n, steps, split)
        out[key] = {"value": n * steps / wp, "ms_per_step": wp / steps * 1e3,
                    "algorithmic_bytes_per_fish_step": nb / (n * steps),
                    "hbm_frac": nb / wp / 1e9 / HBM_PEAK_GBS}
    out["plain"]["launches"] = "pipelined: one per iteration (FSB_RUN_PLAIN)"
    out["plain_split"]["launches"] = "two per iteration (fsb_step, FSB_RUN_PLAIN_SPLIT)"
    out["fused_speedup"] = out["fused"]["value"] / out["plain"]["value"]
    out["fused_speedup_vs_split"] = out["fused"]["value"] / out["plain_split"]["value"]
    return out


def column_reference(sch):
    """Reference values of the last iteration from the columns the kernels
    left behind: binary64 sums (a binary32 product is exact in binary64;
    numpy's pairwise summation adds ~1e-15 relative) and the max of
    |prev - cur| formed in binary32 like the kernels' diff."""
    import numpy as np

    st = sch.state()
    w = st["w"].astype(np.float64)
    wx = w * st["x"].astype(np.float64)
    wy = w * st["y"].astype(np.float64)
    ref = np.array([w.sum(), wx.sum(), wy.sum()])
    den = np.array([np.abs(w).sum(), np.abs(wx).sum(), np.abs(wy).sum()])
    m = np.abs(st["prev"] - st["cur"]).max() if len(w) else np.float32(0)
    return ref, den, m


def checked_iterations(sch, k: int):
    """k single iterations, each checked against its column reference: the
    largest sum error (|got - ref| / sum|terms|) and whether M was exact."""
    import numpy as np

    errs, exact = [], True
    for _ in range(k):
        sch.step()
        _, got = sch.barycentre()
        ref, den, m = column_reference(sch)
        errs.append((np.abs(np.asarray(got) - ref) / den).tolist())
        exact &= bool(sch.max_delta() == m)
    return errs, exact


def column_sums_f64(sch):
    """Binary64 sums of the school's current columns, on the GPU with plain
    torch ops (each binary32 product is exact in binary64; torch's float64
    tree sum adds ~1e-15 relative): (sums[3], sum of |terms|[3])."""
    import torch

    w = sch.cols["w"].double()
    wx = w * sch.cols["x"].double()
    wy = w * sch.cols["y"].double()
    ref = torch.stack([w.sum(), wx.sum(), wy.sum()])
    den = torch.stack([w.abs().sum(), wx.abs().sum(), wy.abs().sum()])
    return ref.cpu().numpy(), den.cpu().numpy()


def precision_form(n: int, steps: int):
    """Compensated (default) vs naive float32-atomic barycentre sums on one
    school: throughput of each over `steps` iterations, and the error of every
    one of those iterations.  The errors come from a second, untimed run of
    the same iterations, one at a time, each record compared with binary64
    sums of the columns that iteration left (a column-based reference, not
    the oracle: the oracle comparison at this size is in the tests); that
    run's records equal the timed run's bit for bit (checked), so the errors
    are those of the timed iterations."""
    import numpy as np
    import torch

    import paper_2507_20173_amd as fsb

    out = {"workload": f"precision form: N=2^{n.bit_length() - 1} fish, {steps} iterations, "
                       "per-iteration launches; compensated float32 lane sums + binary64 block "
                       "combine vs float32 trees + float32 atomicAdd",
           "n_fish": n, "iterations": steps}
    for name, mode in (("compensated", fsb.FSB_REDUCE_COMPENSATED),
                       ("naive_f32_atomics", fsb.FSB_REDUCE_NAIVE_F32)):
        cfg = fsb.FsbConfig(n_fish=n, seed=0, reduce_mode=mode, history_len=steps)
        sch = fsb.School(cfg)
        sch.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sch.run(steps)
        sch.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        timed = sch.history(0, steps)
        sch.close()
        del sch
        torch.cuda.empty_cache()
        # the same iterations again, one at a time, each checked
        sch = fsb.School(cfg)
        errs, exact = [], True
        for t in range(steps):
            sch.step()
            rec = sch.history(t, 1)[0]
            ref, den = column_sums_f64(sch)
            got = np.array([rec["sum_w"], rec["sum_wx"], rec["sum_wy"]])
            errs.append(np.abs(got - ref) / den)
            st_prev, st_cur = sch.cols["prev"], sch.cols["cur"]
            exact &= bool((st_prev - st_cur).abs().max().item() == float(rec["max_delta"]))
        same = sch.history(0, steps).tobytes() == timed.tobytes()
        sch.close()
        del sch
        torch.cuda.empty_cache()
        e = np.array(errs)
        out[name] = {"value": n * steps / wall, "ms_per_step": wall / steps * 1e3,
                     "max_error_per_sum": e.max(0).tolist(),
                     "max_error": float(e.max()), "mean_error": float(e.mean()),
                     "worst_iteration": int(e.max(1).argmax()),
                     "iterations_checked": steps, "max_exact": exact,
                     "records_equal_timed_run": same,
                     "note": "the re-run's records equal the timed run's: these are the timed "
                             "iterations' errors" if same else
                             "float32 atomics add in a different order each run: the re-run is "
                             "a sample of the same distribution, not the timed records",
                     "within_1e-6_gate": bool((e <= 1e-6).all())}
        log(f"precision {name}: max error {e.max():.3e} over {steps} iterations")
    out["error_definition"] = ("|got - ref| / sum|terms| per sum (sum w, sum w*x, sum w*y), every "
                               "iteration; ref = binary64 sums of that iteration's columns "
                               "(column-based reference: exact products, torch float64 sums on "
                               "the GPU)")
    return out


def ablation_form(sizes, checked_steps: int, budget_s: float = 0.5):
    """Construct ablation (Sec. 2.3.2, Experiment 3: reduction clause vs
    critical section) on the plain path: the compensated tree, float32 trees
    with one atomic per block, and the critical mode's one atomic per fish for
    the max and the three sums.  Per school size: time per iteration, the two
    passes' event-timed durations, and the first iterations' errors against
    binary64 sums of their columns (the max must be exact in every mode)."""
    import torch

    import paper_2507_20173_amd as fsb

    modes = (("tree_compensated", fsb.FSB_REDUCE_COMPENSATED),
             ("tree_f32_block_atomics", fsb.FSB_REDUCE_NAIVE_F32),
             ("critical_f32_fish_atomics", fsb.FSB_REDUCE_CRITICAL_F32))
    out = {"workload": "construct ablation: one school, fsb_step's two passes per iteration, seed 0; "
                       "the three reductions of the school max and the barycentre sums",
           "error_definition": "max over the first iterations of |got - ref| / sum|terms| "
                               "(sum w, sum w*x, sum w*y); ref = binary64 sums of the columns"}
    for n in sizes:
        row = {}
        for name, mode in modes:
            sch = fsb.School(fsb.FsbConfig(n_fish=n, seed=0, reduce_mode=mode, history_len=1))
            errs, exact = checked_iterations(sch, checked_steps)
            sch.sync()
            t0 = time.perf_counter()
            sch.step()
            sch.sync()
            one = time.perf_counter() - t0
            steps = int(min(200, max(3, budget_s / max(one, 1e-6))))
            fsb.fsb_profile_enable(sch.h, 1)
            fsb.fsb_kernel_times(sch.h)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            # every mode on fsb_step's two passes (the critical one has no other)
            sch.run(steps, fsb.FSB_RUN_PLAIN_SPLIT)
            sch.sync()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            counts, ms = fsb.fsb_kernel_times(sch.h)
            sch.close()
            del sch
            torch.cuda.empty_cache()
            per = {k: ms[kind] / max(int(counts[kind]), 1) * 1e3
                   for k, kind in (("swim_us", fsb.FSB_KERNEL_SWIM_EVAL),
                                   ("feed_us", fsb.FSB_KERNEL_FEED_BARY))}
            row[name] = {"iterations": steps, "value": n * steps / wall,
                         "ms_per_step": wall / steps * 1e3, **per,
                         "max_exact": exact, "max_error": max(max(e) for e in errs)}
        base = row["tree_compensated"]["ms_per_step"]
        for name in row:
            row[name]["slowdown_vs_tree"] = row[name]["ms_per_step"] / base
        out[f"n={n}"] = row
        log(f"ablation n={n}: " + ", ".join(f"{k} {v['ms_per_step']:.4f} ms"
                                            for k, v in row.items()))
    return out


def rules_form(n: int, steps: int):
    """Cost of the swim rules (greedy, weighted, both) against the plain
    random swim on one school, per-iteration launches and the persistent form
    (the variant FSB_RUN_FUSED picks)."""
    import paper_2507_20173_amd as fsb

    out = {"workload": f"swim rules: N=2^{n.bit_length() - 1} fish, {steps} iterations"}
    for name, rule in (("plain_swim", 0), ("greedy", fsb.FSB_SWIM_GREEDY),
                       ("weighted", fsb.FSB_SWIM_WEIGHTED),
                       ("greedy_weighted", fsb.FSB_SWIM_GREEDY | fsb.FSB_SWIM_WEIGHTED)):
        row = {}
        for form, mode in (("per_iteration", fsb.FSB_RUN_PLAIN), ("persistent", fsb.FSB_RUN_FUSED)):
            wall, _, _ = run_form(n, steps, mode, swim_rule=rule)
            row[form] = {"ms_per_step": wall / steps * 1e3, "value": n * steps / wall}
        out[name] = row
        log(f"rule {name}: " + ", ".join(f"{k} {v['ms_per_step']:.4f} ms" for k, v in row.items()))
    return out


SCHEDULES = (("static", 0, 0), ("static_1", 0, 1), ("static_4", 0, 4), ("static_16", 0, 16),
             ("dynamic_1", 1, 1), ("dynamic_4", 1, 4), ("dynamic_16", 1, 16),
             ("dynamic_64", 1, 64), ("guided_1", 2, 1), ("guided_16", 2, 16))


def schedule_form(b, tune, steps: int):
    """Tile schedules of the batched kernel (Sec. 2.3.2, Experiment 2's
    static / dynamic / guided and chunk sizes) on the same batch and launch
    shape: one persistent launch of `steps` iterations each, after an
    identical untimed launch (table upload, graph capture)."""
    import torch

    import paper_2507_20173_amd as fsb

    out = {}
    for name, sched, chunk in SCHEDULES:
        tu = fsb.tuning(tune.block_size, tune.fish_per_thread, steps, tune.blocks_per_cu,
                        tune.variant, sched, chunk)
        b.run(steps, tu)
        b.sync()
        fsb.fsb_batch_profile_enable(b.h, 1)
        fsb.fsb_batch_kernel_times(b.h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run(steps, tu)
        b.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        _, ms = fsb.fsb_batch_kernel_times(b.h)
        fsb.fsb_batch_profile_enable(b.h, 0)
        out[name] = {"schedule": sched, "chunk_tiles": chunk, "ms_per_step": wall / steps * 1e3,
                     "kernel_ms_per_step": ms / steps}
        log(f"schedule {name}: {ms / steps:.3f} ms per iteration")
    base = out["static"]["kernel_ms_per_step"]
    for v in out.values():
        v["relative_to_static"] = v["kernel_ms_per_step"] / base
    return out


def batched_form(n_schools: int, steps: int, probe_steps: int, baseline_schools: int,
                 schedule_steps: int):
    """4096 independent schools of log-uniform sizes, each its own seed,
    advanced by graph-replayed persistent launches with an autotuned shape;
    against advancing the same schools one by one with per-iteration launches
    (on the first `baseline_schools` schools); then the tile schedules
    compared on the same batch."""
    import numpy as np
    import torch

    import paper_2507_20173_amd as fsb
    from paper_2507_20173_amd.workloads import log_uniform_school_sizes, school_seeds

    sizes = log_uniform_school_sizes(n_schools)
    seeds = school_seeds(n_schools)
    total = int(sizes.sum())
    common = fsb.FsbConfig(n_fish=0)
    probe = fsb.Batch(common, sizes, seeds)
    tune = probe.autotune(probe_steps)
    probe.close()
    del probe
    torch.cuda.empty_cache()

    b = fsb.Batch(common, sizes, seeds)
    b.sync()
    fsb.fsb_batch_profile_enable(b.h, 1)
    fsb.fsb_batch_kernel_times(b.h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(steps, tune)
    b.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, ms = fsb.fsb_batch_kernel_times(b.h)
    xy, sums, mx = b.results()
    fsb.fsb_batch_profile_enable(b.h, 0)
    schedules = schedule_form(b, tune, schedule_steps) if schedule_steps else None
    b.close()
    del b
    torch.cuda.empty_cache()
    K = min(tune.steps_per_launch, steps)
    variant = {fsb.FSB_RUN_FUSED_LEAN: "lean", fsb.FSB_RUN_FUSED_DEEP: "deep"}.get(tune.variant,
                                                                                "prev")
    bytes_total = batch_bytes(variant, total, steps, K, launches)

    # baseline: the first schools one by one, one launch per iteration (FSB_RUN_PLAIN)
    base_fish, base_wall = 0, 0.0
    for i in range(baseline_schools):
        sch = fsb.School(fsb.FsbConfig(n_fish=int(sizes[i]), seed=int(seeds[i])))
        sch.sync()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sch.run(steps)
        sch.sync()
        torch.cuda.synchronize()
        base_wall += time.perf_counter() - t1
        base_fish += int(sizes[i])
        sch.close()
    value = total * steps / wall
    base = base_fish * steps / base_wall
    return {
        "workload": f"batched form: {n_schools} schools, sizes log-uniform in [1e3, 1e6] "
                    f"({total} fish), seed_s = s, {steps} iterations, graph-replayed persistent "
                    f"launches of {K} iterations, autotuned",
        "n_schools": n_schools, "total_fish": total, "iterations": steps,
        "tuning": fsb.tuning_dict(tune), "autotune_probe_steps": probe_steps,
        "value": value, "ms_per_step": wall / steps * 1e3, "launches": int(launches),
        "variant": variant,
        "lane_sums": "binary64 accumulation of pairwise float32 group totals" if variant == "deep"
        else "compensated float32 (TwoSum) lanes",
        "algorithmic_bytes_per_fish_step": {"lean": 24, "prev": 32, "deep": 32 / BATCH_DEEP_DEPTH}[variant],
        "kernel_achieved_GBs": bytes_total / (ms / 1e3) / 1e9,
        "kernel_hbm_frac": bytes_total / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
        "roofline_alu": (valu_roofline("batch_deep_cfg5", total * steps, ms / 1e3)
                         if variant == "deep" and n_schools == 4096 else None),
        "baseline_per_school_plain": {"schools": baseline_schools, "fish": base_fish,
                                      "value": base, "speedup_of_batched": value / base},
        "mean_max_delta_last_iteration": float(np.mean(mx)),
        "schedules": schedules,
    }


def oracle_prefix(n: int, budget_s: float, max_steps: int = 200) -> dict:
    """The oracle on a bounded prefix of one school's run (N = n, seed 0):
    iterations until the budget is spent, the initialisation not timed."""
    from oracle.oracle import Config, default

    O = default()
    cfg = Config(numFish=n, seed=0)
    school = O.init(cfg)
    done, t0 = 0, time.perf_counter()
    while done < max_steps and (done == 0 or time.perf_counter() - t0 < budget_s):
        O.step(cfg, school, done)
        done += 1
    el = time.perf_counter() - t0
    return {"value": n * done / el, "unit": "fish-updates/s", "cores": O.max_threads(),
            "kind": "oracle",
            "sample": f"first {done} iterations of one school of N={n} (seed 0), {el:.1f} s; "
                      "rate per fish-iteration, taken to hold for the whole run"}


def oracle_schools(sizes, seeds, steps: int, budget_s: float) -> dict:
    """The oracle on the first schools of a batch, one after another, each
    for `steps` iterations, until the budget is spent."""
    from oracle.oracle import Config, default

    O = default()
    fish_steps, k, el = 0, 0, 0.0
    start = time.perf_counter()  # the initialisations count against the budget too
    while k < len(sizes) and (k == 0 or time.perf_counter() - start < budget_s):
        cfg = Config(numFish=int(sizes[k]), seed=int(seeds[k]))
        school = O.init(cfg)
        t0 = time.perf_counter()
        O.run(cfg, school, 0, steps)
        el += time.perf_counter() - t0
        fish_steps += int(sizes[k]) * steps
        k += 1
    return {"value": fish_steps / el, "unit": "fish-updates/s", "cores": O.max_threads(),
            "kind": "oracle",
            "sample": f"the first {k} schools ({fish_steps // steps} fish), {steps} iterations "
                      f"each, {el:.1f} s; rate per fish-iteration, taken to hold for the batch"}


def host_cpu() -> dict:
    """The host's CPU model and the processors this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "usable_cpus": len(os.sched_getaffinity(0)),
            "online_cpus": os.cpu_count()}


def cpu_baseline(n: int, budget_s: float = 12.0, max_steps: int = 400):
    """The oracle as it stands, on this host's cores, on a bounded prefix of
    the same workload."""
    from oracle.oracle import Config, default

    O = default()
    cores = O.max_threads()
    cfg = Config(numFish=n, seed=0)
    school = O.init(cfg)
    done, t0 = 0, time.perf_counter()
    while done < max_steps and time.perf_counter() - t0 < budget_s:
        O.step(cfg, school, done)
        done += 1
    el = time.perf_counter() - t0
    # the same oracle on one thread, for the next iterations (a quarter of the budget)
    O.set_threads(1)
    one, t1 = 0, time.perf_counter()
    while one < max_steps and time.perf_counter() - t1 < budget_s / 4:
        O.step(cfg, school, done + one)
        one += 1
    el1 = time.perf_counter() - t1
    O.set_threads(cores)
    return {"value": n * done / el, "unit": "fish-updates/s", "cores": cores,
            "kind": "oracle", "host": host_cpu(),
            "sample": f"first {done} iterations of the same school (N={n}, seed 0), binary32 "
                      f"oracle with binary64 reference sums, {el:.1f} s on {cores} threads",
            "single_thread": {"value": n * one / el1,
                              "sample": f"iterations {done}..{done + one - 1}, {el1:.1f} s"}}


def drift_report(n: int = 10_000, steps: int = 100) -> dict:
    """The binary64 drift report: the oracle's binary32 school and its
    binary64 variant, from the same seed and the same integer draws, side by
    side for `steps` iterations (information only, not a parity gate: the two
    trajectories legitimately part).  Positions can part by at most k (ulp32(H)
    / 2 + ulp32(S) / 2) after k iterations, each binary32 iteration rounding
    the displacement and the addition once; weights part further, since
    feeding divides differences of nearby objectives by M."""
    import numpy as np

    from oracle.oracle import Config, default

    O = default()
    cfg = Config(numFish=n, seed=0)
    s32, s64 = O.init(cfg), O.init_f64(cfg)
    pos, w_drift, m_rel, bary = [], [], [], []
    for t in range(steps):
        m32, sums32, _ = O.step(cfg, s32, t)
        m64, sums64 = O.step_f64(cfg, s64, t)
        pos.append(max(np.abs(s32["x"] - s64["x"]).max(), np.abs(s32["y"] - s64["y"]).max()))
        w_drift.append(np.abs(s32["weight"] - s64["weight"]).max())
        m_rel.append(abs(float(m32) - m64) / m64 if m64 > 0 else 0.0)
        b32 = np.array([sums32[1], sums32[2]]) / sums32[0]
        b64 = np.array([sums64[1], sums64[2]]) / sums64[0]
        bary.append(float(np.abs(b32 - b64).max()))
    per = float(np.spacing(np.float32(cfg.pondHalf))) / 2 + \
        float(np.spacing(np.float32(cfg.swimStep))) / 2
    return {"workload": f"oracle binary32 vs binary64, N={n}, {steps} iterations, seed 0",
            "max_position_drift": float(max(pos)),
            "position_bound_last_iteration": (steps + 1) * per,
            "final_position_drift": float(pos[-1]),
            "max_weight_drift": float(max(w_drift)), "final_weight_drift": float(w_drift[-1]),
            "max_relative_M_drift": float(max(m_rel)),
            "max_barycentre_drift": float(max(bary)), "final_barycentre_drift": bary[-1],
            "note": "information only (O2-b): binary32 and binary64 trajectories part "
                    "legitimately; parity is against the binary32 oracle"}


COPY_FLOATS = 1 << 26  # calibration copy: 256 MiB read + 256 MiB written
COPY_REPS = 4


def calibrate_copy(reps: int = COPY_REPS) -> None:
    """Device-to-device copies of a known size (torch's copy_, a plain copy
    kernel), to scale the HBM counters of the same run."""
    import torch
    a = torch.ones(COPY_FLOATS, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()


def _counter_rows(directory: str, counter: str):
    """(kernel name, value) per dispatch from rocprofv3 counter CSVs."""
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


def plain_kernel_names(n: int) -> dict:
    """The instances a default-configuration run launches for a school of n
    fish (cache policy by footprint, as the library picks it): fsb_step's
    swim and feed passes, and FSB_RUN_PLAIN's pipelined pass."""
    pol = 0 if 16 * n <= INFINITY_CACHE_MIB << 20 else 1 if 12 * n <= INFINITY_CACHE_MIB << 20 else 2
    return {"swim_eval": f"swim_eval_kernel<false, {pol}, false>",
            "feed_bary": f"feed_bary_kernel<0, {pol}, false>",
            "feed_swim": f"feed_swim_kernel<false, {pol}>"}


def ingest_counters(fetch_dir: str, write_dir: str, n_fish: int, out_path: str = TRAFFIC_FILE) -> dict:
    """Per-launch HBM bytes of the plain kernels from a FETCH_SIZE run and a
    WRITE_SIZE run (KiB per dispatch), each scaled by what the same counter
    reads for the calibration copy of known size."""
    import statistics
    out = {"n_fish": n_fish, "source_digest": source_digest(), "kernels": {}}
    scale = {}
    per = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _counter_rows(d, counter)
        # the calibration copies (a copy may be split over several dispatches;
        # the library's own small read-backs are left out by size)
        copy = [v for k, v in rows if "copyBuffer" in k and v > 1024.0]
        if not copy:
            raise SystemExit(f"no calibration copy dispatches with {counter} in {d}")
        known_kib = COPY_REPS * COPY_FLOATS * 4 / 1024
        scale[counter] = known_kib / sum(copy)
        for key, name in plain_kernel_names(n_fish).items():
            vals = [v for k, v in rows if name in k]
            if vals:
                per.setdefault(key, {})[counter] = statistics.mean(vals)
    out["copy_scale"] = scale
    for key in plain_kernel_names(n_fish):
        c = per.get(key, {})
        if "FETCH_SIZE" in c and "WRITE_SIZE" in c:
            rd = c["FETCH_SIZE"] * scale["FETCH_SIZE"] * 1024
            wr = c["WRITE_SIZE"] * scale["WRITE_SIZE"] * 1024
            out["kernels"][key] = {"fetch_bytes_per_launch": rd, "write_bytes_per_launch": wr,
                                   "bytes_per_launch": rd + wr,
                                   "algorithmic_bytes_per_launch": BYTES_PER_FISH[key] * n_fish}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def ingest_valu(fused_dir: str, batch_dir: str, fused_steps: int, batch_steps: int,
                out_path: str = VALU_FILE) -> dict:
    """Vector-ALU lane instructions per fish-iteration of the deep kernels from
    two rocprofv3 --pmc SQ_INSTS_VALU runs: the persistent forms
    (`--forms fused,registers --fused-steps fused_steps`) and the batched form
    (`--forms batched --batch-steps batch_steps`).  Each kernel's timed launch
    is its dispatch with the most instructions."""
    from paper_2507_20173_amd.workloads import log_uniform_school_sizes
    out = {"source_digest": valu_digest(), "fused_steps": fused_steps, "batch_steps": batch_steps,
           "lane_instructions_per_fish_iteration": {}}
    lanes = out["lane_instructions_per_fish_iteration"]
    rows = _counter_rows(fused_dir, "SQ_INSTS_VALU")
    for key, (name, n) in DEEP_COUNTER_KERNELS.items():
        vals = [v for k, v in rows if name in k]
        if vals:
            lanes[key] = max(vals) * 64 / (n * fused_steps)
    total = int(log_uniform_school_sizes(4096).sum())
    vals = [v for k, v in _counter_rows(batch_dir, "SQ_INSTS_VALU") if BATCH_DEEP_COUNTER_KERNEL in k]
    if vals:
        lanes["batch_deep_cfg5"] = max(vals) * 64 / (total * batch_steps)
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n-fish", type=int, default=1 << 24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--hbm-companion-fish", type=int, default=HBM_RESIDENT_FISH,
                    help="school of the HBM-resident companion roofline (0 = skip it, e.g. "
                         "for counter runs that must see the headline's kernels alone)")
    ap.add_argument("--plain-only", action="store_true", help="skip the other forms")
    ap.add_argument("--forms", default="fused,registers,precision,batched,ablation,rules",
                    help="comma list of the forms to measure beside the headline")
    ap.add_argument("--fused-steps", type=int, default=2000)
    ap.add_argument("--precision-steps", type=int, default=200)
    ap.add_argument("--schools", type=int, default=4096)
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--autotune-steps", type=int, default=16)
    ap.add_argument("--baseline-schools", type=int, default=64)
    ap.add_argument("--schedule-steps", type=int, default=100,
                    help="iterations per tile schedule compared in the batched form (0 = skip)")
    ap.add_argument("--ablation-sizes", default="10000,1048576,16777216",
                    help="school sizes of the construct ablation")
    ap.add_argument("--ablation-checked-steps", type=int, default=2)
    ap.add_argument("--rules-steps", type=int, default=300)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run known-size device copies first (for counter scaling)")
    ap.add_argument("--traffic-out", default=TRAFFIC_FILE,
                    help="where --ingest-counters writes the per-launch traffic")
    ap.add_argument("--form-oracle-seconds", type=float, default=4.0,
                    help="CPU seconds of oracle timing beside each large form (0: none)")
    ap.add_argument("--cpu-baseline-seconds", type=float, default=12.0,
                    help="budget of the oracle's timed sample")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the plain kernels' measured HBM traffic from two rocprofv3 "
                         "--pmc runs (FETCH_SIZE, WRITE_SIZE) and exit")
    ap.add_argument("--ingest-valu", nargs=4,
                    metavar=("FUSED_DIR", "BATCH_DIR", "FUSED_STEPS", "BATCH_STEPS"),
                    help="write the deep kernels' VALU instructions per fish-iteration from "
                         "two rocprofv3 --pmc SQ_INSTS_VALU runs and exit")
    ap.add_argument("--valu-out", default=VALU_FILE,
                    help="where --ingest-valu writes the instruction counts")
    args = ap.parse_args()
    if args.ingest_counters:
        print(json.dumps(ingest_counters(*args.ingest_counters, args.n_fish, args.traffic_out),
                         indent=1))
        return 0
    if args.ingest_valu:
        fd, bd, fs, bs = args.ingest_valu
        print(json.dumps(ingest_valu(fd, bd, int(fs), int(bs), args.valu_out), indent=1))
        return 0
    if args.gpus != 1:
        log(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
            "the school would shard across GPUs with one small all-gather per iteration, "
            "which is not built.")
        return 2

    import torch
    if not torch.cuda.is_available():
        log("bench.py needs a GPU")
        return 1
    n = args.n_fish
    if args.calibrate_copy:
        calibrate_copy()
    global MEASURED_VALU
    MEASURED_VALU = valu_ceiling()
    wall, kernels, xy = plain_run(n, args.steps, args.warmup)
    value = n * args.steps / wall
    dom = dominant(kernels)
    dk = kernels[dom]
    traffic = measured_traffic(dom, n)
    pattern = sweep_ceiling(n)
    residency = cache_residency(n)
    line = {
        "metric": "fish-updates/sec (N x steps/s) on 1 MI355X + % of HBM peak; fused vs plain",
        "value": value,
        "unit": "fish-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"plain FSB, one school: N=2^{n.bit_length() - 1} fish, "
                               f"{args.steps} iterations, one kernel launch per iteration "
                               "(FSB_RUN_PLAIN: the feed of iteration t-1 pipelined into the "
                               "swim of t; a swim pass first, a feed pass last)",
                   "n_fish": n, "iterations": args.steps, "seed": 0, "mode": "plain",
                   "infinity_cache": residency},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": dk["achieved_GBs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dk["achieved_GBs"] / HBM_PEAK_GBS, "traffic": traffic,
                     "pattern_ceiling": pattern,
                     "frac_of_pattern_ceiling": dk["achieved_GBs"] / pattern["achieved_GBs"],
                     "cache_assisted": residency["live_columns_fit"],
                     "note": "algorithmic bytes / event-timed duration; the reused columns fit "
                             "the 256 MiB Infinity Cache at this size, so part of the traffic "
                             "(counted by FETCH_SIZE/WRITE_SIZE as L2 egress) is served from "
                             "it: see roofline_hbm_resident for the same kernels from HBM"
                     if residency["live_columns_fit"] else "columns exceed the Infinity Cache"},
        "kernels": kernels,
        "valu_ceiling": MEASURED_VALU,
        "algorithmic_bytes_per_fish_step": plain_bytes(n, args.steps) / (n * args.steps),
        "hbm_frac_whole_step": plain_bytes(n, args.steps) / wall / 1e9 / HBM_PEAK_GBS,
    }
    # the same iterations as fsb_step's two passes (44 B per fish-iteration)
    wall_s, kernels_s, _ = plain_run(n, args.steps, args.warmup, split=True)
    line["plain_split"] = {
        "value": n * args.steps / wall_s, "ms_per_step": wall_s / args.steps * 1e3,
        "algorithmic_bytes_per_fish_step": SPLIT_BYTES_PER_FISH_STEP,
        "hbm_frac_whole_step": plain_bytes(n, args.steps, True) / wall_s / 1e9 / HBM_PEAK_GBS,
        "kernels": kernels_s, "pipelined_speedup": value / (n * args.steps / wall_s)}
    if args.hbm_companion_fish:
        # the same passes on a school whose columns cannot stay in the 256 MiB
        # Infinity Cache: every byte comes from HBM
        n_hbm = args.hbm_companion_fish
        hbm_steps = min(args.steps, 200)
        wall_h, kernels_h, _ = plain_run(n_hbm, hbm_steps, min(args.warmup, 5))
        dom_h = dominant(kernels_h)
        pattern_h = sweep_ceiling(n_hbm)
        wall_hs, kernels_hs, _ = plain_run(n_hbm, hbm_steps, min(args.warmup, 5), split=True)
        line["roofline_hbm_resident"] = {
            "bound": "hbm", "kernel": dom_h, "n_fish": n_hbm, "iterations": hbm_steps,
            "achieved": kernels_h[dom_h]["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": kernels_h[dom_h]["achieved_GBs"] / HBM_PEAK_GBS,
            "pattern_ceiling": pattern_h,
            "frac_of_pattern_ceiling": kernels_h[dom_h]["achieved_GBs"] / pattern_h["achieved_GBs"],
            "whole_step_frac": plain_bytes(n_hbm, hbm_steps) / wall_h / 1e9 / HBM_PEAK_GBS,
            "ms_per_step": wall_h / hbm_steps * 1e3, "kernels": kernels_h,
            "split": {"swim_frac": kernels_hs["swim_eval"]["achieved_GBs"] / HBM_PEAK_GBS,
                      "feed_frac": kernels_hs["feed_bary"]["achieved_GBs"] / HBM_PEAK_GBS,
                      "whole_step_frac": plain_bytes(n_hbm, hbm_steps, True) / wall_hs / 1e9
                      / HBM_PEAK_GBS,
                      "ms_per_step": wall_hs / hbm_steps * 1e3, "kernels": kernels_hs},
            "infinity_cache": cache_residency(n_hbm)}
    forms = set() if args.plain_only else set(args.forms.split(","))
    line["forms"] = {}
    if "fused" in forms:
        line["forms"]["fused_cfg4"] = fused_vs_plain(
            1 << 26, args.fused_steps,
            f"persistent form: N=2^26 fish, {args.fused_steps} iterations in one cooperative "
            "launch vs per-iteration launches")
        line["forms"]["fused_cfg2"] = fused_vs_plain(
            n, args.steps,
            f"persistent form on the headline school (N=2^24, {args.steps} iterations)")
    if "registers" in forms:
        line["forms"]["fused_registers"] = fused_vs_plain(
            1 << 21, args.fused_steps,
            f"persistent forms at N=2^21 fish (the largest school the register-resident kernel "
            f"holds), {args.fused_steps} iterations in one cooperative launch, every variant "
            "against per-iteration launches")
    if "precision" in forms:
        line["forms"]["precision_cfg3"] = precision_form(1 << 27, args.precision_steps)
    if "batched" in forms:
        line["forms"]["batched_cfg5"] = batched_form(args.schools, args.batch_steps,
                                                     args.autotune_steps, args.baseline_schools,
                                                     args.schedule_steps)
    if "rules" in forms:
        line["forms"]["swim_rules"] = rules_form(n, args.rules_steps)
    if "ablation" in forms:
        line["forms"]["construct_ablation"] = ablation_form(
            [int(v) for v in args.ablation_sizes.split(",")], args.ablation_checked_steps)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(n, args.cpu_baseline_seconds)
        line["cpu_baseline"]["drift_f64"] = drift_report()
        if args.form_oracle_seconds > 0:
            # the oracle beside each large form's GPU figure (bounded samples)
            budget = args.form_oracle_seconds
            f = line["forms"]
            if "fused_cfg4" in f:
                f["fused_cfg4"]["oracle"] = oracle_prefix(1 << 26, budget)
            if "precision_cfg3" in f:
                f["precision_cfg3"]["oracle"] = oracle_prefix(1 << 27, budget)
            if "batched_cfg5" in f:
                from paper_2507_20173_amd.workloads import log_uniform_school_sizes, school_seeds
                f["batched_cfg5"]["oracle"] = oracle_schools(
                    log_uniform_school_sizes(args.schools), school_seeds(args.schools), 2, budget)
    # every handle is closed by now; free the tensors and drain the device
    # before the line goes out and the interpreter shuts down
    import gc
    gc.collect()
    torch.cuda.synchronize()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
