"""Our own gfx950 assembly keeps the binary32 contract: the only fused
multiply-adds in any kernel are those inside the correctly rounded sqrtf
(two residual checks per v_sqrt_f32) and division (five per
v_div_fixup_f32) expansions, plus the swim displacements' explicit
fma(S * 2^-23, r >> 8, -S), which rounds once exactly as S * v(r) does (its
addend is the uniform -S, read from a scalar register, negated there or by the
operand modifier), and the deep kernels' look-ahead skip test fma(dx, dx,
RN(dy * dy)), a bound on a move's length that feeds no fish's state (both
multiplicands the same register, only in the deep kernels' plain-swim
instances); and no packed-FP32 instruction is emitted, in the single-school and
the batch kernels alike.  The VALU ceiling probes issue exactly the
instructions per round that the library's rate assumes."""
import re

import pytest

from paper_2507_20173_amd import build as fsb_build


@pytest.fixture(scope="module")
def kernels():
    bodies, name = {}, None
    for source in ("fsb_kernels.hip", "fsb_batch.hip", "fsb_probe.hip"):
        text = open(fsb_build.assembly(source)).read()
        for line in text.splitlines():
            m = re.match(r"^(_Z\w+):", line)
            if m:
                name = m.group(1)
                bodies[name] = []
            elif name:
                bodies[name].append(line)
                if line.strip().startswith(".Lfunc_end"):
                    name = None
    return {k: "\n".join(v) for k, v in bodies.items()}


def count(body, pattern):
    return len(re.findall(pattern, body))


def test_kernels_found(kernels):
    names = " ".join(kernels)
    for k in ("init_kernel", "swim_eval_kernel", "feed_bary_kernel", "combine_kernel",
              "fused_kernel", "fused_lean_kernel", "batch_kernel", "batch_init_kernel"):
        assert k in names, k


DRAW_FMA = r"\bv_fma_f32\s+v\d+,\s*v\d+,\s*v\d+,\s*-?s\d+"
# the skip test's fma(dx, dx, q): the same register as both multiplicands
SQUARE_FMA = r"\bv_fma_f32\s+v\d+,\s*(v\d+),\s*\1,\s*v\d+|\bv_fmac_f32_e32\s+v\d+,\s*(v\d+),\s*\2\b"


def is_deep_plain_swim(name):
    # fused_deep_kernel<KD, NT, 0u> and batch_deep_kernel<B, GPL, NT, KD, 0u>
    return ("fused_deep_kernel" in name or "batch_deep_kernel" in name) and name.endswith(
        "Lj0EEEvNS_10SchoolArgsENS_9FusedArgsE") or (
        "batch_deep_kernel" in name and name.endswith("Lj0EEEvNS_9BatchArgsE"))


def test_no_contraction_outside_sqrt_and_div(kernels):
    draws_seen = squares_seen = 0
    for name, body in kernels.items():
        if "valu_probe_fma_kernel" in name or "valu_probe_mixed_kernel" in name:
            continue  # instrumentation: explicit fma chains, no fish state
        fma = count(body, r"\bv_(fma|fmac|mac|mad)_f32|\bv_fma_mix")
        draws = count(body, DRAW_FMA)
        squares = count(body, SQUARE_FMA)
        sqrt = count(body, r"\bv_sqrt_f32")
        div = count(body, r"\bv_div_fixup_f32")
        assert squares == 0 or is_deep_plain_swim(name), f"{name}: {squares} square fmas"
        assert fma - draws - squares == 2 * sqrt + 5 * div, (
            f"{name}: {fma} fused ops ({draws} draws, {squares} skip tests) vs {sqrt} sqrt "
            f"and {div} div expansions")
        assert draws % 2 == 0, f"{name}: draws come in (dx, dy) pairs"
        draws_seen += draws
        squares_seen += squares
    assert draws_seen > 0 and squares_seen > 0


def test_no_packed_fp32(kernels):
    for name, body in kernels.items():
        assert count(body, r"\bv_pk_(add|mul|fma)_f32") == 0, name


def test_critical_mode_issues_one_atomic_per_fish(kernels):
    """The critical-mode passes update the shared words from every lane: the
    swim pass one global atomic max per fish (4 per float4 group, 1 group in
    flight, plus the tail fish: 5), the feed pass three float32 atomic adds
    per fish (1 group in flight plus the tail fish: 15), and neither folds
    lanes first (no DPP or lane-read reduction, which the compiler's atomic
    optimiser would otherwise insert)."""
    swim = {k: v for k, v in kernels.items()
            if "swim_eval_kernel" in k and k.endswith("Lb1EEEvNS_10SchoolArgsENS_8StepArgsE")}
    feed = {k: v for k, v in kernels.items() if "feed_bary_kernelILi2E" in k}
    assert len(swim) == 6 and len(feed) == 3
    for name, body in swim.items():
        assert count(body, r"\bglobal_atomic_umax\b") == 5, name
        assert count(body, r"\bdpp|\bv_readlane") == 0, name
    for name, body in feed.items():
        assert count(body, r"\bglobal_atomic_add_f32\b") == 15, name
        assert count(body, r"\bdpp|\bv_readlane") == 0, name


def test_grid_barrier_waits_for_every_waves_stores(kernels):
    """Each persistent kernel passes its grid barrier after the prologue and
    in the iteration loop; where memory operations may be outstanding, every
    wave waits for its own (vmcnt 0) right before the workgroup barrier that
    precedes thread 0's release, so tile partials, max atomics and columns
    written by any wave are covered by that release.  (The compiler drops the
    wait where it can prove nothing is outstanding, as after the register-
    resident kernel's prologue, whose loads have all been consumed.)"""
    persistent = {k: v for k, v in kernels.items()
                  if re.search(r"fused_kernel|fused_lean_kernel|fused_regs_kernel|"
                               r"fused_deep_kernel|batch_kernel", k)}
    assert len(persistent) >= 20
    for name, body in persistent.items():
        waits = len(re.findall(r"s_waitcnt vmcnt\(0\)[^\n]*\n(?:[^\n]*\n){0,2}?\s*s_barrier\b",
                               body))
        assert waits >= (1 if "regs" in name else 2), f"{name}: {waits} barriers after a wait"


def loop_blocks(body):
    """Instruction mnemonics of each basic block that branches back to itself."""
    blocks, cur = {}, None
    for line in body.splitlines():
        m = re.match(r"^(\.LBB\w+):", line)
        if m:
            cur = m.group(1)
            blocks[cur] = []
            continue
        t = line.strip()
        if cur and t and not t.startswith((";", ".")):
            blocks[cur].append(t)
    return {b: [t.split()[0] for t in ins] for b, ins in blocks.items()
            if any(t.split()[0].startswith(("s_cbranch", "s_branch")) and t.split()[-1] == b
                   for t in ins)}


@pytest.mark.parametrize("kernel,per_round", [
    ("valu_probe_fma_kernel", {"v_fma_f32": 8}),
    ("valu_probe_philox_kernel", {"v_mad_u64_u32": 40, "v_bitop3_b32": 40}),
    ("valu_probe_mixed_kernel", {"v_mad_u64_u32": 20, "v_bitop3_b32": 20, "v_fma_f32": 40}),
])
def test_valu_probe_loops(kernels, kernel, per_round):
    """The probe's loop holds the vector instructions fsb_valu_probe counts
    (FSB_PROBE_FMA 8, FSB_PROBE_PHILOX and FSB_PROBE_MIXED 80 per round) and no
    others."""
    (body,) = [b for n, b in kernels.items() if kernel in n]
    loops = loop_blocks(body)
    assert len(loops) == 1, loops
    (ins,) = loops.values()
    vector = [i for i in ins if i.startswith("v_")]
    assert {k: vector.count(k) for k in set(vector)} == per_round
