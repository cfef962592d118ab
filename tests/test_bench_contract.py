"""bench.py's host logic: the one-GPU refusal, the counter ingestion that
scales rocprofv3 FETCH_SIZE / WRITE_SIZE by a known-size copy, the deep
kernels' VALU instruction counts and their "alu" roofline, the digests that
void stale figures, and (on a GPU) the shape of the JSON line."""
import csv
import json
import re
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def _counter_csv(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "x_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": counter, "Counter_Value": v})


def test_counter_ingestion_scales_by_the_copy(tmp_path):
    n = 1 << 20
    copy_kib = bench.COPY_REPS * bench.COPY_FLOATS * 4 / 1024
    # FETCH_SIZE reads half of the copy's bytes, WRITE_SIZE all of them (as
    # measured on MI355X); the library's own small read-back is ignored
    fetch = [("__amd_rocclr_copyBuffer", copy_kib / 2 / bench.COPY_REPS)] * bench.COPY_REPS
    fetch += [("__amd_rocclr_copyBuffer", 0.5)]
    fetch += [("void fsb::swim_eval_kernel<false, 0, false>(...)", 8 * n / 1024 / 2)] * 3
    fetch += [("void fsb::feed_bary_kernel<0, 0, false>(...)", 16 * n / 1024 / 2)] * 3
    fetch += [("void fsb::feed_swim_kernel<false, 0>(...)", 16 * n / 1024 / 2)] * 5
    # a pipelined run's closing feed pass (it also writes cur) is not the split pass
    fetch += [("void fsb::feed_bary_kernel<0, 0, true>(...)", 99 * n / 1024)]
    write = [("__amd_rocclr_copyBuffer", copy_kib / bench.COPY_REPS)] * bench.COPY_REPS
    write += [("void fsb::swim_eval_kernel<false, 0, false>(...)", 16 * n / 1024)] * 3
    write += [("void fsb::feed_bary_kernel<0, 0, false>(...)", 4 * n / 1024)] * 3
    write += [("void fsb::feed_swim_kernel<false, 0>(...)", 16 * n / 1024)] * 5
    write += [("void fsb::feed_bary_kernel<0, 0, true>(...)", 99 * n / 1024)]
    _counter_csv(tmp_path / "f", "FETCH_SIZE", fetch)
    _counter_csv(tmp_path / "w", "WRITE_SIZE", write)
    out = tmp_path / "traffic.json"
    t = bench.ingest_counters(str(tmp_path / "f"), str(tmp_path / "w"), n, str(out))
    assert t["copy_scale"]["FETCH_SIZE"] == pytest.approx(2.0)
    assert t["copy_scale"]["WRITE_SIZE"] == pytest.approx(1.0)
    for k, per_fish in (("swim_eval", 24), ("feed_bary", 20), ("feed_swim", 32)):
        assert t["kernels"][k]["bytes_per_launch"] == pytest.approx(per_fish * n)
        assert t["kernels"][k]["algorithmic_bytes_per_launch"] == per_fish * n
    assert json.loads(out.read_text())["source_digest"] == bench.source_digest()
    assert bench.measured_traffic("swim_eval", n, str(out)) == pytest.approx(24 * n)
    assert bench.measured_traffic("swim_eval", 2 * n, str(out)) is None
    stale = json.loads(out.read_text())
    stale["source_digest"] = "0" * 16
    out.write_text(json.dumps(stale))
    assert bench.measured_traffic("swim_eval", n, str(out)) is None


def test_code_digest_ignores_comments(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text("int f(int a) {\n  return a + 1;  // one more\n}\n")
    d0 = bench.code_digest([str(src)])
    src.write_text("/* a kernel */\nint f(int a) {\n\n  return a + 1;   // plus one\n}\n")
    assert bench.code_digest([str(src)]) == d0
    src.write_text("int f(int a) {\n  return a + 2;  // one more\n}\n")
    assert bench.code_digest([str(src)]) != d0


def test_valu_ingestion_and_roofline(tmp_path):
    from paper_2507_20173_amd.workloads import log_uniform_school_sizes
    n = 1 << 26
    # the timed launch is each kernel's dispatch with the most instructions
    fused = [("void fsb::fused_deep_kernel<4, true, 0u>(fsb::SchoolArgs, fsb::FusedArgs)", 100 * n * 20 / 64),
             ("void fsb::fused_deep_kernel<4, true, 0u>(fsb::SchoolArgs, fsb::FusedArgs)", 1000.0),
             ("void fsb::fused_deep_kernel<8, false, 0u>(fsb::SchoolArgs, fsb::FusedArgs)",
              120 * (1 << 21) * 20 / 64)]
    total = int(log_uniform_school_sizes(4096).sum())
    batch = [("void fsb::batch_deep_kernel<256, 4, true, 8, 0u>(fsb::BatchArgs)", 110 * total * 16 / 64)]
    _counter_csv(tmp_path / "f", "SQ_INSTS_VALU", fused)
    _counter_csv(tmp_path / "b", "SQ_INSTS_VALU", batch)
    out = tmp_path / "valu.json"
    v = bench.ingest_valu(str(tmp_path / "f"), str(tmp_path / "b"), 20, 16, str(out))
    lanes = v["lane_instructions_per_fish_iteration"]
    assert lanes["fused_deep_n67108864"] == pytest.approx(100)
    assert lanes["fused_deep_n2097152"] == pytest.approx(120)
    assert lanes["batch_deep_cfg5"] == pytest.approx(110)
    assert "fused_deep_n16777216" not in lanes
    # 100 lane instructions per fish-iteration at the nominal rate
    kernel_s = 100 * n * 10 / bench.VALU_LANE_PEAK
    r = bench.valu_roofline("fused_deep_n67108864", n * 10, kernel_s, str(out))
    assert r["bound"] == "alu" and r["frac"] == pytest.approx(1.0)
    assert r["peak"] == pytest.approx(39.3216)
    assert r["measured_ceiling"] is None and r["frac_of_measured_ceiling"] is None
    bench.MEASURED_VALU = {"ceiling": 39.3216 / 1.25}
    try:
        r = bench.valu_roofline("fused_deep_n67108864", n * 10, kernel_s, str(out))
        assert r["frac_of_measured_ceiling"] == pytest.approx(1.25)
    finally:
        bench.MEASURED_VALU = None
    assert bench.valu_roofline("fused_deep_n16777216", n, 1.0, str(out)) is None
    stale = json.loads(out.read_text())
    stale["source_digest"] = "0" * 16
    out.write_text(json.dumps(stale))
    assert bench.valu_roofline("fused_deep_n67108864", n * 10, kernel_s, str(out)) is None


def test_persistent_bytes_accounting():
    n = 1000
    assert bench.persistent_bytes("lean", n, 10) == n * (8 + 24 * 10 + 8)
    assert bench.persistent_bytes("prev", n, 10) == n * (20 + 32 * 9 + 24)
    assert bench.persistent_bytes("regs", n, 10) == n * 32
    assert bench.persistent_bytes("deep", n, 16) == n * (8 + 32 * 2)
    assert bench.persistent_bytes("deep", n, 17) == n * (8 + 32 * 3)
    big = (1 << 23) + 4  # above 5 x 2^20 fish the single-school deep kernel runs four per barrier
    assert bench.persistent_bytes("deep", 5 << 20, 16) == (5 << 20) * (8 + 32 * 2)
    assert bench.persistent_bytes("deep", big, 16) == big * (8 + 32 * 4)
    assert bench.fused_variant(1 << 26) == "deep"
    assert bench.batch_bytes("deep", n, 500, 1000, 1) == n * (8 + 32 * 63)
    assert bench.batch_bytes("deep", n, 20, 8, 3) == n * (8 * 3 + 32 * 3)
    assert bench.batch_bytes("lean", n, 500, 500, 1) == n * (16 + 24 * 500)
    assert bench.batch_bytes("prev", n, 10, 10, 1) == n * (20 + 32 * 9 + 24)
    f = bench.fused_variant
    assert f(1 << 21, False) == "regs" and f((1 << 21) + 4, False) == "prev"
    assert f(1 << 24, False) == "lean" and f(1 << 26, False) == "lean"
    assert bench.SPLIT_BYTES_PER_FISH_STEP == 44
    # pipelined: swim pass 24 B, 32 B per further iteration, closing feed pass 24 B (cur too)
    assert bench.plain_bytes(n, 1000) == n * (24 + 32 * 999 + 24)
    assert bench.plain_bytes(n, 1000, split=True) == n * 44 * 1000
    assert bench.plain_bytes(n, 1) == n * 44  # one iteration is fsb_step's two passes
    assert bench.plain_launches(10, False) == {"swim_eval": 1, "feed_swim": 9, "feed_bary": 1}
    assert bench.plain_kernel_names(1 << 24)["feed_swim"] == "feed_swim_kernel<false, 0>"
    assert bench.plain_kernel_names(1 << 26)["swim_eval"] == "swim_eval_kernel<false, 2, false>"


def test_cache_residency_flags():
    # CFG2's five columns (320 MiB) exceed the 256 MiB cache, its three live
    # columns (192 MiB) fit; CFG4's do not
    r = bench.cache_residency(1 << 24)
    assert r["columns_MiB"] == 320 and r["live_columns_MiB"] == 192
    assert not r["columns_fit"] and r["live_columns_fit"]
    r = bench.cache_residency(1 << 26)
    assert not r["columns_fit"] and not r["live_columns_fit"]
    assert bench.cache_residency(10_000)["columns_fit"]


def test_host_cpu_description():
    h = bench.host_cpu()
    assert h["model"] and 1 <= h["usable_cpus"] <= h["online_cpus"]


def test_oracle_samples_beside_the_forms():
    r = bench.oracle_prefix(4099, 0.05, max_steps=3)
    assert r["kind"] == "oracle" and r["value"] > 0 and r["cores"] >= 1
    assert "iterations of one school of N=4099" in r["sample"]
    r = bench.oracle_schools([10, 20, 30], [0, 1, 2], 2, 1e9)
    assert r["value"] > 0 and "first 3 schools (60 fish), 2 iterations" in r["sample"]


@pytest.mark.gpu
def test_json_line_contract():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--forms", "",
                        "--steps", "20", "--warmup", "2", "--cpu-baseline-seconds", "1"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 20 and d["warmup"] == 2
    assert d["value"] > 0 and d["higher_is_better"] is True and d["vs_baseline"] is None
    assert d["dtype"] == "f32" and d["data"] == "synthetic"
    assert "workload" in d["config"]
    rl = d["roofline"]
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s" and rl["peak"] == 8000.0
    assert rl["frac"] == pytest.approx(rl["achieved"] / rl["peak"])
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0 and cb["sample"]
    assert cb["single_thread"]["value"] > 0 and cb["host"]["usable_cpus"] >= 1
    assert d["config"]["infinity_cache"]["columns_MiB"] == 320
    assert "20 iterations" in d["config"]["workload"]
    assert rl["kernel"] == "feed_swim"
    assert d["kernels"]["feed_swim"]["launches"] == 19
    assert d["plain_split"]["value"] > 0 and d["algorithmic_bytes_per_fish_step"] < 44
    pc = rl["pattern_ceiling"]
    assert 0 < pc["achieved_GBs"] < 2 * 8000 and 0 < rl["frac_of_pattern_ceiling"] < 1.5
    assert not pc["streamed"]
    vc = d["valu_ceiling"]
    assert 0 < vc["fma"] < 2 * vc["nominal"] and 0 < vc["philox"] < 2 * vc["nominal"]
    assert 0 < vc["mixed"] < 2 * vc["nominal"]
    assert vc["ceiling"] == max(vc["fma"], vc["philox"], vc["mixed"])
    assert rl["cache_assisted"] is True
    hr = d["roofline_hbm_resident"]
    assert hr["pattern_ceiling"]["streamed"] and 0 < hr["frac_of_pattern_ceiling"] < 1.5
    assert hr["n_fish"] == 1 << 26 and not hr["infinity_cache"]["live_columns_fit"]
    assert hr["kernel"] == "feed_swim" and 0 < hr["frac"] < 1
    assert 0 < hr["split"]["swim_frac"] < 1 and 0 < hr["split"]["feed_frac"] < 1
    dr = cb["drift_f64"]
    assert dr["max_position_drift"] <= dr["position_bound_last_iteration"]


def test_drift_report_stays_within_the_rounding_bound():
    d = bench.drift_report(n=257, steps=6)
    assert 0 < d["max_position_drift"] <= d["position_bound_last_iteration"]
    assert d["max_weight_drift"] >= 0 and d["max_relative_M_drift"] < 1e-3
    assert "information only" in d["note"]


def test_deep_depth_follows_the_library_rule(monkeypatch):
    """Eight iterations per barrier up to 5 x 2^20 fish, four above, unless
    FSB_DEEP_DEPTH says 2, 4 or 8 (anything else is ignored), as
    include/fsb.h documents for FSB_RUN_FUSED_DEEP."""
    monkeypatch.delenv("FSB_DEEP_DEPTH", raising=False)
    assert bench.deep_depth(1000) == 8 and bench.deep_depth(5 << 20) == 8
    assert bench.deep_depth((5 << 20) + 1) == 4 and bench.deep_depth(1 << 23) == 4
    assert bench.deep_depth(1 << 26) == 4
    monkeypatch.setenv("FSB_DEEP_DEPTH", "2")
    assert bench.deep_depth(1 << 26) == 2 and bench.deep_depth(1000) == 2
    monkeypatch.setenv("FSB_DEEP_DEPTH", "3")
    assert bench.deep_depth(1 << 26) == 4
    header = open(os.path.join(os.path.dirname(__file__), "..", "include", "fsb.h")).read()
    assert "5 x 2^20" in header


def test_counter_names_match_the_built_kernels():
    """The instance names the counter ingestion looks for (plain kernels at
    2^24 and 2^26, the deep kernels' counter keys) are kernels the library
    really builds, as the profiler prints them (demangled)."""
    import shutil

    from paper_2507_20173_amd import build as fsb_build
    filt = shutil.which("c++filt")
    if filt is None:
        pytest.skip("no c++filt")
    symbols = []
    for source in ("fsb_kernels.hip", "fsb_batch.hip"):
        text = open(fsb_build.assembly(source)).read()
        symbols += re.findall(r"^(_Z\w+):", text, re.M)
    out = subprocess.run([filt], input="\n".join(symbols), capture_output=True, text=True,
                         check=True).stdout
    names = [ln.split("(")[0].replace("void fsb::", "") for ln in out.splitlines()]
    wanted = list(bench.plain_kernel_names(1 << 24).values())
    wanted += list(bench.plain_kernel_names(1 << 26).values())
    wanted += [k for k, _ in bench.DEEP_COUNTER_KERNELS.values()]
    wanted.append(bench.BATCH_DEEP_COUNTER_KERNEL)
    for w in wanted:
        assert w in names, w
