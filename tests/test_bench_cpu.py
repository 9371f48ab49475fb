"""Host-side checks of bench.py: the one-GPU guard and the algorithmic byte counts that
the roofline uses (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_per_stage():
    n = 1024 * 1024
    # stage 1: U^n (9) + bed vertex (1) read, U^int (9) written
    assert bench.stage_bytes("stage1", n, 8) == 19 * 8 * n
    # stage 2: U^n (9), U^int (9), bed (1) read, U^{n+1} (9) written
    assert bench.stage_bytes("stage2", n, 8) == 28 * 8 * n
    # 376 B per cell-step in FP64, 188 B in FP32
    assert (bench.stage_bytes("stage1", 1, 8) + bench.stage_bytes("stage2", 1, 8)) == 376
    assert (bench.stage_bytes("stage1", 1, 4) + bench.stage_bytes("stage2", 1, 4)) == 188
    # what the kernels move by design: V^n written by stage 1 and read by stage 2
    assert bench.stage_bytes("stage1", 1, 8, bench.IMPL_VALUES) == 224


def test_cpu_baseline_reports_all_threads_and_one():
    from paper_2107_02750_amd import scenarios as S
    r = bench.cpu_baseline(S.fbm_channel_wet(n=48), 0.2)
    assert r["kind"] == "oracle" and r["unit"] == "cell-updates/s"
    assert r["value"] > 0 and r["cores"] >= 1
    assert r["one_core"]["cores"] == 1 and r["one_core"]["value"] > 0
    assert "as_configured" not in r  # no stored state for this grid size


def test_counter_record_is_used_only_for_the_sources_it_was_taken_from(tmp_path, monkeypatch):
    import json
    (tmp_path / "profiles").mkdir()
    rec = {"kernel_source_sha256": "abc", "copy_scale": {"fetch": 2.0, "write": 1.0},
           "kib_per_dispatch": {"stage1": {"fetch": 10.0, "write": 4.0}}}
    (tmp_path / "profiles" / "traffic_x.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    assert bench.measured_traffic("traffic_x", "stage1") == 1024.0 * (10.0 * 2.0 + 4.0 * 1.0)
    assert bench.measured_traffic("traffic_x", "stage2") is None
    assert bench.measured_traffic("traffic_missing", "stage1") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "changed")
    assert bench.measured_traffic("traffic_x", "stage1") is None


def test_committed_counter_records_name_their_hashed_sources():
    import json
    names = sorted(f[:-5] for f in os.listdir(os.path.join(ROOT, "profiles"))
                   if f.startswith("traffic_") and f.endswith(".json"))
    assert "traffic_stage_kernels_fbm_channel_wet_1024_fp64" in names
    assert "traffic_fv1_kernel_fbm_channel_wet_1024" in names
    for name in names:
        with open(os.path.join(ROOT, "profiles", name + ".json")) as fh:
            rec = json.load(fh)
        assert rec["hashed"] == ["paper_2107_02750_amd/csrc/dg2_kernels.hpp",
                                 "paper_2107_02750_amd/csrc/dg2.hip",
                                 "paper_2107_02750_amd/build.py"]
        assert len(rec["kernel_source_sha256"]) == 64
        assert os.path.exists(os.path.join(ROOT, "profiles", rec["summary"]))


def test_profile_commands_use_existing_bench_flags():
    """Every bench.py command quoted in the committed rocprofv3 summaries uses only
    options the bench accepts, so each summary can be made again as written."""
    import re
    import subprocess
    import sys
    helptext = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                              capture_output=True, text=True, check=True).stdout
    known = set(re.findall(r"(--[a-z0-9-]+)", helptext))
    seen = 0
    for name in sorted(os.listdir(os.path.join(ROOT, "profiles"))):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            text = fh.read()
        for cmd in re.findall(r"bench\.py([^`\n]*)", text):
            for flag in re.findall(r"(--[a-z0-9-]+)", cmd):
                assert flag in known, (name, flag)
                seen += 1
    assert seen > 10
