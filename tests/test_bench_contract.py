"""Host-side parts of the benchmark: the one-GPU refusal and the rule that
counter-based traffic is reported only for the kernel sources it was taken
with.  No GPU needed."""
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    # a counter record taken with the current sources is reported; once a
    # kernel source differs by one byte, that stage's traffic is withdrawn
    # and the other stage's stays
    import hashlib
    import json
    root = tmp_path / "tree"
    csrc = root / "paper_2412_12382_amd" / "csrc"
    shutil.copytree(os.path.join(ROOT, "paper_2412_12382_amd", "csrc"), csrc)
    h = lambda f: hashlib.sha256(open(csrc / f, "rb").read()).hexdigest()[:16]
    rec = {"triangles": {"sources": {"tc.hip": h("tc.hip")}, "read_bytes": 3.0e12, "write_bytes": 1.0e12},
           "prune_components": {"sources": {"weight.hip": h("weight.hip"), "cc.hip": h("cc.hip")},
                                "read_bytes": 1.0e10, "write_bytes": 5.0e9}}
    (root / "profiles").mkdir()
    (root / "profiles" / "pipeline_rmat_s26_hbm_traffic.md").write_text(
        "# record\n\n```json\n" + json.dumps(rec, indent=1) + "\n```\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.profiled_traffic(["triangles"]) == 4.0e12
    assert bench.profiled_traffic(["prune_components"]) == 1.5e10
    assert bench.profiled_traffic(["no_such_stage"]) is None
    with open(csrc / "tc.hip", "a") as f:
        f.write("\n")
    assert bench.profiled_traffic(["triangles"]) is None
    assert bench.profiled_traffic(["prune_components"]) == 1.5e10


def test_roofline_objects():
    # the triangle roofline names its algorithmic unit; counted bytes give a
    # second fraction when present, and none when the counters are stale
    r = bench.tc_roofline(3200.0, 9.65e11, 300.0, 1.2e12)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == bench.HBM_PEAK_GBS
    assert abs(r["frac"] - 3200.0 / bench.HBM_PEAK_GBS) < 1e-12
    assert abs(r["traffic_frac"] - 1.2e12 / 0.3 / 1e9 / bench.HBM_PEAK_GBS) < 1e-12
    assert "4S" in r["unit_basis"]
    r = bench.tc_roofline(3200.0, 9.65e11, 300.0, None)
    assert r["traffic"] is None and "traffic_frac" not in r
    # the weight+prune+CC pass: moved bytes (16 per edge + 1/8 + 8 per kept
    # edge + 20 per vertex + 8) over the time
    m, n, kept, ms = 1000, 100, 10, 1e-3
    w = bench.wpc_roofline(m, n, kept, ms, None)
    assert w["bound"] == "hbm" and w["traffic"] is None
    assert abs(w["achieved"] - w["algorithmic_bytes"] / (ms * 1e-3) / 1e9) < 1e-9
    assert w["survey_formula_bytes"] > w["algorithmic_bytes"]
