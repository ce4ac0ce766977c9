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
    # the committed summary matches the committed sources
    tri = bench.profiled_traffic(["triangles"])
    wpc = bench.profiled_traffic(["prune_components"])
    assert tri is not None and tri > 0 and wpc is not None and wpc > 0
    assert bench.profiled_traffic(["no_such_stage"]) is None
    # a copy of the tree whose triangle kernel differs by one byte: that
    # stage's traffic is withdrawn, the other stage's stays
    root = tmp_path / "tree"
    shutil.copytree(os.path.join(ROOT, "profiles"), root / "profiles")
    shutil.copytree(os.path.join(ROOT, "paper_2412_12382_amd", "csrc"), root / "paper_2412_12382_amd" / "csrc")
    with open(root / "paper_2412_12382_amd" / "csrc" / "tc.hip", "a") as f:
        f.write("\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.profiled_traffic(["triangles"]) is None
    assert bench.profiled_traffic(["prune_components"]) == wpc
