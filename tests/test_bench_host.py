"""Host-side checks of bench.py (no GPU): the one-GPU refusal and the rule that counter
traffic is reported only for the kernels and workload it was measured on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr


def test_kernel_hash_ignores_comments(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_1901_02211_amd", "csrc")
    fake = tmp_path / "paper_1901_02211_amd" / "csrc"
    fake.mkdir(parents=True)
    for f in ("kernels.hip", "wilson_site.h"):
        with open(os.path.join(src, f)) as fh:
            (fake / f).write_text(fh.read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    with open(fake / "kernels.hip", "a") as fh:
        fh.write("\n// a comment only\n\n")
    assert bench.kernel_source_hash() == h0
    with open(fake / "kernels.hip", "a") as fh:
        fh.write("static int changed_code = 1;\n")
    assert bench.kernel_source_hash() != h0


def test_traffic_only_for_its_workload_and_kernels(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    entry = {"kernel_hash": bench.kernel_source_hash(), "traffic_over_algorithmic": 1.25}
    (prof / "traffic.json").write_text(json.dumps({"workload": "noise16x32", "shift_update": entry}))
    csrc = tmp_path / "paper_1901_02211_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("kernels.hip", "wilson_site.h"):
        with open(os.path.join(ROOT, "paper_1901_02211_amd", "csrc", f)) as fh:
            (csrc / f).write_text(fh.read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("shift_update", "noise16x32")["traffic_over_algorithmic"] == 1.25
    assert bench.measured_traffic("shift_update", "noise24") is None      # another workload
    assert bench.measured_traffic("dslash", "noise16x32") is None         # not measured
    with open(csrc / "kernels.hip", "a") as fh:
        fh.write("static int changed_code = 1;\n")
    assert bench.measured_traffic("shift_update", "noise16x32") is None   # other kernels
