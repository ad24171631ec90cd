"""Host-side checks of bench.py (no GPU): the one-GPU refusal and the rule that counter
traffic is reported only for the kernels and workload it was measured on."""
import json
import os
import subprocess
import sys

import numpy as np

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


class FakeTime:
    """Stands in for the time module inside bench: a clock that only the stub advances."""

    def __init__(self):
        self.t = 0.0

    def perf_counter(self):
        return self.t


def test_timed_maps_keep_the_budget():
    ft = FakeTime()
    clock = bench.Clock(470.0, now=ft.perf_counter, t0=0.0)
    reserve = lambda m: 2.4 * m + 75.0 + 25.0   # noqa: E731
    ft.t = 75.0

    def one_map():
        ft.t += 37.0
        return (37.0,)

    runs = bench.timed_maps(one_map, 20, clock, reserve, 37.0)
    assert 1 <= len(runs) < 20
    assert clock.left() >= reserve(37.0)          # the legs after the maps still fit
    # a generous budget: exactly the requested maps
    ft.t = 0.0
    assert len(bench.timed_maps(one_map, 3, bench.Clock(1e6, now=ft.perf_counter, t0=0.0), reserve, 37.0)) == 3
    # an exhausted budget still times one map
    ft.t = 1000.0
    assert len(bench.timed_maps(one_map, 20, clock, reserve, 37.0)) == 1


class StubBinding:
    """The binding's calls that bench.py makes, with a fake clock: a whole mixed map of the
    default workload takes 37 s, an FP64 map 83 s, set-up calls a few seconds."""

    SMPQ_FP64, SMPQ_MIXED_FP32, SMPQ_MIXED_FP16DIR, SMPQ_MIXED_BF16DIR = 0, 1, 2, 3

    def __init__(self, ft, ncls=256, V=131072):
        self.ft, self.ncls, self.V = ft, ncls, V
        self.prec = 1
        self.calls = []

    def _tick(self, s):
        self.ft.t += s

    def smpq_create(self, dims, device=0):
        return object()

    def smpq_load_gauge(self, c, U):
        self._tick(1.0)

    def smpq_set_scheme(self, c, r, mode=0):
        return self.ncls, 12 * self.ncls

    def smpq_set_solver(self, c, prec, tol, max_iter, rel):
        self.prec = prec

    def smpq_estimate_bounds(self, c, steps):
        self._tick(0.5)
        return 0.14, 2.73

    def smpq_set_zolotarev(self, c, n, lo, hi):
        pass

    def smpq_autotune(self, c, n):
        self._tick(20.0)
        return {"f32_kind": 1, "f32_nr": 8, "f64_lgr": 0, "plane_band": 1, "f64_kind": 1, "f64_nr": 2,
                "f32_interleave": 1, "f64_interleave": 2, "f32_dag_kind": 4, "f32_dag_nr": 1, "f32_dag_interleave": 2}

    def smpq_prepare(self, c):
        self._tick(2.0)

    def smpq_set_timing(self, c, on):
        pass

    def _stats(self, n):
        return {"t_solve_s": 36.0 * n / self.ncls, "t_contract_s": 0.01, "n_sources": 12 * n, "n_batches": 5,
                "total_iters": 197 * 12 * n, "max_iters": 198, "n_reliable_updates": 20, "shift_updates": 10 ** 7,
                "dslash_ms": 8000.0, "dslash_bytes": 3.2e13, "dslash_launches": 2000, "update_ms": 25000.0,
                "update_bytes": 1.5e14, "update_launches": 1000, "max_true_resid": 1e-12, "max_abs_imag_q": 1e-3,
                "sum_imag_q": 1e-9, "lam_min": 0.14, "lam_max": 2.73, "zolo_delta": 1e-13}

    def smpq_compute_qx_classes(self, c, classes):
        n = len(classes)
        self._tick((83.0 if self.prec == 0 else 37.0) * n / self.ncls)
        self.calls.append(("classes", self.prec, n))
        q = np.zeros(self.V)
        return q, q.copy(), self._stats(n)

    def smpq_compute_qx(self, c):
        q, qi, st = self.smpq_compute_qx_classes(c, list(range(self.ncls)))
        return q, qi, 0.0, st

    def smpq_bench_copy(self, c, nbytes, launches):
        self._tick(1.0)
        return 0.87

    def smpq_bench_dslash(self, c, prec, n, sets, launches):
        self._tick(2.0)
        return 1.0, 4e9

    def smpq_get_coloring(self, c):
        return np.arange(self.V) % self.ncls

    def smpq_destroy(self, c):
        pass


def test_driver_command_fits_its_time_limit(monkeypatch, capsys):
    """The driver's command (20 steps, 5 warmup) with a stubbed library and clock: the process
    ends inside its budget, times fewer maps than requested, runs one warmup map and compares
    with a whole FP64 map."""
    import types
    ft = FakeTime()
    stub = StubBinding(ft)
    monkeypatch.setattr(bench, "time", ft)
    monkeypatch.setattr(bench, "T_START", 0.0)
    monkeypatch.setitem(sys.modules, "paper_1901_02211_amd", stub)
    inputs = types.SimpleNamespace(WORKLOADS={"noise16x32": {"dims": (16, 16, 16, 32)}},
                                   workload=lambda name: None)
    monkeypatch.setitem(sys.modules, "smpq_inputs", inputs)
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "1", "--steps", "20", "--warmup", "5", "--no-cpu"])
    bench.main()
    line = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert line["wall_s"] <= 470.0
    assert line["steps_requested"] == 20 and 1 <= line["steps"] < 20
    assert line["warmup"] == 1 and line["warmup_requested"] == 5
    assert line["fp64"]["classes"] == 256 and not line["fp64"]["scaled"]
    assert line["accuracy"]["dQ_over"] == "whole map"
    assert line["value"] == 37.5 and line["roofline"]["bound"] == "hbm"
    sv = line["config"]["stencil_variants"]
    assert sv["f32_kind"] == bench.F32_KINDS[1] and sv["f64_kind"] == "xy-tile" and sv["f64_rhs_per_block"] == 2
    assert sv["f32_dag_kind"] == bench.F32_KINDS[4] and sv["f32_dag_rhs_per_thread"] == 1
    assert sv["f32_dag_interleave"] == sv["f64_interleave"] == 2 and sv["f32_interleave"] == 1
    mixed_maps = [c for c in stub.calls if c[1] == 1 and c[2] == 256]
    assert len(mixed_maps) == line["steps"] + line["warmup"]


def test_cpu_leg_that_does_not_finish_reports_no_value():
    res = bench.cpu_baseline("noise16x32", (16, 16, 16, 32), 4, 10 ** 6, 3072, 8, bench.SMALL_MAP, 0.5)
    assert res["value"] is None and res["kind"] == "oracle" and res["cores"] >= 1
    assert "not finished" in res["sample"]


def test_stencil_bench_variant_parsing():
    """The standalone stencil driver reads kind,nr,band,interleave tuples."""
    from paper_1901_02211_amd.stencil_bench import parse_variant
    assert parse_variant("4,1,1,2") == (4, 1, 1, 2)
    import pytest
    with pytest.raises(ValueError):
        parse_variant("4,1,1")
