"""Host logic of bench.py (no GPU): the multi-GPU refusal, the byte accounting of the
roofline, and the committed traffic file that the benchmark line's measured traffic comes
from (its figures recompute from its own counter values, and it is used only while its
kernel source hash matches the sources)."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("nf, fp32, want", [(3, False, 240.0), (2, False, 120.0), (3, True, 120.0),
                                            (2, True, 60.0)])
def test_bytes_per_beam_step(nf, fp32, want):
    # the state read at stages 2, 3, 4 and the final pass and written once: 5 passes over
    # 2 NF - 1 (two flavours: the Bloch vector, 3) or 2 NF (three: psi, 6) reals
    assert bench.bytes_per_beam_step(nf, fp32) == want


def test_kernel_source_hash_is_stable():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and all(c in "0123456789abcdef" for c in h)
    assert bench.kernel_source_hash() == h


def test_traffic_file_is_consistent():
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic_k_advance_3f_fp64_800k.json")))
    # calibration: the 1 GiB copy reads and writes 1048576 KiB
    assert t["read_scale"] == pytest.approx(1048576.0 / t["copy_kernel_fetch_kib_for_1GiB_read"])
    assert t["write_scale"] == pytest.approx(1048576.0 / t["copy_kernel_write_kib_for_1GiB_write"])
    steps, beams = 50, 800000
    rd = t["fetch_kib_per_launch"] * 1024 * t["read_scale"] / steps
    wr = t["write_kib_per_launch"] * 1024 * t["write_scale"] / steps
    assert t["hbm_read_bytes_per_step"] == pytest.approx(rd)
    assert t["hbm_write_bytes_per_step"] == pytest.approx(wr)
    assert t["hbm_bytes_per_beam_step"] == pytest.approx((rd + wr) / beams)
    # a stepper that moves more than its algorithmic bytes would be re-reading state
    assert 0.0 < t["hbm_bytes_per_beam_step"] <= t["algorithmic_bytes_per_beam_step"]


def test_traffic_is_used_only_with_matching_sources(monkeypatch):
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic_k_advance_3f_fp64_800k.json")))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: t["kernel_source_hash"])
    assert bench.traffic_from_profile("k_advance_3f_fp64_800k", 20, 800000) == pytest.approx(
        t["hbm_bytes_per_beam_step"] * 20 * 800000)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.traffic_from_profile("k_advance_3f_fp64_800k", 20, 800000) is None
    assert bench.traffic_from_profile("no_such_kernel", 20, 800000) is None


class _CountingModel:
    """Stands in for a model: counts the steps and resets the clock warm-up asks for."""

    def __init__(self, n_steps):
        self.ds = [{"n_steps": n_steps}]
        self.i, self.calls, self.resets = 0, [], 0

    def step_index(self):
        return self.i

    def step(self, k):
        self.calls.append(k)
        self.i = min(self.i + k, self.ds[0]["n_steps"])

    def reset(self):
        self.resets += 1
        self.i = 0


def test_clock_warmup_stays_within_the_run_and_resets():
    m = _CountingModel(100)
    cw = bench.warm_clock(m, 10.0)     # the run's end stops it long before 10 s
    assert m.calls == [1, 2, 4, 8, 16, 32, 32]
    assert cw["steps"] == 95 and cw["launches"] == 7
    assert m.resets == 1 and m.step_index() == 0


def test_clock_warmup_off():
    m = _CountingModel(100)
    cw = bench.warm_clock(m, 0.0)
    assert m.calls == [] and cw["steps"] == 0 and cw["launches"] == 0
    assert m.resets == 1 and m.step_index() == 0
