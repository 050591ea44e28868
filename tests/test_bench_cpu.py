"""CPU tests of bench.py's host logic: the one-GPU contract, the timing
helper's warm-up rule and the per-pass byte accounting."""
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


class _Clock:
    """A fake torch whose synchronize advances a fake clock."""

    def __init__(self, step):
        self.t = 0.0
        self.step = step
        self.cuda = types.SimpleNamespace(synchronize=lambda: None)


def test_timed_counts_and_warm_up(monkeypatch):
    clock = _Clock(0.01)
    calls = []

    def fn():
        calls.append(1)
        clock.t += clock.step

    monkeypatch.setattr(bench.time, "perf_counter", lambda: clock.t)
    sec = bench.timed(fn, steps=7, warmup=3, torch=clock)
    assert len(calls) == 10
    assert sec == pytest.approx(0.01)
    # with warm_s, calls continue until that much time has passed, then exactly `steps` are timed
    calls.clear()
    sec = bench.timed(fn, steps=7, warmup=3, torch=clock, warm_s=0.1)
    assert len(calls) == 10 + 7
    assert sec == pytest.approx(0.01)


def test_pass_bytes_and_kind_rows():
    fb = 512 * 512 * 4
    # generation passes write the packed spectrum once; transforms read and write it
    assert bench.pass_bytes(0, fb) == fb
    assert bench.pass_bytes(5, fb) == 2 * fb
    # the column pass without its last stage writes once; the pass that completes it reads and writes
    assert bench.pass_bytes(111, fb) == fb
    assert bench.pass_bytes(112, fb) == 2 * fb
    assert bench.gen_pass_ops_per_point(512, 2) == bench.gen_pass_ops_per_point(512) - (7 + 3.5) / 2
    agg = bench.by_kind([(0, 256, 0.085), (5, 256, 0.080), (0, 256, 0.085), (5, 256, 0.080)], fb)
    assert agg[0]["launches"] == 2 and agg[0]["fields"] == 512
    assert agg[5]["bytes"] == 2 * 2 * fb * 256
    rows = {r["kernel"]: r for r in bench.kind_rows(agg)}
    assert rows[bench.PASS_NAMES[5]]["GBps"] == pytest.approx(2 * 2 * fb * 256 / 0.16e-3 / 1e9, rel=1e-3)
