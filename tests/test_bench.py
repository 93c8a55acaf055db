"""CPU checks of bench.py's contract: refusal of more than one GPU, a loud
failure without a GPU, the algorithmic byte counts per launch, and the HBM
traffic figure, which is reported only while the kernel sources match the
ones the committed counter summary was taken on."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=600, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    p = run_bench("--gpus", "2")
    assert p.returncode == 2
    assert "exactly one GPU" in p.stderr


def test_without_a_gpu_it_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = run_bench("--steps", "1", "--warmup", "0", "--no-cpu", "--no-check")
    assert p.returncode != 0
    assert "needs a GPU" in p.stderr
    assert '"metric"' not in p.stdout


def test_algorithmic_bytes():
    n = 431695
    # fused 2D iteration: read r, q, p, D^-1, x, c (2), write r, x, p, q
    assert bench.fused_bytes(1, n) == 11 * 4 * n
    assert bench.fused_bytes(2, n) == 11 * 8 * n
    # two-kernel iteration: (5 + c) words for the apply, 7 for the update
    assert bench.algorithmic_bytes(2, 1, n) == (7 * 4 * n, 7 * 4 * n)
    a3, u3 = bench.algorithmic_bytes(3, 2, n)
    assert a3 == pytest.approx((5 + 11 / 6) * 8 * n) and u3 == 7 * 8 * n


def test_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    text = open(bench.COUNTERS).read()
    recorded = float(re.search(r"HBM traffic per launch \(bytes, scaled\) \| ([0-9.eE+-]+)", text).group(1))
    # the committed summary matches the committed kernel sources
    assert bench.measured_traffic() == recorded
    # a summary taken on other sources is ignored
    stale = tmp_path / "counters.md"
    stale.write_text(re.sub(r"(sha256 \(k_fused2d.hip \+ vfs_reduce.h\): )[0-9a-f]+", r"\g<1>" + "0" * 64, text))
    monkeypatch.setattr(bench, "COUNTERS", str(stale))
    assert bench.measured_traffic() is None
    # and so is a missing one
    monkeypatch.setattr(bench, "COUNTERS", str(tmp_path / "absent.md"))
    assert bench.measured_traffic() is None
