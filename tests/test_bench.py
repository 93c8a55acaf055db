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
    """12 + c values per active DOF and iteration: direction + apply (read r,
    D^-1, p, c coefficients, write p, q) and update (read x, p, r, q, D^-1,
    write x, r); c = 2 in 2D, 11/6 in 3D; FP32 words."""
    n = 431695
    assert bench.pcg_values_per_dof(2) == 14.0
    assert bench.pcg_values_per_dof(3) == pytest.approx(13.0 + 5.0 / 6.0)
    assert bench.fused2d_bytes(n) == 56 * n
    assert bench.fused3d_bytes(n) == pytest.approx(55.333333 * n, rel=1e-6)
    assert bench.fused3d_bytes(38582254) == pytest.approx(2.135e9, rel=1e-3)


def test_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    text = open(bench.COUNTERS_2D).read()
    recorded = float(re.search(r"HBM traffic per launch \(bytes, scaled\) \| ([0-9.eE+-]+)", text).group(1))
    # the committed summary matches the committed kernel sources
    assert bench.measured_traffic_2d() == recorded
    # a summary taken on other sources is ignored
    stale = tmp_path / "counters.md"
    stale.write_text(re.sub(r"(sha256 \(k_fused2d.hip \+ vfs_reduce.h\): )[0-9a-f]+", r"\g<1>" + "0" * 64, text))
    monkeypatch.setattr(bench, "COUNTERS_2D", str(stale))
    assert bench.measured_traffic_2d() is None
    # and so is a missing one
    monkeypatch.setattr(bench, "COUNTERS_2D", str(tmp_path / "absent.md"))
    assert bench.measured_traffic_2d() is None


def test_3d_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    text = open(bench.COUNTERS_3D).read()
    recorded = float(re.search(r"HBM traffic per launch \(one PCG iteration\) \| ([0-9.eE+-]+)",
                               text).group(1))
    assert bench.measured_traffic_3d() == recorded
    # an edit of any of the kernel's sources makes the figure stale
    src = tmp_path / "k_apply3d.hip"
    src.write_text(open(bench.os.path.join(bench.ROOT, bench.KERNEL_SOURCES_3D[0])).read() + "\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES_3D", (str(src),) + bench.KERNEL_SOURCES_3D[1:])
    assert bench.measured_traffic_3d() is None

def test_cpu_oracle_leg_on_the_oracles_own_outputs():
    """The CPU leg fed with the oracle's own step in place of GPU outputs
    reports zero error everywhere (a 2D result, a batched problem, a 3D
    result on sub-boxes), and a planted velocity error shows up in the 3D
    sub-box figure.  The baseline runs on a sub-box and records the host."""
    import numpy as np

    import cases
    from cases import crop_maps
    from oracle import system

    c2 = cases.pool2d(48, 2)
    c2.setdefault("name", "pool2d_48")
    asm, x, u = system.step(c2)
    main = {"velocity": system.split_faces(asm.grid, u), "solution": x,
            "active": asm.active.astype(np.uint8)}
    cb = cases.drop2d(40, 4)
    ab, xb, ub = system.step(cb)
    batch = [{"problem": 0, "case": cb, "tol": 1e-9, "velocity": system.split_faces(ab.grid, ub),
              "solution": xb}]
    c3 = cases.column3d(36, 3)
    a3, x3, u3 = system.step(c3)
    v3 = system.split_faces(a3.grid, u3)
    got3 = {"exact": {"velocity": v3, "solution": x3, "rhs": a3.b_full,
                      "active": a3.active.astype(np.uint8)},
            "planted": {"velocity": [q * (1.0 + 1e-5) for q in v3], "solution": x3}}
    base = cases.crop(cases.pool3d(32, 5), (4, 4, 4), (16, 16, 16))
    res = bench.cpu_oracle_leg(base, 5, None, batch, baseline=True, check=True,
                               extra3d=[("c3", c3, crop_maps.sites_column, got3)],
                               extra2d=[("c2", c2, main)])
    e = res["c2"]
    assert e["velocity_rel_linf"] == 0.0 and e["active_mask_identical"]
    assert e["rel_residual_measured_by_oracle"] < 1e-10
    eb = res["batch64_error_vs_fp64_oracle"][0]
    assert eb["velocity_rel_linf"] == 0.0 and eb["rel_residual_measured_by_oracle"] < 1e-10
    assert eb["tol"] == 1e-9
    e3 = res["c3"]
    assert e3["active_mask_identical"] and len(e3["sub_boxes"]) == 2
    assert all(b["active_compared"] > 0 for b in e3["sub_boxes"])
    assert e3["exact"]["local_backward_error"] < 1e-13
    assert e3["exact"]["local_residual_vs_global_b"] < 1e-12
    assert e3["exact"]["velocity_rel_linf_vs_oracle_recovery"] < 1e-12
    assert 5e-6 < e3["planted"]["velocity_rel_linf_vs_oracle_recovery"] < 2e-5
    # a planted error in the solution shows in the local backward error
    noise = np.random.default_rng(0).normal(size=x3.size) * a3.active
    got_bad = {"exact": dict(got3["exact"], solution=x3 + 1e-3 * np.abs(x3).max() * noise)}
    r_bad = bench.cpu_oracle_leg(None, 0, None, None, baseline=False, check=True,
                                 extra3d=[("c3", c3, crop_maps.sites_column, got_bad)])
    assert r_bad["c3"]["exact"]["local_backward_error"] > 1e-5
    cb_ = res["cpu_baseline"]
    assert cb_["kind"] == "oracle" and cb_["cores"] == 1 and cb_["value"] > 0
    assert cb_["logical_cpus"] == os.cpu_count() and "sub-box" in cb_["sample"]
