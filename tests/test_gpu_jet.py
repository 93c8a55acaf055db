"""The jet-buckling applications of the fractional step (Section 10) as
qualitative GPU checks: a 2D planar jet at 150^2 (disc container, ceiling
nozzle moving down at 0.5, mu 0.075) and a 3D cylindrical jet at 80^3
(spherical container, mu 0.3), stepped with vfs_advect + vfs_step in mixed
precision with warm-started solves, the nozzle kept filled through the
liquid level set.  Each step must converge; the liquid volume must grow at
the nozzle's inflow rate (within the volume-fraction accuracy of the level
set) and the jet's lowest point must fall under gravity."""
import numpy as np
import pytest

import cases

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[jet] {msg}", flush=True)


def _run(case, steps, tol=1e-6):
    from paper_1010_2832_amd import vfstokes as V
    ctx = V.context_from_case(case, precision=V.VFS_MIXED, tol=tol)
    ctx.vfs_set_warm_start(True)
    dt = case["dt"]
    d = case["dim"]
    cell = V.VFS_SET_CELL
    seed = case["jet_seed"]
    vols, tips, its = [], [], []
    phi = np.asarray(case["phi_l"])
    for step in range(steps):
        ctx.vfs_advect(dt)
        phi = np.minimum(ctx.vfs_get_level_set(), seed)
        ctx.vfs_set_level_sets(phi, case["phi_s"])
        ctx.vfs_step(dt)
        st = ctx.vfs_get_stats()
        assert st["rel_residual"] <= tol, (step, st)
        its.append(st["iterations"])
        wl = ctx.vfs_get_weights(cell, V.VFS_WEIGHT_LIQUID)
        wf = ctx.vfs_get_weights(cell, V.VFS_WEIGHT_FLUID)
        vols.append(float((wl * wf).sum()) * case["h"] ** d)
        liquid_y = np.argwhere(phi < 0)[:, 1] * case["h"]
        tips.append(float(liquid_y.min()))
    u = np.concatenate([np.ravel(q) for q in ctx.vfs_get_velocity()])
    ctx.close()
    assert np.isfinite(u).all()
    return np.array(vols), np.array(tips), its, np.abs(u).max()


def test_planar_jet_2d():
    case = cases.jet2d(150)
    steps = 60
    vols, tips, its, umax = _run(case, steps)
    t = steps * case["dt"]
    inflow = 0.06 * 0.5 * t
    _banner(f"2D jet 150^2, {steps} steps: liquid area {vols[0]:.5f} -> {vols[-1]:.5f} "
            f"(inflow {inflow:.5f}), tip y {tips[0]:.3f} -> {tips[-1]:.3f}, max |u| {umax:.2f}, "
            f"iterations {its[0]} .. {its[-1]} (total {sum(its)})")
    gain = vols[-1] - vols[0]
    assert 0.5 * inflow < gain < 1.5 * inflow
    assert tips[-1] < tips[0] - 0.05
    assert umax < 5.0


def test_cylindrical_jet_3d():
    case = cases.jet3d(80)
    steps = 25
    vols, tips, its, umax = _run(case, steps)
    t = steps * case["dt"]
    inflow = np.pi * 0.04 ** 2 * 0.5 * t
    _banner(f"3D jet 80^3, {steps} steps: liquid volume {vols[0]:.6f} -> {vols[-1]:.6f} "
            f"(inflow {inflow:.6f}), tip y {tips[0]:.3f} -> {tips[-1]:.3f}, max |u| {umax:.2f}, "
            f"iterations {its[0]} .. {its[-1]} (total {sum(its)})")
    gain = vols[-1] - vols[0]
    assert 0.3 * inflow < gain < 2.0 * inflow
    assert tips[-1] < tips[0] - 0.01
    assert umax < 5.0
