"""GPU parity of the fractional step of Section 10 (vfs_advect + vfs_step)
against the oracle (oracle/advect.py): one advection of a given velocity
and level set to 1e-12, several full steps (advection, body force, Stokes
solve) to the FP64 bar, and warm-started mixed solves across steps."""
import numpy as np
import pytest

import cases
from gpu_util import flat_faces, gpu_run, velocity_rel_linf
from oracle import advect, system
from oracle.grid import Grid

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[advect] {msg}", flush=True)


def _swirl(case, amp=0.8):
    """A smooth rotating velocity (so departure points are off the grid)."""
    out = dict(case)
    n, h, d = case["n"], case["h"], case["dim"]
    u = []
    for a in range(d):
        F = cases.face_coords(n, h, (0.0,) * d, a)
        r = [F[q] - 0.5 for q in range(d)]
        rot = [-r[1], r[0], 0.3 * r[0]][a] if d == 3 else [-r[1], r[0]][a]
        u.append(amp * rot + 0.1 * np.sin(3 * F[0] + 2 * F[1]))
    out["u"] = u
    return out


CASES = {
    "drop2d_33": lambda: _swirl(cases.drop2d(33, 3, dt=0.01)),
    "pool3d_12": lambda: _swirl(cases.pool3d(12, seed=9, dt=0.01)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_one_advection_matches_oracle(name):
    case = CASES[name]()
    grid = Grid(case["n"], case["h"])
    dt = 0.02
    ctx = gpu_run(case, step=False)
    ctx.vfs_advect(dt)
    u_g = flat_faces(grid, ctx.vfs_get_velocity())
    phi_g = ctx.vfs_get_level_set()
    u = [np.asarray(q, np.float64) for q in case["u"]]
    u_o = advect.advect_velocity(grid, u, dt)
    phi_o = advect.advect_level_set(grid, case["phi_l"], u, dt)
    du = np.abs(u_g - flat_faces(grid, u_o)).max() / np.abs(flat_faces(grid, u_o)).max()
    dp = np.abs(phi_g - phi_o).max() / np.abs(phi_o).max()
    _banner(f"{name}: velocity {du:.2e}, level set {dp:.2e}")
    assert du <= 1e-12 and dp <= 1e-12
    ctx.close()


@pytest.mark.parametrize("name", list(CASES))
def test_fractional_steps_match_oracle(name):
    """Three steps: the second and third extend the previous Stokes step's
    velocity into the air before advecting (the faces it defined), so the
    GPU's bookkeeping of known faces is checked too."""
    from paper_1010_2832_amd import vfstokes as V
    case = CASES[name]()
    dt = 0.01
    ctx = gpu_run(case, precision=V.VFS_FP64, tol=1e-12, step=False)
    c = case
    prev = None
    for step in range(3):
        c, (asm, x, u_o) = advect.ns_step(c, dt, prev)
        prev = asm
        ctx.vfs_advect(dt)
        phi_g = ctx.vfs_get_level_set()
        ctx.vfs_step(dt)
        u_g = flat_faces(asm.grid, ctx.vfs_get_velocity())
        err = velocity_rel_linf(asm, u_g, u_o)
        dphi = np.abs(phi_g - c["phi_l"]).max() / np.abs(c["phi_l"]).max()
        _banner(f"{name} step {step}: velocity rel Linf {err:.2e}, level set {dphi:.2e}, "
                f"iterations {ctx.vfs_get_stats()['iterations']}")
        assert np.array_equal(ctx.vfs_get_active(), asm.active)
        assert err <= 1e-6 and dphi <= 1e-9
    ctx.close()


def test_warm_start_across_steps():
    """Mixed solves started from the previous step's solution converge to the
    same velocities as cold starts, from a starting residual well below |b|.
    (The iteration counts are reported, not asserted: each FP32 inner solve
    reduces its residual by a bounded factor, so a tight tolerance needs about
    as many inner iterations from a warm start as from zero.)"""
    from paper_1010_2832_amd import vfstokes as V
    case = cases.pool2d(96, 7)
    dt = case["dt"]
    res = {}
    for warm in (False, True):
        ctx = gpu_run(case, precision=V.VFS_MIXED, tol=1e-8, step=False)
        ctx.vfs_set_warm_start(warm)
        its, vel, start = [], [], []
        for _ in range(4):
            ctx.vfs_advect(dt)
            ctx.vfs_step(dt)
            st = ctx.vfs_get_stats()
            assert st["rel_residual"] <= 1e-8
            its.append(st["iterations"])
            start.append(st["rel_residual_start"])
            vel.append(np.concatenate([np.ravel(q) for q in ctx.vfs_get_velocity()]))
        res[warm] = (its, vel, start)
        ctx.close()
    _banner(f"iterations cold {res[False][0]}, warm {res[True][0]}; starting residual "
            f"warm {np.round(res[True][2], 5)}")
    assert res[True][0][0] == res[False][0][0]
    assert res[False][2] == [1.0] * 4 and res[True][2][0] == 1.0
    assert max(res[True][2][1:]) < 0.5
    for vc, vw in zip(res[False][1], res[True][1]):
        assert np.abs(vc - vw).max() <= 1e-4 * np.abs(vc).max()
