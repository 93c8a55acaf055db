"""GPU parity of the prescribed-traction free surface (Section 6.1) against
the oracle, through the C ABI: the right-hand side to 1e-12 (it carries all
of the traction terms, including the 3D coupling of an eliminated tau_yy),
the velocity after an FP64 step to 1e-6 and after a mixed step to 1e-4, and
the uniform-pressure shift."""
import numpy as np
import pytest

import cases
import manufactured
from gpu_util import flat_faces, gpu_run, velocity_rel_linf
from oracle import system
from oracle.grid import Grid
from test_oracle_system import _box_case, _moving_solid_case
from test_oracle_traction import _smooth_bc, _with_traction

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[traction] {msg}", flush=True)


def _traction_case(dim, n, seed):
    rng = np.random.default_rng(seed)
    phi_l, phi_s, ubc, _ = _moving_solid_case(dim, n, rng)
    ubc = [q + rng.normal(0, 0.2, size=q.shape) for q in ubc]
    g = [0.0] * dim
    g[1] = -9.8
    c = _box_case(dim, n, phi_l, phi_s, rng, ubc=ubc, g=tuple(g))
    p_bc, tau_bc = _smooth_bc(Grid(c["n"], c["h"]), rng)
    return _with_traction(c, p_bc, tau_bc)


CASES = {
    "2d_24": lambda: _traction_case(2, 24, 71),
    "2d_37": lambda: _traction_case(2, 37, 72),
    "3d_7": lambda: _traction_case(3, 7, 67),
    "3d_14": lambda: _traction_case(3, 14, 73),
}


@pytest.mark.parametrize("name", list(CASES))
def test_traction_rhs_and_velocity_match_oracle(name):
    from paper_1010_2832_amd import vfstokes as V
    case = CASES[name]()
    _banner(f"{name}: {case['n']}")
    asm, x, u = system.step(case)
    ctx = gpu_run(case, step=False)
    b = ctx.vfs_get_rhs()
    assert np.array_equal(ctx.vfs_get_active(), asm.active)
    scale = max(np.abs(asm.b_full).max(), 1e-300)
    err_b = np.abs(b - asm.b_full).max() / scale
    _banner(f"  rhs max rel err {err_b:.2e}")
    assert err_b <= 1e-12
    for prec, tol, bar in ((V.VFS_FP64, 1e-10, 1e-6), (V.VFS_MIXED, 1e-9, 1e-4)):
        ctx.vfs_set_solver(V.VFS_PRECOND_JACOBI, prec, tol, 200000, 1e-3)
        ctx.vfs_set_velocity(case["u"])
        ctx.vfs_step(case["dt"])
        err = velocity_rel_linf(asm, flat_faces(asm.grid, ctx.vfs_get_velocity()), u)
        _banner(f"  precision {prec}: velocity rel Linf vs oracle {err:.2e}")
        assert err <= bar
    ctx.close()


def test_uniform_pressure_shift_on_gpu():
    from paper_1010_2832_amd import vfstokes as V
    rng = np.random.default_rng(81)
    n = 40
    phi_l, phi_s, ubc, _ = _moving_solid_case(2, n, rng)
    base = _box_case(2, n, phi_l, phi_s, rng, ubc=ubc, g=(0.0, -9.8))
    p0 = 2.5
    c0 = gpu_run(base, tol=1e-12)
    c1 = gpu_run(_with_traction(base, p_bc=np.full((n, n), p0)), tol=1e-12)
    u0 = np.concatenate([np.ravel(q) for q in c0.vfs_get_velocity()])
    u1 = np.concatenate([np.ravel(q) for q in c1.vfs_get_velocity()])
    assert np.abs(u1 - u0).max() <= 1e-8 * max(np.abs(u0).max(), 1.0)
    act = c0.vfs_get_active_mask(V.VFS_SAMPLE_P)
    dp = (c1.vfs_get_pressure() - c0.vfs_get_pressure())[act]
    _banner(f"uniform p0 = {p0}: pressure shift {dp.min():.9f} .. {dp.max():.9f}")
    assert np.abs(dp - p0).max() <= 1e-8 * p0
    # switching the terms off restores the plain step
    c1.vfs_set_traction(None, None)
    c1.vfs_set_velocity(base["u"])
    c1.vfs_step(base["dt"])
    u2 = np.concatenate([np.ravel(q) for q in c1.vfs_get_velocity()])
    assert np.abs(u2 - u0).max() <= 1e-8 * max(np.abs(u0).max(), 1.0)
    with pytest.raises(V.VfsError) as ei:
        c1.vfs_set_traction(np.full((n, n), np.nan), None)
    assert ei.value.code == V.VFS_EINVAL
    c0.close()
    c1.close()


def test_manufactured_drop_with_surface_traction():
    """The drop of the convergence pin (exact fields with non-zero surface
    traction) at 96^2: the GPU's FP64 step equals the oracle's."""
    from test_oracle_traction import _drop_errors  # noqa: F401  (same construction)
    f = manufactured.functions(2)
    n = 96
    case = manufactured.make_case(2, n)
    h = 1.0 / n
    X, Y = cases.node_coords((n, n), h, (0.0, 0.0))
    case["phi_l"] = np.hypot(X - 0.5, Y - 0.5) - 0.35
    C = cases.cell_coords((n, n), h, (0.0, 0.0))
    N = cases.node_coords((n, n), h, (0.0, 0.0))
    case = _with_traction(case, manufactured._ev(f["p"], C),
                          [manufactured._ev(f["tau00"], C), manufactured._ev(f["tau01"], N)])
    asm, x, u = system.step(case)
    ctx = gpu_run(case, tol=1e-11)
    err = velocity_rel_linf(asm, flat_faces(asm.grid, ctx.vfs_get_velocity()), u)
    ue = np.concatenate([asm.grid.flat(q) for q in manufactured.exact_velocity(2, n)])
    m = asm.K > 0
    ex = np.abs(flat_faces(asm.grid, ctx.vfs_get_velocity())[m] - ue[m]).max()
    _banner(f"manufactured drop {n}^2: velocity vs oracle {err:.2e}, vs exact {ex:.2e}")
    assert err <= 1e-6
    ctx.close()
