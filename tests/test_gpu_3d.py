"""GPU parity of the 3D path against the oracle (through the C ABI): bit-exact
weights and masks, right-hand side and A x to 1e-12, velocity relative
L-inf 1e-6 (FP64) / 1e-4 (mixed)."""
import numpy as np
import pytest

import cases
from gpu_util import expected_tile_samples, flat_faces, gpu_run, oracle, velocity_rel_linf
from oracle import system

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[gpu3d] {msg}", flush=True)


def _random3d(nx, ny, nz, seed, moving=True):
    rng = np.random.default_rng(seed)
    nn = (nx, ny, nz)
    h = 1.0 / max(nn)
    X = cases.node_coords(nn, h, (0.0, 0.0, 0.0))
    L = [q * h for q in nn]
    phi_l = np.minimum(np.sqrt((X[0] - 0.5 * L[0]) ** 2 + (X[1] - 0.6 * L[1]) ** 2 + (X[2] - 0.5 * L[2]) ** 2)
                       - 0.3 * min(L), X[1] - 0.3 * L[1])
    phi_s = np.sqrt((X[0] - 0.45 * L[0]) ** 2 + (X[1] - 0.25 * L[1]) ** 2 + (X[2] - 0.55 * L[2]) ** 2) - 0.15 * min(L)
    u = [rng.normal(0, 0.2, size=s) for s in cases.face_shapes(nn)]
    ubc = [np.full(s, 0.4 * (a - 1)) for a, s in enumerate(cases.face_shapes(nn))] if moving else None
    return dict(dim=3, n=nn, h=h, origin=(0.0, 0.0, 0.0), dt=0.01, phi_l=phi_l, phi_s=phi_s,
                rho=rng.uniform(0.5, 2.0, size=nn), mu=rng.uniform(0.5, 5.0, size=nn),
                u=u, u_bc=ubc, g=(0.0, -9.8, 0.0), name=f"rand3d_{nx}x{ny}x{nz}")


CASES = {
    "rand8": lambda: _random3d(8, 8, 8, 1),
    "rand13x7x9": lambda: _random3d(13, 7, 9, 2),
    "rand70x9x11": lambda: _random3d(70, 9, 11, 3),
    # nx a multiple of 64: the anchors i = 0..nx take one 64-wide x tile more,
    # holding only the wall column i = nx, which the fused mixed iteration
    # folds into the x tile before it
    "rand64x9x11": lambda: _random3d(64, 9, 11, 6),
    "rand128x6x5": lambda: _random3d(128, 6, 5, 7),
    "column32": lambda: cases.column3d(32, seed=3),
    "pool24": lambda: cases.pool3d(24, seed=5),
}


@pytest.mark.parametrize("name", list(CASES))
def test_weights_and_masks_bitexact_3d(name):
    from paper_1010_2832_amd import vfstokes as V
    _banner(f"weights/masks {name}")
    case = CASES[name]()
    asm = system.assemble(case)
    ctx = gpu_run(case, step=False)
    g = asm.grid
    sets = [(V.VFS_SET_CELL, g.cell), (V.VFS_SET_FACE_X, g.faces[0]), (V.VFS_SET_FACE_Y, g.faces[1]),
            (V.VFS_SET_FACE_Z, g.faces[2]), (V.VFS_SET_EDGE_Z, (0, 0, 1)), (V.VFS_SET_EDGE_Y, (0, 1, 0)),
            (V.VFS_SET_EDGE_X, (1, 0, 0))]
    for sid, st in sets:
        assert np.array_equal(ctx.vfs_get_weights(sid, V.VFS_WEIGHT_LIQUID), asm.W[st][0]), (name, sid)
        wf = ctx.vfs_get_weights(sid, V.VFS_WEIGHT_FLUID)
        if st in g.faces:
            lo, hi = g.face_offsets()[g.faces.index(st)]
            assert np.array_equal(g.flat(wf), asm.wf_f[lo:hi]), (name, sid)
        else:
            assert np.array_equal(wf, asm.W[st][1]), (name, sid)
    act = ctx.vfs_get_active()
    assert np.array_equal(act, asm.active), (name, int((act != asm.active).sum()))


@pytest.mark.parametrize("name", list(CASES))
def test_rhs_and_apply_3d(name):
    _banner(f"rhs/apply {name}")
    case = CASES[name]()
    asm = system.assemble(case)
    ctx = gpu_run(case, step=False)
    b = ctx.vfs_get_rhs()
    assert np.abs(b - asm.b_full).max() <= 1e-12 * max(np.abs(asm.b_full).max(), 1e-300)
    rng = np.random.default_rng(4)
    x = rng.normal(size=asm.grid.n_samples())
    y = ctx.vfs_apply(x)
    ref = system.apply(asm, x)
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name", list(CASES))
def test_step_fp64_3d(name):
    _banner(f"step fp64 {name}")
    case = CASES[name]()
    asm, x, u = oracle(case)
    ctx = gpu_run(case, tol=1e-11)
    st = ctx.vfs_get_stats()
    ug = flat_faces(asm.grid, ctx.vfs_get_velocity())
    err = velocity_rel_linf(asm, ug, u)
    _banner(f"  active {st['n_active']} iters {st['iterations']} rel_res {st['rel_residual']:.2e} vel err {err:.2e}")
    assert st["rel_residual"] <= 1e-11
    assert err <= 1e-6
    assert system.true_relative_residual(asm, ctx.vfs_get_solution()) <= 1e-10


@pytest.mark.parametrize("name", ["rand13x7x9", "rand70x9x11", "rand64x9x11", "rand128x6x5",
                                  "column32", "pool24"])
def test_step_mixed_3d(name):
    _banner(f"step mixed {name}")
    case = CASES[name]()
    asm, x, u = oracle(case)
    ctx = gpu_run(case, precision=1, tol=1e-9)
    st = ctx.vfs_get_stats()
    ug = flat_faces(asm.grid, ctx.vfs_get_velocity())
    err = velocity_rel_linf(asm, ug, u)
    _banner(f"  iters {st['iterations']} outer {st['outer_iterations']} rel_res {st['rel_residual']:.2e} vel err {err:.2e}")
    assert st["rel_residual"] <= 1e-9
    assert err <= 1e-4
    # the active-tile list covers exactly the 64x4x8 tiles holding an active sample
    assert st["n_tile_samples"] == expected_tile_samples(asm, (64, 4, 8))


def test_mixed_work_queue_matches_fp64():
    """A grid whose fused work list outlasts two fixed rounds of the resident
    grid, so that the mixed iteration's workgroups claim items from the
    per-XCD counters: the mixed step must give the FP64 step's velocity (the
    FP64 path has no work queue; the oracle cannot solve this size in a test)
    to the mixed bar, on two consecutive solves (the counters carry over)."""
    import torch
    from paper_1010_2832_amd import vfstokes as V
    case = cases.pool3d(192, seed=9)
    _banner("work queue: pool3d 192 FP64 step")
    c64 = gpu_run(case, precision=0, tol=1e-9)
    s64 = c64.vfs_get_stats()
    u64 = np.concatenate([q.ravel() for q in c64.vfs_get_velocity()])
    tiles = s64["n_tile_samples"] // (64 * 4 * 8 * 6)
    grid = 2 * torch.cuda.get_device_properties(0).multi_processor_count
    # the fused list drops the tiles of the folded wall column (one x tile in
    # four at n = 192); more than two rounds of the grid must remain
    assert tiles * 3 // 4 > 2 * grid, (tiles, grid)
    c32 = V.context_from_case(case, precision=1, tol=1e-9, max_iter=200000)
    for rep in range(2):
        _banner(f"work queue: pool3d 192 mixed step, solve {rep}")
        c32.vfs_set_velocity(case["u"])
        c32.vfs_step(case["dt"])
        s32 = c32.vfs_get_stats()
        u32 = np.concatenate([q.ravel() for q in c32.vfs_get_velocity()])
        err = np.abs(u32 - u64).max() / np.abs(u64).max()
        _banner(f"  tiles {tiles} grid {grid} iters {s32['iterations']} rel_res {s32['rel_residual']:.2e} "
                f"vel vs FP64 {err:.2e}")
        assert s32["status"] == 0 and s32["rel_residual"] <= 1e-9
        assert err <= 1e-4


def test_no_liquid_3d():
    c = _random3d(9, 8, 7, 9)
    c["phi_l"] = np.ones_like(c["phi_l"])
    asm, x, u = oracle(c)
    for prec in (0, 1):
        ctx = gpu_run(c, precision=prec)
        assert ctx.vfs_get_stats()["n_active"] == 0
        assert np.array_equal(flat_faces(asm.grid, ctx.vfs_get_velocity()), u)
