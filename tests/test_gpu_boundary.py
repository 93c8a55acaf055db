"""GPU tests of the C-ABI calls that expose the null-space elimination per
sample type, the residual/correction pairs of the learned preconditioner's
training data, and the context-owned network.

Expected values come from the oracle (active sets, b - A x) or are exact
identities of FP64 arithmetic (x* - x_k is one subtraction on both sides)."""
import numpy as np
import pytest

import cases
from gpu_util import gpu_run
from oracle import system

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[boundary] {msg}", flush=True)


@pytest.mark.parametrize("name", ["drop32", "pool3d_16"])
def test_active_mask_per_sample_type_matches_oracle(name):
    from paper_1010_2832_amd import vfstokes as V
    _banner(f"active mask per sample type: {name}")
    case = cases.drop32() if name == "drop32" else cases.pool3d(16, seed=21)
    asm = system.assemble(case)
    ctx = gpu_run(case, step=False)
    act = system.split_samples(asm.grid, asm.active.astype(np.float64))
    for s, (sname, _) in enumerate(asm.grid.samples):
        got = ctx.vfs_get_active_mask(s)
        assert got.shape == act[sname].shape, sname
        assert np.array_equal(got, act[sname] > 0), sname
    # the all-types form is the concatenation of the per-type masks
    allm = ctx.vfs_get_active()
    cat = np.concatenate([asm.grid.flat(ctx.vfs_get_active_mask(s).astype(np.float64))
                          for s in range(len(asm.grid.samples))]) > 0
    assert np.array_equal(allm, cat)
    with pytest.raises(V.VfsError) as ei:
        ctx.vfs_get_active_mask(len(asm.grid.samples))
    assert ei.value.code == V.VFS_EINVAL
    ctx.close()


def test_training_pair_is_residual_and_correction():
    _banner("training pair on pool3d_16")
    case = cases.pool3d(16, seed=22)
    asm = system.assemble(case)
    ctx = gpu_run(case, step=False)
    rng = np.random.default_rng(3)
    n = asm.grid.n_samples()
    x_star = np.where(asm.active, rng.normal(size=n), 0.0)
    x_k = np.where(asm.active, rng.normal(size=n), 0.0)
    x_k_dirty = x_k + np.where(asm.active, 0.0, 7.0)     # ignored entries of inactive samples
    r, e = ctx.vfs_training_pair(x_star, x_k_dirty)
    r_o = np.where(asm.active, asm.b_full - system.apply(asm, x_k), 0.0)
    scale = np.abs(asm.A_full).sum(axis=1).A1 * np.abs(x_k).max() + np.abs(asm.b_full)
    assert np.all(np.abs(r - r_o) <= 1e-12 * scale.max())
    assert np.array_equal(e, np.where(asm.active, x_star - x_k, 0.0))
    assert not r[~asm.active].any()
    ctx.close()


def test_load_preconditioner_matches_attached_network():
    from paper_1010_2832_amd import learned as L
    from paper_1010_2832_amd import vfstokes as V
    _banner("context-owned network")
    case = cases.pool3d(16, seed=23)
    asm = system.assemble(case)
    w = L.he_init(12, last_scale=1.0)
    rng = np.random.default_rng(4)
    r = np.where(asm.active, rng.normal(size=asm.grid.n_samples()), 0.0)
    ctx = gpu_run(case, precision=V.VFS_MIXED, step=False)
    net = V.Unet()
    net.vfs_unet_set_weights(w)
    ctx.vfs_set_preconditioner(net)
    z_attached = ctx.vfs_precond_apply(r)
    ctx.vfs_set_preconditioner(None)
    net.close()
    ctx.vfs_load_preconditioner(w)
    z_owned = ctx.vfs_precond_apply(r)
    assert np.array_equal(z_owned, z_attached)
    # loading again replaces the weights of the same network
    ctx.vfs_load_preconditioner(np.zeros_like(w))
    z0 = ctx.vfs_precond_apply(r)
    assert not np.array_equal(z0, z_owned)
    with pytest.raises(V.VfsError) as ei:
        ctx.vfs_load_preconditioner(w[:-1])
    assert ei.value.code == V.VFS_EINVAL
    ctx.vfs_set_solver(V.VFS_PRECOND_LEARNED, V.VFS_MIXED, 1e-6, 20000)
    ctx.vfs_load_preconditioner(w)
    ctx.vfs_step(case["dt"])
    assert ctx.vfs_get_stats()["rel_residual"] <= 1e-6
    ctx.close()
    c2 = gpu_run(cases.drop32(), step=False)
    with pytest.raises(V.VfsError) as ei:
        c2.vfs_load_preconditioner(w)
    assert ei.value.code == V.VFS_EINVAL
    c2.close()
