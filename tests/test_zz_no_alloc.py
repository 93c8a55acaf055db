"""The allocation-free entry point vfs_liquid_weights_noalloc against the
context path it mirrors (vfs_get_weights(..., VFS_WEIGHT_LIQUID)): bit-exact
liquid weights of every sample set, on two calls in a row through the C ABI,
the second on a smaller grid (the shared work space keeps the first call's
contents), plus the rejection of a grid too large for the fixed work space."""
import numpy as np
import pytest

import cases
from gpu_util import gpu_run
from oracle import system

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[noalloc] {msg}", flush=True)


def _sets(V, dim):
    if dim == 2:
        return [(V.VFS_SET_CELL, (1, 1)), (V.VFS_SET_FACE_X, (0, 1)), (V.VFS_SET_FACE_Y, (1, 0)),
                (V.VFS_SET_NODE, (0, 0))]
    return [(V.VFS_SET_CELL, (1, 1, 1)), (V.VFS_SET_FACE_X, (0, 1, 1)), (V.VFS_SET_FACE_Y, (1, 0, 1)),
            (V.VFS_SET_FACE_Z, (1, 1, 0)), (V.VFS_SET_EDGE_Z, (0, 0, 1)), (V.VFS_SET_EDGE_Y, (0, 1, 0)),
            (V.VFS_SET_EDGE_X, (1, 0, 0))]


def _check_case(V, torch, case, stream):
    dim = case["dim"]
    n = case["n"]
    ctx = gpu_run(case, step=False)
    phi = torch.from_numpy(np.ascontiguousarray(np.asarray(case["phi_l"], np.float64).ravel(order="F"))).cuda()
    for sid, st in _sets(V, dim):
        shp = tuple(n[a] + 1 - st[a] for a in range(dim))
        out = torch.full((int(np.prod(shp)),), np.nan, dtype=torch.float64, device="cuda")
        V.vfs_liquid_weights_noalloc(dim, n, 1e-3, phi, sid, out, stream.cuda_stream)
        stream.synchronize()
        got = out.cpu().numpy().reshape(shp, order="F")
        want = ctx.vfs_get_weights(sid, V.VFS_WEIGHT_LIQUID)
        assert np.array_equal(got, want), (case.get("name"), sid)
    ctx.close()


def test_noalloc_liquid_weights_match_the_context_path():
    import torch
    from paper_1010_2832_amd import vfstokes as V
    stream = torch.cuda.current_stream()
    big = [cases.pool3d(40, seed=31), cases.pool2d(160, 3)]
    small = [cases.column3d(16, 3), cases.drop2d(24, 5)]
    for c_big, c_small in zip(big, small):
        _banner(f"large then small: {c_big['n']} -> {c_small['n']}")
        _check_case(V, torch, c_big, stream)
        _check_case(V, torch, c_small, stream)
    # W_L of a tiny grid is also the oracle's (the liquid weights need no solid)
    c = cases.drop2d(8, 1)
    asm = system.assemble(c)
    phi = torch.from_numpy(np.ascontiguousarray(c["phi_l"].ravel(order="F"))).cuda()
    out = torch.empty((9 * 9,), dtype=torch.float64, device="cuda")
    V.vfs_liquid_weights_noalloc(2, c["n"], 1e-3, phi, V.VFS_SET_NODE, out, stream.cuda_stream)
    stream.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(9, 9, order="F"), asm.W[(0, 0)][0])


def test_noalloc_rejects_grids_beyond_its_work_space():
    import torch
    from paper_1010_2832_amd import vfstokes as V
    phi = torch.zeros(8, dtype=torch.float64, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(V.VfsError) as ei:
        V.vfs_liquid_weights_noalloc(3, (80, 80, 80), 1e-3, phi, 0, out)
    assert ei.value.code == V.VFS_EINVAL and "work space" in str(ei.value)
    for bad_set in (3, 7, -1):      # 2D has cells, x and y faces and nodes (VFS_SET_NODE)
        with pytest.raises(V.VfsError) as ei:
            V.vfs_liquid_weights_noalloc(2, (8, 8), 1e-3, phi, bad_set, out)
        assert ei.value.code == V.VFS_EINVAL
