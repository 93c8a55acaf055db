"""Centred staggered difference operators (paper Section 5).

G is the discrete gradient from cell-centred pressure to faces,
  (G p) at face_a(i) = (p(i) - p(i - e_a)) / h,
so that G^T is minus the discrete divergence.  D is the reduced deformation
operator from face velocities to the kept stress samples: in 2D
  D_xx = u_x - v_y (cells),  D_xy = u_y + v_x (nodes),
and in 3D
  D_xx = u_x - w_z,  D_yy = v_y - w_z (cells),
  D_xy = u_y + v_x (z-edges),  D_xz = u_z + w_x (y-edges),
  D_yz = v_z + w_y (x-edges).
These rows are the strain-rate combinations that pair with the kept stress
unknowns once tau_yy = -tau_xx (2D) or tau_zz = -tau_xx - tau_yy (3D) is
substituted in tau : grad(u) (Section 5's trace-free reduction).

All difference stencils are two-point centred differences; a neighbour
outside the box does not exist and contributes nothing.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def diff_matrix(grid, src, dst, axis):
    """Sparse (size(dst) x size(src)) matrix of d/dx_axis from samples of
    stagger ``src`` to samples of stagger ``dst``; the two staggers differ on
    ``axis`` only.  If dst is cell-centred on that axis, out[i] =
    (f[i+1] - f[i]) / h; if dst lies on grid lines, out[i] = (f[i] - f[i-1]) / h."""
    d = grid.dim
    for b in range(d):
        assert (src[b] != dst[b]) == (b == axis), (src, dst, axis)
    h = grid.h
    di = grid.index(dst)
    si = grid.index(src)
    sshape = grid.shape(src)
    rows, cols, vals = [], [], []
    if dst[axis] == 1:
        hi_off, lo_off = 1, 0
    else:
        hi_off, lo_off = 0, -1
    for off, sign in ((hi_off, +1.0), (lo_off, -1.0)):
        # source index = destination index + off along axis
        dst_idx = np.indices(grid.shape(dst))
        src_idx = dst_idx.copy()
        src_idx[axis] = src_idx[axis] + off
        ok = (src_idx[axis] >= 0) & (src_idx[axis] < sshape[axis])
        r = di[ok]
        c = si[tuple(src_idx[q][ok] for q in range(d))]
        rows.append(r)
        cols.append(c)
        vals.append(np.full(r.shape, sign / h))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(grid.size(dst), grid.size(src)))


def gradient(grid):
    """G: faces x cells (face blocks in order u, v, w)."""
    return sp.vstack([diff_matrix(grid, grid.cell, grid.faces[a], a) for a in range(grid.dim)]).tocsr()


def deformation(grid):
    """Reduced D: stress samples (order of grid.samples without p) x faces."""
    blocks = []
    for name, st in grid.samples:
        if name == "p":
            continue
        row = []
        terms = {fa: (da, sg) for fa, da, sg in grid.dtilde[name]}
        for fa in range(grid.dim):
            if fa in terms:
                da, sg = terms[fa]
                row.append(sg * diff_matrix(grid, grid.faces[fa], st, da))
            else:
                row.append(sp.csr_matrix((grid.size(st), grid.size(grid.faces[fa]))))
        blocks.append(row)
    return sp.bmat(blocks).tocsr()


def b0(grid):
    """Unweighted face-by-sample operator [G | D^T] (columns in sample order)."""
    return sp.hstack([gradient(grid), deformation(grid).T]).tocsr()
