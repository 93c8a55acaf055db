"""Staggered grid with stresses (paper Section 5, Figs. 1 and 2).

A sample type is described by its *stagger* tuple: per axis, 1 if the sample
sits at cell-centre height along that axis and 0 if it sits on a grid line.
  2D: cell (p, tau_xx) = (1,1); u = (0,1); v = (1,0); node (tau_xy) = (0,0)
  3D: cell (p, tau_xx, tau_yy) = (1,1,1); faces u,v,w = (0,1,1),(1,0,1),(1,1,0);
      tau_xy on z-edges (0,0,1), tau_xz on y-edges (0,1,0),
      tau_yz on x-edges (1,0,0).
A sample of stagger s at index i lies at origin + (i + s/2) h and the array
of that type has shape n + 1 - s.

Trace-free reduction (Section 5): 2D keeps tau_xx (tau_yy = -tau_xx) and
tau_xy; 3D keeps tau_xx, tau_yy (tau_zz = -tau_xx - tau_yy) and the three
off-diagonals.
"""
from __future__ import annotations

import numpy as np

CELL2 = (1, 1)
NODE2 = (0, 0)
CELL3 = (1, 1, 1)


def face_stagger(dim, axis):
    return tuple(0 if b == axis else 1 for b in range(dim))


class Grid:
    """Grid of n cells of size h.  Sample order of the unknown vector x:
    2D [p, txx, txy]; 3D [p, txx, tyy, txy, txz, tyz], each block flattened
    x-fastest.  Face order: [u, v(, w)]."""

    def __init__(self, n, h, origin=None):
        self.n = tuple(int(q) for q in n)
        self.dim = len(self.n)
        assert self.dim in (2, 3)
        self.h = float(h)
        self.origin = tuple(origin) if origin is not None else (0.0,) * self.dim
        d = self.dim
        self.cell = (1,) * d
        self.faces = [face_stagger(d, a) for a in range(d)]
        if d == 2:
            self.samples = [("p", CELL2), ("txx", CELL2), ("txy", NODE2)]
            # reduced deformation rows: list of (face axis, derivative axis, sign)
            self.dtilde = {
                "txx": [(0, 0, +1.0), (1, 1, -1.0)],   # u_x - v_y
                "txy": [(0, 1, +1.0), (1, 0, +1.0)],   # u_y + v_x
            }
        else:
            self.samples = [("p", CELL3), ("txx", CELL3), ("tyy", CELL3),
                            ("txy", (0, 0, 1)), ("txz", (0, 1, 0)), ("tyz", (1, 0, 0))]
            self.dtilde = {
                "txx": [(0, 0, +1.0), (2, 2, -1.0)],   # u_x - w_z
                "tyy": [(1, 1, +1.0), (2, 2, -1.0)],   # v_y - w_z
                "txy": [(0, 1, +1.0), (1, 0, +1.0)],   # u_y + v_x
                "txz": [(0, 2, +1.0), (2, 0, +1.0)],   # u_z + w_x
                "tyz": [(1, 2, +1.0), (2, 1, +1.0)],   # v_z + w_y
            }

    # shapes and sizes ------------------------------------------------------
    def shape(self, stagger):
        return tuple(self.n[a] + 1 - stagger[a] for a in range(self.dim))

    def size(self, stagger):
        return int(np.prod(self.shape(stagger)))

    def sample_sizes(self):
        return [self.size(s) for _, s in self.samples]

    def sample_offsets(self):
        off = np.cumsum([0] + self.sample_sizes())
        return {name: (int(off[q]), int(off[q + 1])) for q, (name, _) in enumerate(self.samples)}

    def face_sizes(self):
        return [self.size(s) for s in self.faces]

    def face_offsets(self):
        off = np.cumsum([0] + self.face_sizes())
        return [(int(off[a]), int(off[a + 1])) for a in range(self.dim)]

    def n_samples(self):
        return int(sum(self.sample_sizes()))

    def n_faces(self):
        return int(sum(self.face_sizes()))

    def coords(self, stagger):
        axes = [self.origin[a] + (np.arange(self.shape(stagger)[a]) + 0.5 * stagger[a]) * self.h
                for a in range(self.dim)]
        return np.meshgrid(*axes, indexing="ij")

    # flattening (x fastest) -------------------------------------------------
    @staticmethod
    def flat(arr):
        return np.asarray(arr, dtype=np.float64).ravel(order="F")

    def unflat(self, vec, stagger):
        return np.asarray(vec).reshape(self.shape(stagger), order="F")

    def index(self, stagger):
        """Flat (x-fastest) index array of a sample type, shaped like it."""
        shp = self.shape(stagger)
        return np.arange(int(np.prod(shp))).reshape(shp, order="F")
