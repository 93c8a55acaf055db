"""Index maps between a sub-box of a case (cases.crop) and the full case, for
checks at full size on pieces the oracle can assemble.  Every quantity of one
sample (weights, coefficients, activity, right-hand side, the rows of A and
the recovered velocity) depends only on the case within a few cells of it,
so at samples far enough from the sub-box boundary the oracle's sub-box
values equal the full case's."""
import numpy as np

MARGIN = 3   # index steps between a compared sample and the sub-box boundary


def _block_map(full_shape, crop_shape, lo, margin, f_off, c_off):
    d = len(full_shape)
    rng = [np.arange(margin, crop_shape[a] - margin) for a in range(d)]
    if any(len(q) == 0 for q in rng):
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    g = np.meshgrid(*rng, indexing="ij")
    ci = np.ravel_multi_index([q.ravel() for q in g], crop_shape, order="F") + c_off
    fi = np.ravel_multi_index([(q + lo[a]).ravel() for a, q in enumerate(g)], full_shape,
                              order="F") + f_off
    return ci, fi


def sample_map(full_grid, crop_grid, lo, margin=MARGIN):
    """(crop indices, full indices) in sample order of the crop's samples at
    least `margin` index steps from its boundary (margin 0: every sample)."""
    fo, co = full_grid.sample_offsets(), crop_grid.sample_offsets()
    cs, fs = [], []
    for name, st in full_grid.samples:
        c, f = _block_map(full_grid.shape(st), crop_grid.shape(st), lo, margin, fo[name][0],
                          co[name][0])
        cs.append(c)
        fs.append(f)
    return np.concatenate(cs), np.concatenate(fs)


def face_map(full_grid, crop_grid, lo, margin=MARGIN):
    """(crop indices, full indices) in face order, as sample_map."""
    fo, co = full_grid.face_offsets(), crop_grid.face_offsets()
    cs, fs = [], []
    for a, st in enumerate(full_grid.faces):
        c, f = _block_map(full_grid.shape(st), crop_grid.shape(st), lo, margin, fo[a][0],
                          co[a][0])
        cs.append(c)
        fs.append(f)
    return np.concatenate(cs), np.concatenate(fs)
