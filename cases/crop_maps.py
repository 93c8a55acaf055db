"""Index maps between a sub-box of a case (cases.crop) and the full case, for
checks at full size on pieces the oracle can assemble, and the sub-boxes
those checks use on the two 3D workloads.  Every quantity of one sample
(weights, coefficients, activity, right-hand side, the rows of A and the
recovered velocity) depends only on the case within a few cells of it, so
at samples far enough from the sub-box boundary the oracle's sub-box values
equal the full case's.  Like the rest of this package, nothing here is the
method's arithmetic: grids are passed in and only their index layout is
used."""
import numpy as np

MARGIN = 3   # index steps between a compared sample and the sub-box boundary
CROP = 24    # cells per axis of a 3D sub-box


def crop_lo(case, centre, m=CROP):
    """Lower cell corner of the m^3 sub-box centred (as far as the grid
    allows) on the point `centre`."""
    n, h = case["n"], case["h"]
    return tuple(int(np.clip(round(centre[a] / h) - m // 2, 0, n[a] - m)) for a in range(3))


def sites_pool(case):
    """Sub-boxes of the 3D pool: where the moving solid sphere meets the
    liquid (else a box corner under the pool), on the pool surface and on a
    liquid sphere's surface."""
    h = case["h"]
    ps = np.asarray(case["phi_s"])
    pl = np.asarray(case["phi_l"])
    contact = np.argwhere((np.abs(ps) < 2 * h) & (pl < 0))
    solid = contact[len(contact) // 2] * h if len(contact) else np.array([0.05, 0.05, 0.05])
    ny = pl.shape[1]
    band = np.argwhere((np.abs(pl) < h) & (np.arange(ny)[None, :, None] * h > 0.45))
    drop = band[len(band) // 2] * h
    return [("solid sphere", solid), ("pool surface", (0.5, 0.3, 0.5)), ("liquid sphere", drop)]


def sites_column(case):
    """Sub-boxes of the 3D column: its foot on the floor and its top."""
    return [("column foot", (0.5, 0.1, 0.5)), ("column top", (0.5, 0.8, 0.5))]


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
