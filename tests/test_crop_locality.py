"""The premise of the full-size GPU checks: the oracle's assembly of a
sub-box (cases.crop) agrees exactly with its assembly of the whole case at
every sample and face at least cases.crop_maps.MARGIN index steps inside the
sub-box (weights, coefficients, activity, right-hand side, rows of A, and the
velocity recovered from a given solution)."""
import numpy as np
import pytest

import cases
from cases.crop_maps import MARGIN, face_map, sample_map
from oracle import system


@pytest.mark.parametrize("make,lo,m", [
    (lambda: cases.pool3d(16, seed=3), (2, 3, 4), (11, 10, 11)),
    (lambda: cases.pool512(n=48), (9, 4, ), (26, 24)),
])
def test_crop_interior_matches_full(make, lo, m):
    full = make()
    A = system.assemble(full)
    C = system.assemble(cases.crop(full, lo, m))
    ci, fi = sample_map(A.grid, C.grid, lo)
    fci, ffi = face_map(A.grid, C.grid, lo)
    assert len(ci) > 0 and len(fci) > 0
    assert np.array_equal(A.wl_s[fi], C.wl_s[ci])
    assert np.array_equal(A.wf_s[fi], C.wf_s[ci])
    assert np.array_equal(A.active[fi], C.active[ci])
    assert A.active[fi].any() and not A.active[fi].all()
    assert np.array_equal(A.K[ffi], C.K[fci])
    assert np.array_equal(A.b_full[fi], C.b_full[ci])
    # rows of A and the velocity recovery, from a vector given on the whole crop
    rng = np.random.default_rng(1)
    x = rng.normal(size=A.grid.n_samples())
    ca, fa = sample_map(A.grid, C.grid, lo, 0)
    xc = np.zeros(C.grid.n_samples())
    xc[ca] = x[fa]
    assert np.array_equal(system.apply(A, x)[fi], system.apply(C, xc)[ci])
    uf = system.recover_velocity(A, x * A.active)
    uc = system.recover_velocity(C, xc * C.active)
    assert np.array_equal(uf[ffi], uc[fci])


def test_crop_rejects_out_of_range():
    c = cases.drop32()
    with pytest.raises(ValueError):
        cases.crop(c, (30, 0), (8, 8))
    assert MARGIN >= 2


def test_crop_boxes_stay_inside_the_grid():
    """The sub-box corner of every site used by the full-size checks keeps a
    CROP^3 box inside the grid, also for points at or beyond its faces."""
    from cases.crop_maps import CROP, crop_lo, sites_column, sites_pool
    case = cases.column3d(40, 3)
    n = case["n"]
    for centre in [(0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (0.5, 0.5, 0.5), (-0.2, 1.3, 0.5)]:
        lo = crop_lo(case, centre)
        assert all(0 <= lo[a] <= n[a] - CROP for a in range(3)), (centre, lo)
    mid = crop_lo(case, (0.5, 0.5, 0.5))
    assert all(abs(mid[a] + CROP // 2 - n[a] // 2) <= 1 for a in range(3))
    for label, centre in sites_column(case) + sites_pool(cases.pool3d(40, 5)):
        assert len(centre) == 3, label
        lo = crop_lo(case, centre)
        assert all(0 <= lo[a] <= n[a] - CROP for a in range(3)), label
