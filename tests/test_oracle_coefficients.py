"""Pins of the oracle's compliance block and coefficient averaging.

  * Compliance (Section 5's local stress relations with the trace-free
    reduction): for a smooth divergence-free velocity and tau = mu (grad u +
    grad u^T) sampled at the stress samples, C tau equals the reduced strain
    rates D u at every interior sample up to the O(h^2) truncation of D.  In
    3D this needs the (1/mu)[[1, 1/2], [1/2, 1]] coupling of each cell's
    (tau_xx, tau_yy): tau_xx + tau_yy/2 = mu (u_x - w_z) and
    tau_yy + tau_xx/2 = mu (v_y - w_z) once tau_zz = -tau_xx - tau_yy.
  * Coefficient averaging (P per velocity sample and M per stress sample,
    Section 5, from cell-centred rho and mu): the mean over the in-box cells
    adjacent to a sample reproduces an affine field exactly at the centroid
    of those cells -- the sample itself in the interior, the point half a
    cell inside the box for samples on a wall -- and a 2x2 example is worked
    by hand.
  * Convergence of whole steps on manufactured box solutions with smooth
    variable density and viscosity (tests/manufactured.py), 2D and 3D: the
    velocity error falls at least at first order (second order is observed:
    no irregular boundary is present).
"""
import numpy as np
import pytest

import manufactured
from oracle import operators, system
from oracle.grid import Grid


def _eval(fn, coords):
    return np.asarray(fn(*coords), dtype=np.float64) * np.ones_like(coords[0])


def _interior(grid, st, pad=1):
    idx = np.indices(grid.shape(st))
    ok = np.ones(grid.shape(st), dtype=bool)
    for a in range(grid.dim):
        ok &= (idx[a] >= pad) & (idx[a] < grid.shape(st)[a] - pad)
    return grid.flat(ok).astype(bool)


# tensor component of each kept stress
_COMPONENT = {"txx": (0, 0), "tyy": (1, 1), "txy": (0, 1), "txz": (0, 2), "tyz": (1, 2)}


def _compliance_mismatch(dim, n):
    """max over interior stress samples of |C tau - D u| / max|D u|."""
    f = manufactured.functions(dim)
    grid = Grid((n,) * dim, 1.0 / n)
    u = np.concatenate([grid.flat(_eval(f[f"u{a}"], grid.coords(grid.faces[a])))
                        for a in range(dim)])
    tau = []
    mu_s = []
    for name, st in grid.samples:
        X = grid.coords(st)
        if name == "p":
            tau.append(np.zeros(grid.size(st)))
            mu_s.append(np.full(grid.size(st), np.nan))
            continue
        i, j = _COMPONENT[name]
        tau.append(grid.flat(_eval(f[f"tau{i}{j}"], X)))
        mu_s.append(grid.flat(_eval(f["mu"], X)))
    tau = np.concatenate(tau)
    mu_s = np.concatenate(mu_s)
    ns = grid.n_samples()
    ones = np.ones(ns)
    Dg = system.compliance(grid, ones, ones, mu_s, np.ones(ns, dtype=bool))
    lhs = Dg @ tau
    Du = operators.deformation(grid) @ u
    p_lo, p_hi = grid.sample_offsets()["p"]
    lhs = lhs[p_hi:]
    worst = 0.0
    off = 0
    for name, st in grid.samples:
        if name == "p":
            continue
        m = _interior(grid, st)
        sz = grid.size(st)
        blk = slice(off, off + sz)
        worst = max(worst, float(np.abs(lhs[blk][m] - Du[blk][m]).max()))
        off += sz
    return worst / float(np.abs(Du).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_compliance_reproduces_local_stress_relations(dim):
    e8 = _compliance_mismatch(dim, 8)
    e16 = _compliance_mismatch(dim, 16)
    # C tau = D u holds exactly in the continuum; the remainder is the
    # second-order truncation of the centred differences in D u
    assert e16 < 2e-2, (e8, e16)
    assert e8 / e16 > 3.0, (e8, e16)


def _centroid_axis(n, h, stagger, shape_len):
    """Per axis: the centroid coordinate of the in-box cells adjacent to each
    sample index of a sample type (cell-centred axis: the sample's cell;
    grid-line axis: cells i-1 and i where they exist)."""
    i = np.arange(shape_len, dtype=np.float64)
    if stagger == 1:
        return (i + 0.5) * h
    lo = np.maximum(i - 1, 0)
    hi = np.minimum(i, n - 1)
    return 0.5 * ((lo + 0.5) + (hi + 0.5)) * h


@pytest.mark.parametrize("dim", [2, 3])
def test_cell_mean_is_exact_for_affine_fields(dim):
    n = 5
    h = 1.0 / n
    grid = Grid((n,) * dim, h)
    c = np.array([0.7, -1.3, 2.1])[:dim]
    X = grid.coords(grid.cell)
    mu = 3.0 + sum(c[a] * X[a] for a in range(dim))
    staggers = [grid.cell] + list(grid.faces) + [st for name, st in grid.samples if name != "p"]
    for st in staggers:
        shp = grid.shape(st)
        axes = [_centroid_axis(n, h, st[a], shp[a]) for a in range(dim)]
        C = np.meshgrid(*axes, indexing="ij")
        want = 3.0 + sum(c[a] * C[a] for a in range(dim))
        got = system.cell_mean_at(grid, mu, st)
        assert np.abs(got - want).max() < 1e-13, st


def test_cell_mean_worked_example_2d():
    grid = Grid((2, 2), 0.5)
    mu = np.array([[1.0, 2.0], [3.0, 4.0]])    # mu[i, j], i along x
    node = system.cell_mean_at(grid, mu, (0, 0))
    assert node.shape == (3, 3)
    # corner nodes see one cell, wall midpoints two, the centre node four
    assert node[0, 0] == 1.0 and node[2, 2] == 4.0 and node[2, 0] == 3.0
    assert node[1, 0] == 2.0          # cells (0,0), (1,0): (1 + 3) / 2
    assert node[0, 1] == 1.5          # cells (0,0), (0,1): (1 + 2) / 2
    assert node[1, 1] == 2.5          # all four
    uface = system.cell_mean_at(grid, mu, (0, 1))
    assert uface.shape == (3, 2)
    assert uface[1, 0] == 2.0 and uface[1, 1] == 3.0 and uface[0, 1] == 2.0
    vface = system.cell_mean_at(grid, mu, (1, 0))
    assert vface[0, 1] == 1.5 and vface[1, 1] == 3.5 and vface[1, 2] == 4.0


def _velocity_errors(dim, n):
    case = manufactured.make_case(dim, n)
    asm, x, u = system.step(case)
    ue = np.concatenate([asm.grid.flat(q) for q in manufactured.exact_velocity(dim, n)])
    m = asm.K > 0
    e = np.abs(u[m] - ue[m])
    return e.max(), e.sum() * asm.grid.h ** dim


@pytest.mark.parametrize("dim,ns", [(2, (16, 32, 64)), (3, (8, 12, 16))])
def test_manufactured_variable_coefficient_convergence(dim, ns):
    errs = np.array([_velocity_errors(dim, n) for n in ns])
    logh = -np.log(np.array(ns, dtype=np.float64))
    for col, what in ((0, "Linf"), (1, "L1")):
        order = np.polyfit(logh, np.log(errs[:, col]), 1)[0]
        assert order >= 0.9, (what, errs[:, col], order)
    # the finest grid is close: a consistent discretisation, not just a trend
    assert errs[-1, 0] < 0.05 * 3.0, errs


def test_manufactured_fields_are_consistent():
    """The manufactured velocity is divergence free and vanishes on the
    walls (so the box's no-slip walls hold exactly)."""
    for dim in (2, 3):
        f = manufactured.functions(dim)
        rng = np.random.default_rng(dim)
        P = [rng.uniform(0, 1, 50) for _ in range(dim)]
        assert np.abs(_eval(f["div"], P)).max() < 1e-12
        for a in range(dim):
            W = [q.copy() for q in P]
            W[a][:] = 0.0
            for b in range(dim):
                assert np.abs(_eval(f[f"u{b}"], W)).max() < 1e-12
