"""Pins of the oracle's volume-fraction estimator (paper Section 5, Figs. 3-4).

The estimator must be exact for affine level sets; the reference there is
the closed-form measure of a half-space inside a box (inclusion-exclusion
over the box corners), which shares nothing with the simplex formulas.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import fractions
from oracle.grid import Grid


def halfspace_fraction_box(nrm, t, lo, hi):
    """Fraction of the box [lo, hi] where nrm . x < t (exact, any dimension).

    For positive normal components the measure of {n.x < t} in the unit
    box is sum_v (-1)^{|v|} (t - n.v)_+^d / (d! prod n); negative components
    are handled by reflecting that axis, zero components drop out."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    s = hi - lo
    n = np.asarray(nrm, float) * s          # scale to the unit box
    t = t - float(np.dot(nrm, lo))
    keep = np.abs(n) > 1e-14
    for a in np.flatnonzero(n < 0):          # reflect x_a -> 1 - x_a
        t -= n[a]
        n[a] = -n[a]
    n = n[keep]
    d = len(n)
    if d == 0:
        return 1.0 if t > 0 else 0.0
    tot = 0.0
    for v in itertools.product((0, 1), repeat=d):
        tot += (-1) ** sum(v) * max(t - float(np.dot(n, v)), 0.0) ** d
    return min(max(tot / (math.factorial(d) * float(np.prod(n))), 0.0), 1.0)


def _interior(grid, st):
    """Boolean mask of samples whose control volume lies inside the box."""
    idx = np.indices(grid.shape(st))
    ok = np.ones(grid.shape(st), dtype=bool)
    for a in range(grid.dim):
        if st[a] == 0:
            ok &= (idx[a] > 0) & (idx[a] < grid.n[a])
    return ok


@pytest.mark.parametrize("dim,n,seed", [(2, 7, 0), (2, 9, 1), (3, 5, 2), (3, 4, 3)])
def test_affine_level_set_is_exact(dim, n, seed):
    rng = np.random.default_rng(seed)
    grid = Grid((n,) * dim, 1.0 / n)
    for _ in range(3):
        nrm = rng.normal(size=dim)
        t = float(rng.uniform(0.2, 0.8) * np.abs(nrm).sum())
        X = np.meshgrid(*[np.arange(n + 1) / n] * dim, indexing="ij")
        phi = sum(nrm[a] * X[a] for a in range(dim)) - t
        W = fractions.sample_weights(grid, phi, -phi, w_min=0.0)
        for st, (wl, wf) in W.items():
            C = grid.coords(st)
            mask = _interior(grid, st)
            for ii in zip(*np.nonzero(mask)):
                c = np.array([C[a][ii] for a in range(dim)])
                ex = halfspace_fraction_box(nrm, t, c - 0.5 / n, c + 0.5 / n)
                assert abs(wl[ii] - ex) < 1e-12, (st, ii, wl[ii], ex)
                # solid phi_s = -phi: fluid = where -phi >= 0, i.e. phi <= 0
                is_face = st in grid.faces
                if not (is_face and (ii[grid.faces.index(st)] in (0, grid.n[grid.faces.index(st)]))):
                    assert abs(wf[ii] - ex) < 1e-12


def test_simplex_formulas_brute_force():
    """Closed-form simplex fractions against dense midpoint quadrature of the
    linear interpolant (2D triangle and 3D tetrahedron, all sign cases)."""
    rng = np.random.default_rng(7)
    m = 400
    # reference triangle (0,0),(1,0),(1,1) sampled on a fine grid
    g = (np.arange(m) + 0.5) / m
    X, Y = np.meshgrid(g, g, indexing="ij")
    inside = Y <= X
    for _ in range(30):
        v = rng.normal(size=3)
        phi = v[0] + (v[1] - v[0]) * X + (v[2] - v[1]) * Y
        ref = (inside & (phi < 0)).sum() / inside.sum()
        got = fractions.triangle_fraction(v[None, :])[0]
        assert abs(got - ref) < 1e-2
    m3 = 120
    g = (np.arange(m3) + 0.5) / m3
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    inside = (Z <= Y) & (Y <= X)   # tet 000, 100, 110, 111
    for _ in range(12):
        v = rng.normal(size=4)
        phi = v[0] + (v[1] - v[0]) * X + (v[2] - v[1]) * Y + (v[3] - v[2]) * Z
        ref = (inside & (phi < 0)).sum() / inside.sum()
        got = fractions.tet_fraction(v[None, :])[0]
        assert abs(got - ref) < 2e-2


def test_uniform_sign_and_complement():
    rng = np.random.default_rng(3)
    for dim, n in ((2, 8), (3, 5)):
        grid = Grid((n,) * dim, 1.0 / n)
        shp = (n + 1,) * dim
        Wm = fractions.sample_weights(grid, -np.ones(shp), None, 0.0)
        Wp = fractions.sample_weights(grid, np.ones(shp), None, 0.0)
        for st in Wm:
            assert np.all(Wm[st][0] == 1.0) and np.all(Wp[st][0] == 0.0)
        phi = rng.normal(size=shp)
        phi[np.abs(phi) < 1e-3] = 1e-3     # avoid exact zeros
        W1 = fractions.sample_weights(grid, phi, None, 0.0)
        W2 = fractions.sample_weights(grid, -phi, None, 0.0)
        for st in W1:
            assert np.allclose(W1[st][0] + W2[st][0], 1.0, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_circle_sphere_area_second_order(dim):
    """Sum of cell weights * h^d approaches the disk area / ball volume at
    second order (piecewise-linear interface)."""
    r = 0.31
    exact = math.pi * r * r if dim == 2 else 4.0 / 3.0 * math.pi * r ** 3
    errs = []
    ns = (16, 32, 64) if dim == 2 else (8, 16, 32)
    for n in ns:
        grid = Grid((n,) * dim, 1.0 / n)
        X = np.meshgrid(*[np.arange(n + 1) / n] * dim, indexing="ij")
        phi = np.sqrt(sum((X[a] - 0.5) ** 2 for a in range(dim))) - r
        W = fractions.sample_weights(grid, phi, None, 0.0)
        errs.append(abs(W[grid.cell][0].sum() / n ** dim - exact))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.6), (errs, orders)


def test_monte_carlo_control_volumes():
    """Random control volumes of a curved interface agree with Monte Carlo
    integration of the exact disk to O(h^2)."""
    rng = np.random.default_rng(11)
    n = 16
    h = 1.0 / n
    grid = Grid((n, n), h)
    X = np.meshgrid(*[np.arange(n + 1) * h] * 2, indexing="ij")
    r = 0.33
    phi = np.hypot(X[0] - 0.5, X[1] - 0.5) - r
    W = fractions.sample_weights(grid, phi, None, 0.0)
    wl = W[grid.cell][0]
    C = grid.coords(grid.cell)
    cut = np.argwhere((wl > 0.05) & (wl < 0.95))
    for ii in cut[rng.choice(len(cut), 10, replace=False)]:
        c = np.array([C[0][tuple(ii)], C[1][tuple(ii)]])
        pts = c + (rng.random((200000, 2)) - 0.5) * h
        mc = (np.hypot(pts[:, 0] - 0.5, pts[:, 1] - 0.5) < r).mean()
        assert abs(wl[tuple(ii)] - mc) < 0.02 + 3 * math.sqrt(0.25 / 200000)


def test_snapping_and_box_faces():
    n = 8
    grid = Grid((n, n), 1.0 / n)
    X = np.meshgrid(*[np.arange(n + 1) / n] * 2, indexing="ij")
    phi = X[1] - (3.0005 / n)             # liquid just above a node row
    W = fractions.sample_weights(grid, phi, None, w_min=1e-3)
    for st, (wl, wf) in W.items():
        assert np.all((wl == 0.0) | (wl >= 1e-3))
    for a, fs in enumerate(grid.faces):
        wf = W[fs][1]
        idx = [slice(None)] * 2
        idx[a] = 0
        assert np.all(wf[tuple(idx)] == 0.0)
        idx[a] = -1
        assert np.all(wf[tuple(idx)] == 0.0)
