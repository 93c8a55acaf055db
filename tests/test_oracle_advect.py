"""Pins of the oracle's advection half of the fractional step (Section 10):
semi-Lagrangian advection of velocity and level set, the velocity extension
into the air, and the composition of steps.

  * a uniform velocity is left unchanged and translates the level set
    exactly by whole cells (dt V = integer multiples of h);
  * multilinear interpolation reproduces affine fields, so an affine
    velocity is advected to its closed form u(x - dt u(x)) wherever the
    departure point lies inside the sample lattice, and an affine level set
    to phi(x - dt v(x)) for any velocity;
  * the extension keeps known values, fills `layers` layers (a constant
    stays constant) and nothing beyond them;
  * a run of two steps equals two single steps fed each other's output.
"""
import numpy as np
import pytest

import cases
from oracle import advect, system
from oracle.grid import Grid


def _faces(grid, fns):
    return [fns[a](*grid.coords(grid.faces[a])) * np.ones(grid.shape(grid.faces[a]))
            for a in range(grid.dim)]


@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_velocity_is_kept_and_translates_exactly(dim):
    n = 12
    grid = Grid((n,) * dim, 1.0 / n)
    V = np.array([2.0, -1.0, 1.0][:dim]) / n / 0.5    # dt V = (2, -1, 1) h at dt = 0.5
    u = [np.full(grid.shape(grid.faces[a]), V[a]) for a in range(dim)]
    dt = 0.5
    ua = advect.advect_velocity(grid, u, dt)
    for a in range(dim):
        assert np.abs(ua[a] - V[a]).max() < 1e-14
    rng = np.random.default_rng(dim)
    phi = rng.normal(size=(n + 1,) * dim)
    new = advect.advect_level_set(grid, phi, u, dt)
    shift = np.rint(dt * V * n).astype(int)
    idx = np.indices(phi.shape)
    src = [idx[b] - shift[b] for b in range(dim)]
    inside = np.all([(src[b] >= 0) & (src[b] <= n) for b in range(dim)], axis=0)
    want = phi[tuple(np.clip(src[b], 0, n) for b in range(dim))]
    assert inside.sum() > 0.5 * inside.size
    assert np.abs(new[inside] - want[inside]).max() < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_affine_fields_are_advected_exactly(dim):
    n = 10
    grid = Grid((n,) * dim, 1.0 / n)
    rng = np.random.default_rng(5 + dim)
    c = rng.normal(size=dim) * 0.3
    A = rng.normal(size=(dim, dim)) * 0.4
    vel = lambda a: (lambda *X: c[a] + sum(A[a, b] * X[b] for b in range(dim)))
    u = _faces(grid, [vel(a) for a in range(dim)])
    dt = 0.3
    ua = advect.advect_velocity(grid, u, dt)
    for a in range(dim):
        X = grid.coords(grid.faces[a])
        v = [vel(b)(*X) for b in range(dim)]
        dep = [X[b] - dt * v[b] for b in range(dim)]
        want = vel(a)(*dep)
        # departure points whose interpolation stencil lies inside every
        # component's sample lattice (no clamping)
        ok = np.ones(X[0].shape, dtype=bool)
        for b in range(dim):
            for st in grid.faces + [(0,) * dim]:
                xi = dep[b] / grid.h - 0.5 * st[b]
                ok &= (xi >= 0) & (xi <= grid.shape(st)[b] - 1)
                xo = X[b] / grid.h - 0.5 * st[b]
                ok &= (xo >= 0) & (xo <= grid.shape(st)[b] - 1)
        assert ok.sum() > 0.2 * ok.size
        assert np.abs(ua[a][ok] - want[ok]).max() < 1e-12
    # an affine level set under the same (affine) velocity
    k = rng.normal(size=dim)
    X = grid.coords((0,) * dim)
    phi = 0.2 + sum(k[b] * X[b] for b in range(dim))
    new = advect.advect_level_set(grid, phi, u, dt)
    v = [vel(b)(*X) for b in range(dim)]
    dep = [X[b] - dt * v[b] for b in range(dim)]
    inside = np.all([(dep[b] >= 0) & (dep[b] <= 1.0) for b in range(dim)], axis=0)
    for b in range(dim):
        for st in grid.faces:
            xo = X[b] / grid.h - 0.5 * st[b]
            inside &= (xo >= 0) & (xo <= grid.shape(st)[b] - 1)
    want = 0.2 + sum(k[b] * dep[b] for b in range(dim))
    assert np.abs(new[inside] - want[inside]).max() < 1e-12


def test_extension_fills_layers_and_keeps_known_values():
    n = 16
    grid = Grid((n, n), 1.0 / n)
    rng = np.random.default_rng(3)
    u = [rng.normal(size=grid.shape(f)) for f in grid.faces]
    known = []
    for a, f in enumerate(grid.faces):
        X = grid.coords(f)
        known.append(X[0] < 0.3)
    const = [np.where(k, 1.75, q) for k, q in zip(known, u)]
    ext = advect.extend_velocity(grid, const, known, layers=3)
    for a in range(2):
        X = grid.coords(grid.faces[a])
        assert np.array_equal(ext[a][known[a]], const[a][known[a]])
        # within three index steps of the known region: filled with the constant
        i = np.indices(X[0].shape)[0]
        first_unknown = np.min(np.where(known[a], 10 ** 6, i))
        band = (~known[a]) & (i < first_unknown + 3)
        assert np.abs(ext[a][band] - 1.75).max() < 1e-15
        # beyond the three layers the faces keep their input values
        far = i >= first_unknown + 3
        assert far.any() and np.array_equal(ext[a][far], const[a][far])
    # the mean of known neighbours: a face with two known neighbours of
    # different values takes their mean
    v = [np.zeros(grid.shape(f)) for f in grid.faces]
    k = [np.zeros(grid.shape(f), dtype=bool) for f in grid.faces]
    v[0][4, 5], v[0][6, 5] = 1.0, 3.0
    k[0][4, 5] = k[0][6, 5] = True
    e = advect.extend_velocity(grid, v, k, layers=1)
    assert e[0][5, 5] == 2.0 and e[0][4, 6] == 1.0 and e[0][7, 5] == 3.0
    assert e[0][8, 5] == 0.0


def test_two_steps_equal_two_single_steps():
    c = cases.drop2d(24, 3, dt=0.01)
    c["g"] = (0.0, -1.0)
    end, hist = advect.ns_run(c, 0.01, 2)
    c1, r1 = advect.ns_step(c, 0.01)
    c2, r2 = advect.ns_step(c1, 0.01, r1[0])
    for a in range(2):
        assert np.array_equal(end["u"][a], c2["u"][a])
    assert np.array_equal(end["phi_l"], c2["phi_l"])
    assert np.array_equal(hist[1][1], r2[1])
    # the liquid moves: the level set changed and the drop fell
    assert np.abs(end["phi_l"] - c["phi_l"]).max() > 1e-4
