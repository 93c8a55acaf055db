"""Pins of the oracle's difference operators (paper Section 5).

The reference values are continuous derivatives of closed-form fields, so
a wrong sign, a transposed index or a factor 2 in the stress reduction
fails the second-order truncation checks."""
import numpy as np
import pytest

from oracle import operators
from oracle.grid import Grid


def _faces_eval(grid, fns):
    return np.concatenate([grid.flat(fns[a](*grid.coords(grid.faces[a]))) for a in range(grid.dim)])


def _interior_mask(grid, st, pad=1):
    idx = np.indices(grid.shape(st))
    ok = np.ones(grid.shape(st), dtype=bool)
    for a in range(grid.dim):
        ok &= (idx[a] >= pad) & (idx[a] < grid.shape(st)[a] - pad)
    return grid.flat(ok).astype(bool)


@pytest.mark.parametrize("dim", [2, 3])
def test_rigid_motion_has_no_strain_and_no_divergence(dim):
    n = 6
    grid = Grid((n,) * dim, 1.0 / n)
    rng = np.random.default_rng(dim)
    V = rng.normal(size=dim)
    if dim == 2:
        w = rng.normal()
        fns = [lambda x, y: V[0] - w * y + 0 * x, lambda x, y: V[1] + w * x + 0 * y]
    else:
        W = rng.normal(size=3)
        fns = [lambda x, y, z: V[0] + W[1] * z - W[2] * y,
               lambda x, y, z: V[1] + W[2] * x - W[0] * z,
               lambda x, y, z: V[2] + W[0] * y - W[1] * x]
    u = _faces_eval(grid, fns)
    Bt = operators.b0(grid).T.tocsr()
    res = Bt @ u
    off = 0
    for name, st in grid.samples:
        m = _interior_mask(grid, st)
        blk = res[off:off + grid.size(st)]
        assert np.abs(blk[m]).max() < 1e-12, name
        off += grid.size(st)


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_of_affine_pressure_is_exact(dim):
    n = 5
    grid = Grid((n,) * dim, 1.0 / n)
    c = np.arange(1, dim + 1) * 0.7
    X = grid.coords(grid.cell)
    p = grid.flat(sum(c[a] * X[a] for a in range(dim)) + 0.3)
    Gp = operators.gradient(grid) @ p
    for a, (lo, hi) in enumerate(grid.face_offsets()):
        fs = grid.faces[a]
        idx = np.indices(grid.shape(fs))[a]
        inner = grid.flat((idx > 0) & (idx < n)).astype(bool)
        assert np.allclose(Gp[lo:hi][inner], c[a], atol=1e-12)


def _stress_2d():
    p = lambda x, y: np.sin(2 * x) * np.cos(3 * y)
    txx = lambda x, y: np.cos(x + 2 * y)
    txy = lambda x, y: np.sin(2 * x - y)
    # grad p - div tau with tau_yy = -tau_xx
    fx = lambda x, y: 2 * np.cos(2 * x) * np.cos(3 * y) - (-np.sin(x + 2 * y) - np.cos(2 * x - y))
    fy = lambda x, y: -3 * np.sin(2 * x) * np.sin(3 * y) - (2 * np.cos(2 * x - y) + 2 * np.sin(x + 2 * y))
    return dict(p=p, txx=txx, txy=txy), [fx, fy]


def _stress_3d():
    p = lambda x, y, z: np.sin(x + y) * np.cos(z)
    txx = lambda x, y, z: np.cos(x + 2 * y - z)
    tyy = lambda x, y, z: np.sin(x - y + 2 * z)
    txy = lambda x, y, z: np.cos(2 * x + z)
    txz = lambda x, y, z: np.sin(y + 2 * z)
    tyz = lambda x, y, z: np.cos(x - 2 * y)
    # div tau with tau_zz = -(tau_xx + tau_yy)
    dx_txx = lambda x, y, z: -np.sin(x + 2 * y - z)
    dz_txx = lambda x, y, z: np.sin(x + 2 * y - z)
    dy_tyy = lambda x, y, z: -np.cos(x - y + 2 * z)
    dz_tyy = lambda x, y, z: 2 * np.cos(x - y + 2 * z)
    dy_txy = lambda x, y, z: 0 * x
    dx_txy = lambda x, y, z: -2 * np.sin(2 * x + z)
    dz_txz = lambda x, y, z: 2 * np.cos(y + 2 * z)
    dx_txz = lambda x, y, z: 0 * x
    dz_tyz = lambda x, y, z: 0 * x
    dy_tyz = lambda x, y, z: 2 * np.sin(x - 2 * y)
    fx = lambda x, y, z: np.cos(x + y) * np.cos(z) - (dx_txx(x, y, z) + dy_txy(x, y, z) + dz_txz(x, y, z))
    fy = lambda x, y, z: np.cos(x + y) * np.cos(z) - (dx_txy(x, y, z) + dy_tyy(x, y, z) + dz_tyz(x, y, z))
    fz = lambda x, y, z: -np.sin(x + y) * np.sin(z) - (dx_txz(x, y, z) + dy_tyz(x, y, z)
                                                      - dz_txx(x, y, z) - dz_tyy(x, y, z))
    return dict(p=p, txx=txx, tyy=tyy, txy=txy, txz=txz, tyz=tyz), [fx, fy, fz]


@pytest.mark.parametrize("dim", [2, 3])
def test_momentum_truncation_second_order(dim):
    """(G p + D^T tau) at interior faces equals grad p - div tau + O(h^2):
    the discrete form of the momentum balance of Section 4."""
    fields, force = _stress_2d() if dim == 2 else _stress_3d()
    errs = []
    for n in ((16, 32, 64) if dim == 2 else (8, 16, 32)):
        grid = Grid((n,) * dim, 1.0 / n)
        x = np.concatenate([grid.flat(fields[name](*grid.coords(st))) for name, st in grid.samples])
        got = operators.b0(grid) @ x
        ex = _faces_eval(grid, force)
        m = np.concatenate([_interior_mask(grid, fs, 2) for fs in grid.faces])
        errs.append(np.abs(got - ex)[m].max())
    ratio = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratio > 3.3), errs


@pytest.mark.parametrize("dim", [2, 3])
def test_strain_truncation_second_order(dim):
    """D u at interior samples equals the kept strain-rate combinations
    (u_x - v_y, u_y + v_x in 2D; u_x - w_z, v_y - w_z, u_y + v_x, u_z + w_x,
    v_z + w_y in 3D) + O(h^2)."""
    if dim == 2:
        U = [lambda x, y: np.sin(x) * np.cos(2 * y), lambda x, y: np.cos(3 * x + y)]
        ex = {"txx": lambda x, y: np.cos(x) * np.cos(2 * y) + np.sin(3 * x + y),
              "txy": lambda x, y: -2 * np.sin(x) * np.sin(2 * y) - 3 * np.sin(3 * x + y)}
    else:
        U = [lambda x, y, z: np.sin(x + z) * np.cos(y),
             lambda x, y, z: np.cos(x - y) * np.sin(z),
             lambda x, y, z: np.sin(2 * x + y - z)]
        ux = lambda x, y, z: np.cos(x + z) * np.cos(y)
        uy = lambda x, y, z: -np.sin(x + z) * np.sin(y)
        uz = lambda x, y, z: np.cos(x + z) * np.cos(y)
        vx = lambda x, y, z: -np.sin(x - y) * np.sin(z)
        vy = lambda x, y, z: np.sin(x - y) * np.sin(z)
        vz = lambda x, y, z: np.cos(x - y) * np.cos(z)
        wx = lambda x, y, z: 2 * np.cos(2 * x + y - z)
        wy = lambda x, y, z: np.cos(2 * x + y - z)
        wz = lambda x, y, z: -np.cos(2 * x + y - z)
        ex = {"txx": lambda *X: ux(*X) - wz(*X), "tyy": lambda *X: vy(*X) - wz(*X),
              "txy": lambda *X: uy(*X) + vx(*X), "txz": lambda *X: uz(*X) + wx(*X),
              "tyz": lambda *X: vz(*X) + wy(*X)}
    errs = []
    for n in ((16, 32, 64) if dim == 2 else (8, 16, 32)):
        grid = Grid((n,) * dim, 1.0 / n)
        Du = operators.deformation(grid) @ _faces_eval(grid, U)
        off = 0
        e = 0.0
        for name, st in grid.samples:
            if name == "p":
                continue
            blk = Du[off:off + grid.size(st)]
            m = _interior_mask(grid, st)
            e = max(e, np.abs(blk - grid.flat(ex[name](*grid.coords(st))))[m].max())
            off += grid.size(st)
        errs.append(e)
    ratio = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratio > 3.3), errs


def test_gradient_is_minus_divergence_adjoint():
    """<G p, u> = -<p, div u> summed over the box with u = 0 on box faces."""
    grid = Grid((7, 5), 0.1)
    rng = np.random.default_rng(0)
    p = rng.normal(size=grid.size(grid.cell))
    u = rng.normal(size=grid.n_faces())
    div = np.zeros(grid.size(grid.cell))
    uu = [grid.unflat(u[lo:hi], grid.faces[a]) for a, (lo, hi) in enumerate(grid.face_offsets())]
    uu[0][0, :] = uu[0][-1, :] = 0.0
    uu[1][:, 0] = uu[1][:, -1] = 0.0
    d2 = (uu[0][1:, :] - uu[0][:-1, :]) / grid.h + (uu[1][:, 1:] - uu[1][:, :-1]) / grid.h
    u0 = np.concatenate([grid.flat(q) for q in uu])
    div = grid.flat(d2)
    assert abs((operators.gradient(grid) @ p) @ u0 + p @ div) < 1e-10
