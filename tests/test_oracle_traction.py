"""Pins of the oracle's prescribed-traction free surface (Section 6.1).

  * A uniform prescribed pressure p0 leaves the flow unchanged and shifts
    every active pressure by exactly p0 (2D and 3D, with gravity, a solid and
    a moving solid): the boundary work of a constant pressure is a constant
    shift, and the eliminated pressures take the boundary value (Section 8).
  * The Schur form with the traction terms folded into u* equals the full
    (u, tau, p) KKT solve with the terms written on the velocity rows as
    the air-region integral gives them (2D and 3D, random smooth p_BC and
    tau_BC, moving solid): this checks the elimination algebra, including
    the compliance coupling of a fixed tau_yy in 3D.
  * Convergence: a drop whose exact solution (tests/manufactured.py fields)
    has a non-zero surface traction, prescribed as (p_BC, tau_BC) = the
    exact (p, tau), converges at first order in velocity; without the
    traction terms, or with the opposite sign, it does not converge.
"""
import numpy as np
import pytest

import cases
import manufactured
from oracle import system
from test_oracle_system import _box_case, _moving_solid_case


def _with_traction(case, p_bc=None, tau_bc=None):
    c = dict(case)
    c["p_bc"] = p_bc
    c["tau_bc"] = tau_bc
    return c


@pytest.mark.parametrize("dim,n", [(2, 20), (3, 9)])
def test_uniform_pressure_shifts_pressure_only(dim, n):
    rng = np.random.default_rng(40 + dim)
    phi_l, phi_s, ubc, _ = _moving_solid_case(dim, n, rng)
    g = [0.0] * dim
    g[1] = -9.8
    base = _box_case(dim, n, phi_l, phi_s, rng, ubc=ubc, g=tuple(g))
    asm0, x0, u0 = system.step(base)
    assert not system.is_enclosed(asm0)
    p0 = 3.7
    asm1, x1, u1 = system.step(_with_traction(base, p_bc=np.full((n,) * dim, p0)))
    m = asm0.K > 0
    assert np.array_equal(asm0.active, asm1.active)
    scale = max(np.abs(u0[m]).max(), 1.0)
    assert np.abs(u1[m] - u0[m]).max() <= 1e-10 * scale
    lo, hi = asm0.grid.sample_offsets()["p"]
    shift = np.zeros_like(x0)
    shift[lo:hi] = p0
    shift *= asm0.active
    assert np.abs(x1 - (x0 + shift)).max() <= 1e-10 * (np.abs(x0).max() + p0)


def _smooth_bc(grid, rng):
    """Random smooth (p_BC, tau_BC) fields at their native sample locations."""
    out = {}
    for name, st in grid.samples:
        X = grid.coords(st)
        k = rng.normal(size=grid.dim) * 3.0
        ph = rng.uniform(0, 2 * np.pi)
        out[name] = rng.uniform(0.5, 2.0) * np.cos(sum(k[a] * X[a] for a in range(grid.dim)) + ph)
    p = out.pop("p")
    return p, [out[name] for name, _ in grid.samples if name != "p"]


@pytest.mark.parametrize("dim,n", [(2, 8), (2, 11), (3, 5)])
def test_traction_kkt_equals_schur(dim, n):
    rng = np.random.default_rng(60 + n)
    phi_l, phi_s, ubc, _ = _moving_solid_case(dim, n, rng)
    ubc = [q + rng.normal(0, 0.2, size=q.shape) for q in ubc]
    c = _box_case(dim, n, phi_l, phi_s, rng, ubc=ubc, g=tuple(rng.normal(size=dim)))
    from oracle.grid import Grid
    p_bc, tau_bc = _smooth_bc(Grid(c["n"], c["h"]), rng)
    ct = _with_traction(c, p_bc, tau_bc)
    asm, x, u = system.step(ct)
    M, rhs, fidx, sidx = system.kkt_dense(asm)
    sol = np.linalg.solve(M, rhs)
    nf = len(fidx)
    assert np.abs(sol[:nf] - u[fidx]).max() <= 1e-9 * max(1.0, np.abs(u).max())
    assert np.abs(sol[nf:] - x[sidx]).max() <= 1e-9 * max(1.0, np.abs(x).max())
    # the traction terms are live in this case
    asm0, x_0, u_0 = system.step(c)
    assert np.abs(u_0 - u)[asm.K > 0].max() > 1e-3


def test_traction_kkt_covers_a_fixed_tau_yy():
    """3D cases where a cell's tau_xx is active and its tau_yy eliminated (or
    the reverse) exist, so the coupling term of the fixed stress is tested."""
    found = 0
    for n in (5, 6, 7):
        rng = np.random.default_rng(60 + n)
        phi_l, phi_s, ubc, _ = _moving_solid_case(3, n, rng)
        c = _box_case(3, n, phi_l, phi_s, rng, ubc=ubc)
        asm = system.assemble(c)
        off = asm.grid.sample_offsets()
        ax = asm.active[off["txx"][0]:off["txx"][1]]
        ay = asm.active[off["tyy"][0]:off["tyy"][1]]
        wl = asm.wl_s[off["txx"][0]:off["txx"][1]]
        found += int(((ax != ay) & (wl > 0)).sum())
    assert found > 0


def _drop_errors(n, mode):
    """Velocity errors of one step of the drop r < 0.35 around (0.5, 0.5)
    whose exact fields are the manufactured 2D solution."""
    f = manufactured.functions(2)
    case = manufactured.make_case(2, n)
    h = 1.0 / n
    X, Y = cases.node_coords((n, n), h, (0.0, 0.0))
    case["phi_l"] = np.hypot(X - 0.5, Y - 0.5) - 0.35
    grid_c = cases.cell_coords((n, n), h, (0.0, 0.0))
    grid_n = cases.node_coords((n, n), h, (0.0, 0.0))
    p_bc = manufactured._ev(f["p"], grid_c)
    txx = manufactured._ev(f["tau00"], grid_c)
    txy = manufactured._ev(f["tau01"], grid_n)
    if mode == "prescribed":
        case = _with_traction(case, p_bc, [txx, txy])
    elif mode == "flipped":
        case = _with_traction(case, -p_bc, [-txx, -txy])
    asm, x, u = system.step(case)
    ue = np.concatenate([asm.grid.flat(q) for q in manufactured.exact_velocity(2, n)])
    m = asm.K > 0
    e = np.abs(u[m] - ue[m])
    return e.max(), e.sum() * h * h


def test_prescribed_traction_convergence():
    ns = (32, 64, 128)
    logh = -np.log(np.array(ns, dtype=np.float64))
    res = {mode: np.array([_drop_errors(n, mode) for n in ns])
           for mode in ("prescribed", "none", "flipped")}
    for col in (0, 1):
        order = np.polyfit(logh, np.log(res["prescribed"][:, col]), 1)[0]
        assert order >= 0.8, (col, res["prescribed"][:, col], order)
    # without the terms, or with the other sign, the surface condition is wrong
    # and the error stays at O(1) of the traction
    for mode in ("none", "flipped"):
        assert res[mode][-1, 1] > 10 * res["prescribed"][-1, 1], (mode, res[mode], res["prescribed"])
