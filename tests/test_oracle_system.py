"""Pins of the oracle's SPD system, solve and velocity recovery.

  * symmetry and positive definiteness by brute force on tiny random
    geometries (eq. stokesmixedsystemspd, null-space elimination of
    Section 8);
  * agreement with a dense solve at 8x8;
  * equivalence of the Schur form with the full (u, tau, p) KKT system
    (eq. stokesmixedsystem; Section 6.2 right-hand side for moving solids);
  * minimum dissipation: the recovered velocity is the constrained
    minimiser of the primal functional (Section 7);
  * exact states claimed in Section 9: hydrostatic rest, rigid translation
    and rotation of a free-surface body, and co-motion with a moving solid;
  * first-order velocity convergence on the four closed-form 2D cases.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import analytic
import cases
from oracle import cg, system
from oracle.grid import Grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_velocity_errors.json")


def _box_case(dim, n, phi_l, phi_s, rng, dt=0.1, ubc=None, g=None, u=None, mu=None, rho=None):
    h = 1.0 / n
    nn = (n,) * dim
    if u is None:
        u = [rng.normal(0.0, 0.3, size=s) for s in cases.face_shapes(nn)]
    return dict(dim=dim, n=nn, h=h, origin=(0.0,) * dim, dt=dt, phi_l=phi_l, phi_s=phi_s,
                rho=rho if rho is not None else rng.uniform(0.5, 2.0, size=nn),
                mu=mu if mu is not None else rng.uniform(0.2, 3.0, size=nn),
                u=u, u_bc=ubc, g=g if g is not None else (0.0,) * dim)


def _random_geometry(dim, n, rng, solid=True):
    X = cases.node_coords((n,) * dim, 1.0 / n, (0.0,) * dim)
    c = rng.uniform(0.3, 0.7, size=dim)
    r = rng.uniform(0.25, 0.45)
    phi_l = np.sqrt(sum((X[a] - c[a]) ** 2 for a in range(dim))) - r
    phi_l = phi_l + rng.normal(0.0, 0.5 / n, size=phi_l.shape)
    phi_s = None
    if solid:
        cs = rng.uniform(0.2, 0.8, size=dim)
        phi_s = np.sqrt(sum((X[a] - cs[a]) ** 2 for a in range(dim))) - rng.uniform(0.1, 0.25)
        phi_s = np.minimum(phi_s, X[1] - rng.uniform(0.05, 0.3))
    return phi_l, phi_s


@pytest.mark.parametrize("dim,n,seed", [(2, 4, 0), (2, 6, 1), (2, 8, 2), (2, 8, 3), (2, 7, 4),
                                        (3, 3, 5), (3, 4, 6), (3, 4, 7)])
def test_spd_bruteforce(dim, n, seed):
    rng = np.random.default_rng(seed)
    phi_l, phi_s = _random_geometry(dim, n, rng, solid=seed % 2 == 0)
    asm = system.assemble(_box_case(dim, n, phi_l, phi_s, rng))
    A = asm.A.toarray()
    if A.shape[0] == 0:
        pytest.skip("no active samples for this geometry")
    scale = np.abs(A).max()
    assert np.abs(A - A.T).max() <= 1e-14 * scale
    ev = np.linalg.eigvalsh(A)
    null = int((ev < 1e-11 * ev[-1]).sum())
    assert null == (1 if system.is_enclosed(asm) else 0), ev[:4]
    assert ev[null] > 0.0


@pytest.mark.parametrize("seed", [0, 1])
def test_spd_enclosed_has_exactly_the_pressure_constant(seed):
    """A liquid-filled box with an inner solid: pressure is defined up to a
    constant (Section 8, last paragraph) and nothing else is singular."""
    rng = np.random.default_rng(seed)
    n = 8
    X = cases.node_coords((n, n), 1.0 / n, (0.0, 0.0))
    phi_s = np.hypot(X[0] - 0.5, X[1] - 0.45) - 0.2
    asm = system.assemble(_box_case(2, n, -np.ones((n + 1, n + 1)), phi_s, rng))
    assert system.is_enclosed(asm)
    ev = np.linalg.eigvalsh(asm.A.toarray())
    assert ev[0] < 1e-11 * ev[-1] < ev[1]


def test_dense_solve_agreement_8x8():
    rng = np.random.default_rng(42)
    c = cases.drop2d(8, seed=3, radius=0.3)
    asm, x, u = system.step(c)
    xd = np.linalg.solve(asm.A.toarray(), asm.b)
    assert np.abs(x[asm.act_idx] - xd).max() <= 1e-12 * max(1.0, np.abs(xd).max())
    xc, it, _ = cg.jacobi_pcg(asm.A, asm.b, tol=1e-14)
    assert np.abs(xc - xd).max() <= 1e-10 * np.abs(xd).max()


def _moving_solid_case(dim, n, rng):
    X = cases.node_coords((n,) * dim, 1.0 / n, (0.0,) * dim)
    cl = np.full(dim, 0.5)
    phi_l = np.sqrt(sum((X[a] - cl[a]) ** 2 for a in range(dim))) - 0.36
    phi_s = np.sqrt(sum((X[a] - 0.47) ** 2 for a in range(dim))) - 0.14
    V = rng.uniform(-1, 1, size=dim)
    ubc = [np.full(s, V[a]) for a, s in enumerate(cases.face_shapes((n,) * dim))]
    return phi_l, phi_s, ubc, V


@pytest.mark.parametrize("dim,n", [(2, 8), (2, 10), (3, 5)])
def test_kkt_equals_schur(dim, n):
    rng = np.random.default_rng(n)
    phi_l, phi_s, ubc, _ = _moving_solid_case(dim, n, rng)
    # non-rigid prescribed velocity so every right-hand-side term is live
    ubc = [q + rng.normal(0, 0.2, size=q.shape) for q in ubc]
    c = _box_case(dim, n, phi_l, phi_s, rng, ubc=ubc, g=tuple(rng.normal(size=dim)))
    asm, x, u = system.step(c)
    M, rhs, fidx, sidx = system.kkt_dense(asm)
    sol = np.linalg.solve(M, rhs)
    nf = len(fidx)
    assert np.abs(sol[:nf] - u[fidx]).max() <= 1e-9 * max(1.0, np.abs(u).max())
    assert np.abs(sol[nf:] - x[sidx]).max() <= 1e-9 * max(1.0, np.abs(x).max())


def test_minimum_dissipation():
    """The recovered u minimises 1/2 (u-u*)^T M (u-u*) + 1/2 s_t^T Dg^-1 s_t
    subject to s_p = 0, where s = B^T W_F u + c (the primal form of the
    saddle point): the gradient is orthogonal to the feasible directions."""
    rng = np.random.default_rng(5)
    n = 8
    phi_l, phi_s, ubc, _ = _moving_solid_case(2, n, rng)
    ubc = [q + rng.normal(0, 0.2, size=q.shape) for q in ubc]
    c = _box_case(2, n, phi_l, phi_s, rng, ubc=ubc)
    asm, x, u = system.step(c)
    fidx = np.flatnonzero(asm.K > 0)
    sidx = asm.act_idx
    grid = asm.grid
    Bw = (asm.B.toarray() * asm.wf_f[:, None])[np.ix_(fidx, sidx)]
    a = asm.wl_s * asm.active
    corr = a * (asm.B0.T @ ((1 - asm.wf_f) * asm.u_bc) - (1 - asm.wf_s) * (asm.B0.T @ asm.u_bc))
    cvec = corr[sidx]
    lo, hi = grid.sample_offsets()["p"]
    is_p = (sidx >= lo) & (sidx < hi)
    Dg = asm.Dg.toarray()[np.ix_(sidx[~is_p], sidx[~is_p])]
    Dinv = np.linalg.inv(Dg)
    us = np.concatenate([grid.flat(q) for q in asm.u_star])[fidx]
    M = asm.rho_f[fidx] * asm.wf_f[fidx] * asm.wl_f[fidx] / asm.dt
    uf = u[fidx]
    s = Bw.T @ uf + cvec
    assert np.abs(s[is_p]).max() < 1e-10 * max(1.0, np.abs(Bw).max() * np.abs(uf).max())
    grad = M * (uf - us) + Bw[:, ~is_p] @ (Dinv @ s[~is_p])
    N = sla.null_space(Bw[:, is_p].T)
    assert N.shape[1] > 0
    assert np.abs(N.T @ grad).max() < 1e-8 * np.abs(grad).max()

    def J(v):
        sv = Bw.T @ v + cvec
        return 0.5 * np.sum(M * (v - us) ** 2) + 0.5 * sv[~is_p] @ Dinv @ sv[~is_p]

    for _ in range(5):
        d = N @ rng.normal(size=N.shape[1])
        assert J(uf + 1e-3 * d) > J(uf)


@pytest.mark.parametrize("dim,n", [(2, 32), (3, 12)])
def test_hydrostatic_rest_is_exact(dim, n):
    rng = np.random.default_rng(dim)
    X = cases.node_coords((n,) * dim, 1.0 / n, (0.0,) * dim)
    phi_l = X[1] - 0.537
    ctr = np.array([0.45, 0.25, 0.5][:dim])
    phi_s = np.sqrt(sum((X[a] - ctr[a]) ** 2 for a in range(dim))) - 0.13
    g = [0.0] * dim
    g[1] = -9.8
    zero = [np.zeros(s) for s in cases.face_shapes((n,) * dim)]
    c = _box_case(dim, n, phi_l, phi_s, rng, dt=0.05, g=tuple(g), u=zero,
                  rho=np.full((n,) * dim, 1.3))
    asm, x, u = system.step(c)
    assert np.abs(x).max() > 0.1            # a genuine hydrostatic pressure
    assert np.abs(u).max() <= 1e-12 * 0.05 * 9.8 * 1e3


@pytest.mark.parametrize("dim,n", [(2, 24), (3, 10)])
def test_rigid_motion_of_free_surface_body_is_exact(dim, n):
    rng = np.random.default_rng(10 + dim)
    X = cases.node_coords((n,) * dim, 1.0 / n, (0.0,) * dim)
    phi_l = np.sqrt(sum((X[a] - 0.5) ** 2 for a in range(dim))) - 0.3
    V = rng.normal(size=dim)
    W = rng.normal(size=3)
    u = []
    for a in range(dim):
        F = cases.face_coords((n,) * dim, 1.0 / n, (0.0,) * dim, a)
        r = [F[q] - 0.5 for q in range(dim)]
        if dim == 2:
            rot = [-W[2] * r[1], W[2] * r[0]][a]
        else:
            rot = [W[1] * r[2] - W[2] * r[1], W[2] * r[0] - W[0] * r[2], W[0] * r[1] - W[1] * r[0]][a]
        u.append(V[a] + rot)
    c = _box_case(dim, n, phi_l, None, rng, u=u)
    asm, x, uh = system.step(c)
    us = np.concatenate([asm.grid.flat(q) for q in asm.u_star])
    m = asm.K > 0
    assert np.abs(x).max() < 1e-11
    assert np.abs(uh - us)[m].max() < 1e-12


@pytest.mark.parametrize("dim,n", [(2, 24), (3, 10)])
def test_co_motion_with_moving_solid_is_exact(dim, n):
    rng = np.random.default_rng(20 + dim)
    phi_l, phi_s, ubc, V = _moving_solid_case(dim, n, rng)
    u = [np.full(s, V[a]) for a, s in enumerate(cases.face_shapes((n,) * dim))]
    c = _box_case(dim, n, phi_l, phi_s, rng, u=u, ubc=ubc)
    asm, x, uh = system.step(c)
    m = asm.K > 0
    assert np.abs(x).max() < 1e-10
    assert np.abs(uh[m] - np.concatenate([np.full(asm.grid.size(fs), V[a])
                                          for a, fs in enumerate(asm.grid.faces)])[m]).max() < 1e-12


def _errors(name, n):
    c = analytic.make_case(name, n)
    asm, x, u = system.step(c)
    ex = analytic.exact_on_grid(name, n)
    g = asm.grid
    ue = np.concatenate([g.flat(ex["u"]), g.flat(ex["v"])])
    m = asm.K > 0
    e = np.abs(u - ue)[m]
    lo, hi = g.sample_offsets()["p"]
    act = asm.active[lo:hi]
    dp = (x[lo:hi] - g.flat(ex["p"]))[act]
    if system.is_enclosed(asm):
        dp = dp - dp.mean()
    return e.max(), e.sum() * g.h ** 2, np.abs(dp).sum() * g.h ** 2


@pytest.mark.parametrize("name", ["E2", "E3", "E4", "E5"])
def test_first_order_velocity_convergence(name):
    """Least-squares orders over n = 32..512: velocity L1 >= 0.9 and L-inf
    >= 0.7 (the paper's per-level orders scatter between 0.46 and 2.5 and its
    summary table states first order), pressure L1 >= 0.8.  Velocity L1 is
    within a factor 3 of the paper's table at 128..512 (context pin)."""
    ns = np.array([32, 64, 128, 256, 512])
    E = np.array([_errors(name, int(n)) for n in ns])
    slope = lambda k: -np.polyfit(np.log(ns), np.log(E[:, k]), 1)[0]
    assert slope(0) >= 0.7, E[:, 0]
    assert slope(1) >= 0.9, E[:, 1]
    assert slope(2) >= 0.8, E[:, 2]
    gold = json.load(open(GOLDEN))
    for n, e1 in zip(ns[2:], E[2:, 1]):
        ref = gold[name]["l1"][gold["grids"].index(int(n))]
        assert ref / 3 <= e1 <= 3 * ref, (name, n, e1, ref)


def test_analytic_fields_satisfy_their_boundary_conditions():
    """The readings of the printed cases: traction-free at r = 0.75 (E2) and
    r = 0.65 (E4); static walls for E3; E5's inner wall rotates clockwise
    with omega = 2 and its outer wall is static."""
    ang = np.linspace(0.1, 6.0, 7)
    for name, R in (("E2", 0.75), ("E4", 0.65)):
        f = analytic.exact_functions(name)
        x, y = R * np.cos(ang), R * np.sin(ang)
        p = f["p"](x, y)
        txx, txy = f["txx"](x, y), f["txy"](x, y)
        nx, ny = np.cos(ang), np.sin(ang)
        tx = (-p + txx) * nx + txy * ny
        ty = txy * nx + (-p - txx) * ny
        assert np.abs(tx).max() < 1e-12 and np.abs(ty).max() < 1e-12
    f = analytic.exact_functions("E3")
    for R in (0.5, 1.0):
        assert np.abs(f["u"](R * np.cos(ang), R * np.sin(ang))).max() < 1e-9
    f = analytic.exact_functions("E5")
    x, y = 0.5 * np.cos(ang), 0.5 * np.sin(ang)
    assert np.allclose(f["u"](x, y), 2 * y) and np.allclose(f["v"](x, y), -2 * x)
    x, y = np.cos(ang), np.sin(ang)
    assert np.abs(f["u"](x, y)).max() < 1e-12 and np.abs(f["v"](x, y)).max() < 1e-12
