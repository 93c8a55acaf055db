"""Closed-form 2D test cases of the paper's convergence study (Section 9).

Each case gives a divergence-free final velocity through a stream function
psi (u = psi_y, v = -psi_x), a pressure p, density 1, viscosity 0.1 and
dt = 1 on the box [-1, 1]^2 with n^2 cells (h = 2/n).  The input velocity
follows from the backward-Euler equations of Section 4:
    u* = u - (dt/rho) (mu Lap u - grad p)       (constant mu, div u = 0)
and the stresses from tau = mu (grad u + grad u^T).  Derivatives are taken
symbolically with SymPy.

  E2 free-surface disk: liquid r < 0.75 (the printed stream function is
     traction-free at r = 0.75, not at r = 1; checked in the tests).
  E3 solid annulus 0.5 < r < 1, both walls static.
  E4 inner solid r < 0.1, free surface at r = 0.65 (the printed fields are
     traction-free there); the inner solid moves with the exact velocity.
  E5 annulus 0.5 < r < 1, inner wall rotating clockwise with omega = 2,
     outer wall static.
"""
from __future__ import annotations

import functools

import numpy as np
import sympy as S

import cases

X, Y = S.symbols("x y", real=True)
R = S.sqrt(X ** 2 + Y ** 2)
COS2 = (X ** 2 - Y ** 2) / R ** 2
SIN2 = 2 * X * Y / R ** 2
MU = S.Rational(1, 10)
RHO = 1
DT = 1


def _psi_p(name):
    if name == "E2":
        psi = S.Rational(128, 81) * R ** 4 * COS2 * S.cos(S.sqrt(3) * S.log(R)) * (15 - 30 * R + 16 * R ** 2)
        p = S.Rational(512, 81) * S.sqrt(3) * R ** 2 * MU * SIN2 * S.sin(S.sqrt(3) * S.log(R)) * (15 - 30 * R + 16 * R ** 2)
    elif name in ("E3",):
        psi = 256 * R ** 4 - 768 * R ** 3 + 832 * R ** 2 - 384 * R + 64
        p = X * Y
    elif name == "E4":
        psi = S.Rational(80000, 371293) * COS2 * R ** 4 * S.cos(S.sqrt(3) * S.log(R)) * (169 - 390 * R + 240 * R ** 2)
        p = S.Rational(320000, 371293) * S.sqrt(3) * MU * R ** 2 * SIN2 * S.sin(S.sqrt(3) * S.log(R)) * (169 - 390 * R + 240 * R ** 2)
    elif name == "E5":
        psi = R ** 4 - 3 * R ** 3 + S.Rational(9, 4) * R ** 2 + S.Rational(1, 2) * R + S.Rational(1, 4)
        p = X * Y
    else:
        raise KeyError(name)
    return psi, p


@functools.lru_cache(maxsize=None)
def exact_functions(name):
    """Numeric functions (x, y) -> value for u, v, p, txx, txy, ustar, vstar."""
    psi, p = _psi_p(name)
    u = S.diff(psi, Y)
    v = -S.diff(psi, X)
    txx = 2 * MU * S.diff(u, X)            # = mu (u_x - v_y) since div u = 0
    txy = MU * (S.diff(u, Y) + S.diff(v, X))
    lap = lambda f: S.diff(f, X, 2) + S.diff(f, Y, 2)
    us = u - S.Rational(DT, RHO) * (MU * lap(u) - S.diff(p, X))
    vs = v - S.Rational(DT, RHO) * (MU * lap(v) - S.diff(p, Y))
    out = {}
    for key, expr in dict(u=u, v=v, p=p, txx=txx, txy=txy, us=us, vs=vs).items():
        out[key] = S.lambdify((X, Y), expr, "numpy")
    return out


def _safe(f, x, y):
    """Evaluate away from the origin singularity of log r (values there are
    never used: the origin is inside a solid or the fields vanish)."""
    rr = np.hypot(x, y)
    xs = np.where(rr < 1e-12, 1e-12, x)
    with np.errstate(all="ignore"):
        val = np.asarray(f(xs, y), dtype=np.float64) * np.ones_like(x)
    return np.nan_to_num(val)


def make_case(name, n):
    h = 2.0 / n
    nn = (n, n)
    o = (-1.0, -1.0)
    f = exact_functions(name)
    XN, YN = cases.node_coords(nn, h, o)
    rn = np.hypot(XN, YN)
    if name == "E2":
        phi_l, phi_s = rn - 0.75, None
    elif name in ("E3", "E5"):
        phi_l = -np.ones_like(rn)
        phi_s = np.minimum(rn - 0.5, 1.0 - rn)
    elif name == "E4":
        phi_l, phi_s = rn - 0.65, rn - 0.1
    FU = cases.face_coords(nn, h, o, 0)
    FV = cases.face_coords(nn, h, o, 1)
    ustar = [_safe(f["us"], *FU), _safe(f["vs"], *FV)]
    u_bc = None
    if name == "E4":
        u_bc = [_safe(f["u"], *FU), _safe(f["v"], *FV)]
    elif name == "E5":
        u_bc = []
        for F, comp in ((FU, 0), (FV, 1)):
            rr = np.hypot(F[0], F[1])
            rot = 2.0 * F[1] if comp == 0 else -2.0 * F[0]     # clockwise, omega = 2
            u_bc.append(np.where(rr < 0.75, rot, 0.0))
    c = dict(dim=2, n=nn, h=h, origin=o, dt=float(DT), phi_l=phi_l, phi_s=phi_s,
             rho=np.full(nn, float(RHO)), mu=np.full(nn, float(MU)),
             u=ustar, u_bc=u_bc, g=(0.0, 0.0), name=f"{name}_{n}")
    return c


def exact_on_grid(name, n):
    """Exact u, v at faces, p and txx at cells, txy at nodes."""
    h = 2.0 / n
    nn = (n, n)
    o = (-1.0, -1.0)
    f = exact_functions(name)
    FU = cases.face_coords(nn, h, o, 0)
    FV = cases.face_coords(nn, h, o, 1)
    C = cases.cell_coords(nn, h, o)
    N = cases.node_coords(nn, h, o)
    return dict(u=_safe(f["u"], *FU), v=_safe(f["v"], *FV), p=_safe(f["p"], *C),
                txx=_safe(f["txx"], *C), txy=_safe(f["txy"], *N))
