"""Manufactured solutions of one backward-Euler Stokes step in a box full of
liquid, with smooth variable density and viscosity (2D and 3D).

The final velocity is divergence free and vanishes with its first
derivatives on the box walls:
  2D  u = (psi_y, -psi_x),        psi = sin^2(pi x) sin^2(pi y)
  3D  u = grad(psi) x a,           psi = sin^2(pi x) sin^2(pi y) sin^2(pi z),
                                   a = (1, 1/2, -7/10)
so the no-slip walls of the box hold exactly.  Stresses follow Section 4's
constitutive law tau = mu (grad u + grad u^T) with the point value of the
smooth viscosity field, and the input velocity from the momentum equation
of the backward-Euler step,
  u* = u - (dt / rho) (div tau - grad p),
with the smooth density at the face.  Derivatives are symbolic (SymPy).
Cell-centred rho and mu are the point values at cell centres; the method
averages them to faces and stress samples itself.
"""
from __future__ import annotations

import functools

import numpy as np
import sympy as S

import cases

DT = 0.1


def _fields(dim):
    x, y, z = S.symbols("x y z", real=True)
    X = (x, y, z)[:dim]
    pi = S.pi
    if dim == 2:
        psi = S.sin(pi * x) ** 2 * S.sin(pi * y) ** 2
        u = [S.diff(psi, y), -S.diff(psi, x)]
        mu = 1 + S.Rational(1, 2) * S.sin(2 * pi * x + 1) * S.cos(pi * y)
        rho = S.Rational(3, 2) + S.Rational(1, 2) * S.cos(pi * x - 2 * pi * y)
        p = S.cos(pi * x) * S.sin(pi * y)
    else:
        psi = S.sin(pi * x) ** 2 * S.sin(pi * y) ** 2 * S.sin(pi * z) ** 2
        a = (1, S.Rational(1, 2), -S.Rational(7, 10))
        g = [S.diff(psi, q) for q in X]
        u = [g[1] * a[2] - g[2] * a[1], g[2] * a[0] - g[0] * a[2], g[0] * a[1] - g[1] * a[0]]
        mu = 1 + S.Rational(1, 2) * S.sin(2 * pi * x + 1) * S.cos(pi * y) * S.cos(pi * z / 2)
        rho = S.Rational(3, 2) + S.Rational(1, 2) * S.cos(pi * x - 2 * pi * y + pi * z)
        p = S.cos(pi * x) * S.sin(pi * y) * S.cos(pi * z)
    tau = [[mu * (S.diff(u[i], X[j]) + S.diff(u[j], X[i])) for j in range(dim)] for i in range(dim)]
    ustar = [u[i] - DT / rho * (sum(S.diff(tau[i][j], X[j]) for j in range(dim)) - S.diff(p, X[i]))
             for i in range(dim)]
    return X, dict(u=u, ustar=ustar, tau=tau, mu=mu, rho=rho, p=p,
                   div=sum(S.diff(u[i], X[i]) for i in range(dim)))


@functools.lru_cache(maxsize=None)
def functions(dim):
    """Numeric (x, y[, z]) -> value callables of the manufactured fields:
    'u0'.., 'us0'.., 'tau{i}{j}', 'mu', 'rho', 'p', 'div'."""
    X, f = _fields(dim)
    out = {}
    lam = lambda e: S.lambdify(X, e, "numpy")
    for i in range(dim):
        out[f"u{i}"] = lam(f["u"][i])
        out[f"us{i}"] = lam(f["ustar"][i])
        for j in range(dim):
            out[f"tau{i}{j}"] = lam(f["tau"][i][j])
    for k in ("mu", "rho", "p", "div"):
        out[k] = lam(f[k])
    return out


def _ev(fn, coords):
    return np.asarray(fn(*coords), dtype=np.float64) * np.ones_like(coords[0])


def make_case(dim, n):
    """The box [0,1]^dim with n cells per axis, full of liquid (no solid
    besides the box walls, no gravity: the body force is inside u*)."""
    h = 1.0 / n
    nn = (n,) * dim
    o = (0.0,) * dim
    f = functions(dim)
    C = cases.cell_coords(nn, h, o)
    ustar = [_ev(f[f"us{a}"], cases.face_coords(nn, h, o, a)) for a in range(dim)]
    return dict(dim=dim, n=nn, h=h, origin=o, dt=DT,
                phi_l=-np.ones(tuple(q + 1 for q in nn)), phi_s=None,
                rho=_ev(f["rho"], C), mu=_ev(f["mu"], C),
                u=ustar, u_bc=None, g=(0.0,) * dim, name=f"manufactured{dim}d_{n}")


def exact_velocity(dim, n):
    h = 1.0 / n
    nn = (n,) * dim
    f = functions(dim)
    return [_ev(f[f"u{a}"], cases.face_coords(nn, h, (0.0,) * dim, a)) for a in range(dim)]
