"""Seeded synthetic inputs for the variational Stokes step.

This module only *generates inputs*: level sets at grid nodes, cell-centred
density and viscosity, face velocities, prescribed solid velocities, gravity.
It contains none of the method's arithmetic (no fractions, no operators, no
solve), so both the CPU oracle tests and the GPU path can consume the same
arrays without sharing any computation.

Conventions (used by every consumer):
  * index order [i, j(, k)] = (x, y(, z)); arrays flatten x-fastest with
    ``np.ravel(order="F")``;
  * grid of nx*ny(*nz) cells of size h, box [origin, origin + n*h];
  * nodal level sets have shape (nx+1, ny+1(, nz+1)); phi < 0 is inside;
  * face arrays: u (nx+1, ny(, nz)), v (nx, ny+1(, nz)), w (nx, ny, nz+1);
  * cell arrays (rho, mu): (nx, ny(, nz)).

Workloads (one base seed each, recorded by the caller):
  drop32     2D 32^2 drop above a solid floor, FP64 reference case.
  pool512    2D 512^2 pool + 8 random circles + moving solid disc,
             smooth log-uniform viscosity [1,1000] and density [0.5,2].
  column128  3D 128^3 falling column with perturbed radius onto a floor.
  batch64    64 independent 2D problems, n in {64,96,...,512}, each shaped as
             drop32 with its own seed.
  pool256    3D 256^3 analogue of pool512 (pool + 8 spheres + moving sphere).
  sphere_core3d  liquid sphere with a static solid core (3D convergence study).
  jet2d, jet3d   viscous jets from a moving nozzle (fractional-step demos).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "node_coords", "face_coords", "cell_coords",
    "drop32", "pool512", "column128", "batch64", "pool256",
    "drop2d", "pool2d", "pool3d", "column3d", "sphere_core3d", "jet2d", "jet3d",
]


# --------------------------------------------------------------------------
# coordinates
# --------------------------------------------------------------------------
def _axis(n, h, o, staggered_half):
    k = np.arange(n, dtype=np.float64)
    return o + (k + (0.5 if staggered_half else 0.0)) * h


def node_coords(n, h, origin):
    """Coordinates of grid nodes, one meshgrid array per axis (ij indexing)."""
    axes = [_axis(n[a] + 1, h, origin[a], False) for a in range(len(n))]
    return np.meshgrid(*axes, indexing="ij")


def cell_coords(n, h, origin):
    axes = [_axis(n[a], h, origin[a], True) for a in range(len(n))]
    return np.meshgrid(*axes, indexing="ij")


def face_coords(n, h, origin, axis):
    """Coordinates of the faces normal to ``axis`` (MAC velocity samples)."""
    axes = []
    for a in range(len(n)):
        if a == axis:
            axes.append(_axis(n[a] + 1, h, origin[a], False))
        else:
            axes.append(_axis(n[a], h, origin[a], True))
    return np.meshgrid(*axes, indexing="ij")


def face_shapes(n):
    d = len(n)
    return [tuple(n[b] + (1 if b == a else 0) for b in range(d)) for a in range(d)]


# --------------------------------------------------------------------------
# smooth random fields
# --------------------------------------------------------------------------
def _gauss_field(rng, X, count=4):
    """Sum of ``count`` random Gaussians, min-max normalised to [0, 1]."""
    d = len(X)
    s = np.zeros_like(X[0])
    for _ in range(count):
        a = rng.uniform(0.5, 1.0)
        m = rng.uniform(0.0, 1.0, size=d)
        sig = rng.uniform(0.1, 0.3)
        r2 = sum((X[q] - m[q]) ** 2 for q in range(d))
        s = s + a * np.exp(-r2 / (2.0 * sig * sig))
    lo, hi = s.min(), s.max()
    return (s - lo) / (hi - lo) if hi > lo else np.zeros_like(s)


def _case(dim, n, h, origin, dt, phi_l, phi_s, rho, mu, u, u_bc, g, **meta):
    c = dict(dim=dim, n=tuple(int(q) for q in n), h=float(h),
             origin=tuple(float(o) for o in origin), dt=float(dt),
             phi_l=phi_l, phi_s=phi_s, rho=rho, mu=mu, u=list(u),
             u_bc=None if u_bc is None else list(u_bc), g=tuple(float(q) for q in g))
    c.update(meta)
    return c


# --------------------------------------------------------------------------
# 2D drop above a floor (drop32, and each member of batch64)
# --------------------------------------------------------------------------
def drop2d(n, seed, dt=0.01, radius=0.35, centre=(0.5, 0.5), floor=0.1,
           sigma=0.1, rho=1.0, mu=1.0, g=(0.0, -1.0)):
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    nn = (n, n)
    X, Y = node_coords(nn, h, (0.0, 0.0))
    phi_l = np.hypot(X - centre[0], Y - centre[1]) - radius
    phi_s = Y - floor
    u = [rng.normal(0.0, sigma, size=s) for s in face_shapes(nn)]
    return _case(2, nn, h, (0.0, 0.0), dt, phi_l, phi_s,
                 np.full(nn, rho), np.full(nn, mu), u, None, g,
                 name=f"drop2d_{n}", seed=seed)


def drop32(seed=1):
    c = drop2d(32, seed)
    c.update(name="drop32", tol=1e-10, precision="fp64")
    return c


# --------------------------------------------------------------------------
# 2D pool with random circles and a moving disc (pool512)
# --------------------------------------------------------------------------
def pool2d(n, seed, dt=1e-3, n_circles=8, depth=0.3, g=(0.0, -1.0)):
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    nn = (n, n)
    X, Y = node_coords(nn, h, (0.0, 0.0))
    phi_l = Y - depth
    for _ in range(n_circles):
        r = rng.uniform(0.05, 0.2)
        cx = rng.uniform(r, 1.0 - r)
        cy = rng.uniform(depth + r, 1.0 - r)
        phi_l = np.minimum(phi_l, np.hypot(X - cx, Y - cy) - r)
    rs = rng.uniform(0.05, 0.15)
    cs = rng.uniform(0.25, 0.75, size=2)
    V = rng.uniform(-1.0, 1.0, size=2)
    phi_s = np.hypot(X - cs[0], Y - cs[1]) - rs
    XC = cell_coords(nn, h, (0.0, 0.0))
    mu = 10.0 ** (3.0 * _gauss_field(rng, XC))
    rho = 0.5 + 1.5 * _gauss_field(rng, XC)
    u = [rng.normal(0.0, 0.1, size=s) for s in face_shapes(nn)]
    # prescribed solid velocity: the disc's rigid translation V on faces
    # within 3h of the disc (its value elsewhere never enters the system)
    u_bc = []
    for a in range(2):
        F = face_coords(nn, h, (0.0, 0.0), a)
        near = np.hypot(F[0] - cs[0], F[1] - cs[1]) - rs < 3.0 * h
        u_bc.append(np.where(near, V[a], 0.0))
    return _case(2, nn, h, (0.0, 0.0), dt, phi_l, phi_s, rho, mu, u, u_bc, g,
                 name=f"pool2d_{n}", seed=seed, solid_velocity=tuple(V))


def pool512(seed=2, n=512):
    c = pool2d(n, seed)
    c.update(name="pool512", tol=1e-6, precision="mixed")
    return c


# --------------------------------------------------------------------------
# 3D falling column with a perturbed surface (column128)
# --------------------------------------------------------------------------
def column3d(n, seed, dt=1e-3, top=0.8, floor=0.1, radius=0.05, amp=0.01,
             mu=50.0, rho=1.0, speed=-0.5, g=(0.0, -9.8, 0.0)):
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    nn = (n, n, n)
    X, Y, Z = node_coords(nn, h, (0.0, 0.0, 0.0))
    m = int(rng.integers(2, 5))
    lam = rng.uniform(0.1, 0.3)
    alpha, beta = rng.uniform(0.0, 2.0 * np.pi, size=2)
    rr = np.hypot(X - 0.5, Z - 0.5)
    th = np.arctan2(Z - 0.5, X - 0.5)
    R = radius + amp * np.cos(m * th + alpha) * np.cos(2.0 * np.pi * Y / lam + beta)
    phi_l = np.maximum(rr - R, Y - top)
    phi_s = Y - floor
    u = [np.zeros(s) for s in face_shapes(nn)]
    u[1][...] = speed
    return _case(3, nn, h, (0.0, 0.0, 0.0), dt, phi_l, phi_s,
                 np.full(nn, rho), np.full(nn, mu), u, None, g,
                 name=f"column3d_{n}", seed=seed)


def column128(seed=3, n=128):
    c = column3d(n, seed)
    c.update(name="column128", tol=1e-6, precision="mixed")
    return c


# --------------------------------------------------------------------------
# batched 2D (batch64)
# --------------------------------------------------------------------------
def batch64_sizes(seed=4, count=64):
    rng = np.random.default_rng(seed)
    return [int(v) for v in rng.choice(np.arange(64, 513, 32), size=count)]


def batch64(seed=4, count=64):
    sizes = batch64_sizes(seed, count)
    return [dict(drop2d(n, seed * 1000 + q), tol=1e-6, precision="mixed")
            for q, n in enumerate(sizes)]


# --------------------------------------------------------------------------
# 3D pool with random spheres and a moving sphere (pool256)
# --------------------------------------------------------------------------
def pool3d(n, seed, dt=1e-3, n_spheres=8, depth=0.3, g=(0.0, -9.8, 0.0)):
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    nn = (n, n, n)
    X, Y, Z = node_coords(nn, h, (0.0, 0.0, 0.0))
    phi_l = Y - depth
    for _ in range(n_spheres):
        r = rng.uniform(0.05, 0.2)
        cx, cz = rng.uniform(r, 1.0 - r, size=2)
        cy = rng.uniform(depth + r, 1.0 - r)
        phi_l = np.minimum(phi_l, np.sqrt((X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2) - r)
    del X, Y, Z
    rs = rng.uniform(0.05, 0.15)
    cs = rng.uniform(0.25, 0.75, size=3)
    V = rng.uniform(-1.0, 1.0, size=3)
    X, Y, Z = node_coords(nn, h, (0.0, 0.0, 0.0))
    phi_s = np.sqrt((X - cs[0]) ** 2 + (Y - cs[1]) ** 2 + (Z - cs[2]) ** 2) - rs
    del X, Y, Z
    XC = cell_coords(nn, h, (0.0, 0.0, 0.0))
    mu = 10.0 ** (3.0 * _gauss_field(rng, XC))
    rho = 0.5 + 1.5 * _gauss_field(rng, XC)
    del XC
    u = [rng.normal(0.0, 0.1, size=s) for s in face_shapes(nn)]
    u_bc = []
    for a in range(3):
        F = face_coords(nn, h, (0.0, 0.0, 0.0), a)
        dist = np.sqrt((F[0] - cs[0]) ** 2 + (F[1] - cs[1]) ** 2 + (F[2] - cs[2]) ** 2) - rs
        del F
        u_bc.append(np.where(dist < 3.0 * h, V[a], 0.0))
    return _case(3, nn, h, (0.0, 0.0, 0.0), dt, phi_l, phi_s, rho, mu, u, u_bc, g,
                 name=f"pool3d_{n}", seed=seed, solid_velocity=tuple(V))


def pool256(seed=5, n=256):
    c = pool3d(n, seed)
    c.update(name="pool256", tol=1e-6, precision="mixed")
    return c


# --------------------------------------------------------------------------
# sub-box of a case (full-size checks on pieces the oracle can assemble)
# --------------------------------------------------------------------------
def crop(case, lo, m):
    """The case restricted to the cells [lo[a], lo[a] + m[a]) of each axis:
    level sets at the nodes of those cells, rho and mu at the cells, face
    velocities and solid velocities at their faces, the origin moved to the
    sub-box corner.  The sub-box's own boundary acts as a box wall, so only
    quantities far enough from it agree with the full case."""
    d = case["dim"]
    lo = tuple(int(q) for q in lo)
    m = tuple(int(q) for q in m)
    for a in range(d):
        if lo[a] < 0 or m[a] < 1 or lo[a] + m[a] > case["n"][a]:
            raise ValueError(f"crop {lo}+{m} outside the grid {case['n']}")
    node = tuple(slice(lo[a], lo[a] + m[a] + 1) for a in range(d))
    cell = tuple(slice(lo[a], lo[a] + m[a]) for a in range(d))

    def faces(arrs):
        out = []
        for ax, f in enumerate(arrs):
            sl = tuple(slice(lo[b], lo[b] + m[b] + (1 if b == ax else 0)) for b in range(d))
            out.append(np.array(np.asarray(f)[sl]))
        return out

    h = case["h"]
    origin = tuple(case["origin"][a] + lo[a] * h for a in range(d))
    return _case(d, m, h, origin, case["dt"], np.array(case["phi_l"][node]),
                 np.array(case["phi_s"][node]), np.array(np.asarray(case["rho"])[cell]),
                 np.array(np.asarray(case["mu"])[cell]), faces(case["u"]),
                 None if case["u_bc"] is None else faces(case["u_bc"]), case["g"],
                 name=f"{case.get('name', 'case')}_crop{lo}+{m}")


# --------------------------------------------------------------------------
# 3D sphere with a solid core (the three-dimensional convergence study)
# --------------------------------------------------------------------------
def sphere_core3d(n, half=1.2, radius=1.0, core=0.25, mu=0.1, rho=1.0, dt=1.0):
    """A liquid sphere of the given radius centred at the origin with a free
    surface, a static solid sphere of radius `core` at its centre, one step
    from the input velocity
        (0.5 + x sin(yz), cos(y/4) + xyz/2, x + yz^2/2 + sqrt(2 + y^2)),
    no gravity; box [-half, half]^3 with n cells per axis (its walls, static
    solids, do not touch the liquid when half > radius)."""
    h = 2.0 * half / n
    nn = (n, n, n)
    o = (-half, -half, -half)
    X, Y, Z = node_coords(nn, h, o)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    phi_l = r - radius
    phi_s = r - core
    del X, Y, Z, r
    fns = (lambda x, y, z: 0.5 + x * np.sin(y * z),
           lambda x, y, z: np.cos(0.25 * y) + 0.5 * x * y * z,
           lambda x, y, z: x + 0.5 * y * z * z + np.sqrt(2.0 + y * y))
    u = []
    for a in range(3):
        F = face_coords(nn, h, o, a)
        u.append(fns[a](*F))
        del F
    return _case(3, nn, h, o, dt, phi_l, phi_s, np.full(nn, rho), np.full(nn, mu), u, None,
                 (0.0, 0.0, 0.0), name=f"sphere_core3d_{n}")


# --------------------------------------------------------------------------
# viscous jet buckling (the application of the fractional step)
# --------------------------------------------------------------------------
def jet2d(n=150, dt=2e-3, mu=0.075, rho=1.0, speed=0.5, width=0.06, ceiling=0.8,
          radius=0.4, g=(0.0, -9.81)):
    """2D planar jet: a disc-shaped container of the given radius around
    (0.5, 0.5) (solid outside), a solid ceiling above y = ceiling whose part
    over |x - 0.5| < width/2 (the nozzle) moves down at `speed`, and a short
    liquid column under the nozzle.  `jet_seed` is the liquid level set the
    nozzle keeps filled (the caller takes the minimum with it each step)."""
    h = 1.0 / n
    nn = (n, n)
    X, Y = node_coords(nn, h, (0.0, 0.0))
    phi_s = np.minimum(radius - np.hypot(X - 0.5, Y - 0.5), ceiling - Y)
    seed = np.maximum(np.abs(X - 0.5) - 0.5 * width, ceiling - 2.0 * h - Y)
    phi_l = np.maximum(np.abs(X - 0.5) - 0.5 * width, ceiling - 0.05 - Y)
    u_bc = []
    for a in range(2):
        F = face_coords(nn, h, (0.0, 0.0), a)
        inside = (np.abs(F[0] - 0.5) < 0.5 * width) & (F[1] > ceiling - 2.0 * h)
        u_bc.append(np.where(inside, -speed if a == 1 else 0.0, 0.0))
    u = [np.where(q != 0.0, q, 0.0) for q in u_bc]
    c = _case(2, nn, h, (0.0, 0.0), dt, phi_l, phi_s, np.full(nn, rho), np.full(nn, mu), u, u_bc, g,
              name=f"jet2d_{n}")
    c["jet_seed"] = seed
    return c


def jet3d(n=80, dt=2e-3, mu=0.3, rho=1.0, speed=0.5, diameter=0.08, ceiling=0.8,
          radius=0.4, g=(0.0, -9.81, 0.0)):
    """3D cylindrical jet: a spherical container of the given radius around
    (0.5, 0.5, 0.5) (solid outside), a solid ceiling above y = ceiling whose
    part over the inlet disc of the given diameter around x = z = 0.5 moves
    down at `speed`, and a short liquid column under the inlet; `jet_seed` as
    in jet2d."""
    h = 1.0 / n
    nn = (n, n, n)
    X, Y, Z = node_coords(nn, h, (0.0, 0.0, 0.0))
    rr = np.hypot(X - 0.5, Z - 0.5)
    phi_s = np.minimum(radius - np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2),
                       ceiling - Y)
    seed = np.maximum(rr - 0.5 * diameter, ceiling - 2.0 * h - Y)
    phi_l = np.maximum(rr - 0.5 * diameter, ceiling - 0.05 - Y)
    del X, Y, Z, rr
    u_bc = []
    for a in range(3):
        F = face_coords(nn, h, (0.0, 0.0, 0.0), a)
        inside = (np.hypot(F[0] - 0.5, F[2] - 0.5) < 0.5 * diameter) & (F[1] > ceiling - 2.0 * h)
        u_bc.append(np.where(inside, -speed if a == 1 else 0.0, 0.0))
    u = [q.copy() for q in u_bc]
    c = _case(3, nn, h, (0.0, 0.0, 0.0), dt, phi_l, phi_s, np.full(nn, rho), np.full(nn, mu), u,
              u_bc, g, name=f"jet3d_{n}")
    c["jet_seed"] = seed
    return c
