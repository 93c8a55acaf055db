"""The advection half of the fractional step (Section 10): first-order
semi-Lagrangian advection of the face velocities (bilinear in 2D, trilinear in
3D) and of the nodal liquid level set, before the body force and the Stokes
step.  Test infrastructure only: plain NumPy, FP64.

Definitions (the paper names the scheme and leaves the details open; these
readings are shared with nothing else in the repository):
  * A sample type of stagger s (1 = cell-centred along that axis) has values
    at origin + (i + s/2) h, i = 0 .. shape - 1.  Its value at a point x is
    the multilinear interpolant of the 2^d surrounding samples, at the
    continuous index (x - origin)/h - s/2 clamped to [0, shape - 1] per axis
    (points outside the sample lattice take the value on its boundary).
  * The velocity at a point is the vector of the interpolated components.
  * Velocity extension: the Stokes step defines the velocity on faces with
    K > 0 (liquid) and W_F = 0 (solid and box walls); the others (air) are
    filled layer by layer, each face of a layer taking the mean of its
    already-known neighbours of the same component one index step away
    along each axis, for `layers` layers.  Faces still unknown keep their
    value (0 on air faces after a Stokes step).
  * Departure point of a sample at x: x - dt v(x) with the extended velocity
    (one backward Euler step).  The advected value is the interpolant of the
    extended field at the departure point; the level set uses the same
    velocity, interpolated at the nodes.
"""
from __future__ import annotations

import numpy as np


def interpolate(grid, values, stagger, points):
    """Multilinear interpolation of a sample field (native shape) at points
    (list of d coordinate arrays)."""
    d = grid.dim
    shp = values.shape
    base = []
    frac = []
    for b in range(d):
        xi = (np.asarray(points[b], np.float64) - grid.origin[b]) / grid.h - 0.5 * stagger[b]
        xi = np.clip(xi, 0.0, shp[b] - 1)
        i0 = np.minimum(np.floor(xi).astype(np.int64), max(shp[b] - 2, 0))
        base.append(i0)
        frac.append(xi - i0)
    out = np.zeros(np.broadcast(*points).shape)
    for corner in range(1 << d):
        w = np.ones_like(out)
        idx = []
        for b in range(d):
            up = (corner >> b) & 1
            w = w * (frac[b] if up else 1.0 - frac[b])
            idx.append(np.minimum(base[b] + up, shp[b] - 1))
        out = out + w * values[tuple(idx)]
    return out


def velocity_at(grid, u_faces, points):
    return [interpolate(grid, u_faces[a], grid.faces[a], points) for a in range(grid.dim)]


def extend_velocity(grid, u_faces, known, layers=3):
    """Fill unknown faces layer by layer with the mean of their known
    neighbours (same component, one index step along each axis)."""
    d = grid.dim
    out = [np.array(u, dtype=np.float64) for u in u_faces]
    kn = [np.array(k, dtype=bool) for k in known]
    for _ in range(layers):
        new_vals, new_known = [], []
        for a in range(d):
            v, k = out[a], kn[a]
            acc = np.zeros_like(v)
            cnt = np.zeros(v.shape)
            for b in range(d):
                for step in (-1, 1):
                    src = [slice(None)] * d
                    dst = [slice(None)] * d
                    if step == 1:     # neighbour at i + 1 feeds i
                        src[b], dst[b] = slice(1, None), slice(0, -1)
                    else:             # neighbour at i - 1 feeds i
                        src[b], dst[b] = slice(0, -1), slice(1, None)
                    kk = k[tuple(src)]
                    acc[tuple(dst)] += np.where(kk, v[tuple(src)], 0.0)
                    cnt[tuple(dst)] += kk
            fill = (~k) & (cnt > 0)
            nv = v.copy()
            nv[fill] = acc[fill] / cnt[fill]
            new_vals.append(nv)
            new_known.append(k | fill)
        out, kn = new_vals, new_known
    return out


def advect_velocity(grid, u_ext, dt):
    """Semi-Lagrangian advection of every face component by the extended
    velocity field."""
    out = []
    for a in range(grid.dim):
        X = grid.coords(grid.faces[a])
        v = velocity_at(grid, u_ext, X)
        dep = [X[b] - dt * v[b] for b in range(grid.dim)]
        out.append(interpolate(grid, u_ext[a], grid.faces[a], dep))
    return out


def advect_level_set(grid, phi_nodes, u_ext, dt):
    node = (0,) * grid.dim
    X = grid.coords(node)
    v = velocity_at(grid, u_ext, X)
    dep = [X[b] - dt * v[b] for b in range(grid.dim)]
    return interpolate(grid, np.asarray(phi_nodes, np.float64), node, dep)


def known_faces(asm):
    """Faces whose velocity the Stokes step of `asm` defines: K > 0 (liquid)
    or W_F = 0 (solid, box walls and invalid faces)."""
    known = (asm.K > 0.0) | (asm.wf_f == 0.0)
    return [asm.grid.unflat(known[lo:hi], asm.grid.faces[a])
            for a, (lo, hi) in enumerate(asm.grid.face_offsets())]


def ns_step(case, dt, prev=None, layers=3):
    """One step of the fractional step of Section 10 on a case dict: extend
    the velocity of the previous Stokes step into the air (all faces known
    before the first step), advect velocity and liquid level set, then the
    Stokes step (body force, solve, velocity recovery).  Returns the case of
    the next step (advected level set, new velocity) and the step's
    (assembly, solution, face velocity vector)."""
    from . import system
    from .grid import Grid
    grid = Grid(case["n"], case["h"], case.get("origin"))
    u = [np.asarray(q, np.float64) for q in case["u"]]
    known = [np.ones(q.shape, dtype=bool) for q in u] if prev is None else known_faces(prev)
    u_ext = extend_velocity(grid, u, known, layers)
    nxt = dict(case)
    nxt["u"] = advect_velocity(grid, u_ext, dt)
    nxt["phi_l"] = advect_level_set(grid, case["phi_l"], u_ext, dt)
    asm, x, uf = system.step(nxt, dt)
    out = dict(nxt)
    out["u"] = system.split_faces(grid, uf)
    return out, (asm, x, uf)


def ns_run(case, dt, steps, layers=3):
    """`steps` fractional steps from `case`; returns the final case and the
    list of per-step (assembly, solution, velocity)."""
    prev = None
    hist = []
    for _ in range(steps):
        case, res = ns_step(case, dt, prev, layers)
        prev = res[0]
        hist.append(res)
    return case, hist
