"""Volume fractions of sample control volumes (paper Section 5, Figs. 3-4).

The paper weights every term by the fraction of material inside an h-sized
control volume centred on the sample and leaves the estimator open (it
cites a level-set based one).  This oracle uses an exact integrator of the
piecewise-linear interpolant on a half-resolution lattice:

 1. Nodal level set phi (phi < 0 inside, phi == 0 counts as outside) is
    refined to the h/2 lattice by multilinear interpolation, done as
    successive midpoint averaging along x, then y, then z:
    mid = (a + b) * 0.5.
 2. Every h/2 sub-cell is split into Kuhn simplices that share the diagonal
    from its min corner to its max corner: 2 triangles in 2D, 6 tetrahedra
    in 3D (one per axis permutation, in the order xyz, xzy, yxz, yzx, zxy,
    zyx).  The measure fraction of {phi < 0} in a simplex with linear phi is
    the closed form below; the sub-cell fraction is the simplex mean,
    (f1 + f2) * 0.5 in 2D and (((((f1+f2)+f3)+f4)+f5)+f6) / 6 in 3D.
 3. A control volume covers 2^d sub-cells; its weight is their mean, summed
    pairwise along x, then y, then z, times 0.25 or 0.125.

Simplex fraction of {phi < 0} (vertex values in simplex order; N = the
negative values in that order, P = the others in that order):
  triangle |N|=1: s^2 / ((s-t)(s-u))           with s=N0, (t,u)=P
  triangle |N|=2: 1 - t^2 / ((t-s)(t-r))       with (s,r)=N, t=P0
  tet      |N|=1: s^3 / ((s-t)(s-u)(s-w))
  tet      |N|=3: 1 - t^3 / ((t-s)(t-r)(t-q))
  tet      |N|=2: [s^2 r^2 - s r (s+r)(t+u) + t u (s^2 + s r + r^2)]
                  / ((s-t)(s-u)(r-t)(r-u))      with (s,r)=N, (t,u)=P
  none negative: 0, all negative: 1; results are clamped to [0, 1].
These are the sums over negative vertices v_i of v_i^d / prod_{j!=i}(v_i - v_j)
rearranged so that no subtraction of like-signed terms occurs.
"""
from __future__ import annotations

import numpy as np

TET_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def refine_half(phi):
    """Nodal values (n+1 per axis) -> h/2 lattice values (2n+1 per axis)."""
    f = np.asarray(phi, dtype=np.float64)
    for axis in range(f.ndim):
        m = f.shape[axis]
        shp = list(f.shape)
        shp[axis] = 2 * m - 1
        out = np.empty(shp)
        ev = [slice(None)] * f.ndim
        od = [slice(None)] * f.ndim
        lo = [slice(None)] * f.ndim
        hi = [slice(None)] * f.ndim
        ev[axis] = slice(0, None, 2)
        od[axis] = slice(1, None, 2)
        lo[axis] = slice(0, m - 1)
        hi[axis] = slice(1, m)
        out[tuple(ev)] = f
        out[tuple(od)] = (f[tuple(lo)] + f[tuple(hi)]) * 0.5
        f = out
    return f


def _order_neg_first(V):
    """Stable reorder of the last axis: negatives first (in vertex order),
    then non-negatives (in vertex order).  Returns (values, count_neg)."""
    neg = V < 0.0
    idx = np.argsort(~neg, axis=-1, kind="stable")
    return np.take_along_axis(V, idx, axis=-1), neg.sum(axis=-1)


def triangle_fraction(V):
    """V[..., 3] vertex values -> fraction of the triangle with phi < 0."""
    W, k = _order_neg_first(V)
    a, b, c = W[..., 0], W[..., 1], W[..., 2]
    out = np.where(k >= 3, 1.0, 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        one = (a * a) / ((a - b) * (a - c))          # s=a, t=b, u=c
        two = 1.0 - (c * c) / ((c - a) * (c - b))     # s=a, r=b, t=c
    out = np.where(k == 1, one, out)
    out = np.where(k == 2, two, out)
    return np.clip(out, 0.0, 1.0)


def tet_fraction(V):
    """V[..., 4] vertex values -> fraction of the tetrahedron with phi < 0."""
    W, k = _order_neg_first(V)
    a, b, c, d = W[..., 0], W[..., 1], W[..., 2], W[..., 3]
    out = np.where(k >= 4, 1.0, 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        # one negative: s=a; (t,u,w)=(b,c,d)
        one = ((a * a) * a) / (((a - b) * (a - c)) * (a - d))
        # two negatives: (s,r)=(a,b); (t,u)=(c,d)
        num = ((a * a) * (b * b) - ((a * b) * (a + b)) * (c + d)) \
            + (c * d) * (((a * a) + (a * b)) + (b * b))
        den = ((a - c) * (a - d)) * ((b - c) * (b - d))
        two = num / den
        # three negatives: (s,r,q)=(a,b,c); t=d
        three = 1.0 - ((d * d) * d) / (((d - a) * (d - b)) * (d - c))
    out = np.where(k == 1, one, out)
    out = np.where(k == 2, two, out)
    out = np.where(k == 3, three, out)
    return np.clip(out, 0.0, 1.0)


def subcell_fractions_2d(H):
    """H: h/2 lattice values (2nx+1, 2ny+1) -> sub-cell fractions (2nx, 2ny)."""
    c00 = H[:-1, :-1]
    c10 = H[1:, :-1]
    c01 = H[:-1, 1:]
    c11 = H[1:, 1:]
    t1 = triangle_fraction(np.stack([c00, c10, c11], axis=-1))
    t2 = triangle_fraction(np.stack([c00, c01, c11], axis=-1))
    return (t1 + t2) * 0.5


def _corner(H, off, nz_slice):
    sx = slice(off[0], H.shape[0] - 1 + off[0])
    sy = slice(off[1], H.shape[1] - 1 + off[1])
    sz = slice(nz_slice.start + off[2], nz_slice.stop + off[2])
    return H[sx, sy, sz]


def subcell_fractions_3d(H, chunk=16):
    """H: h/2 lattice values (2n+1)^3 -> sub-cell fractions (2n)^3.
    Processed in slabs along z to bound memory."""
    nz = H.shape[2] - 1
    out = np.empty((H.shape[0] - 1, H.shape[1] - 1, nz))
    for z0 in range(0, nz, chunk):
        zs = slice(z0, min(nz, z0 + chunk))
        c000 = _corner(H, (0, 0, 0), zs)
        c111 = _corner(H, (1, 1, 1), zs)
        acc = None
        for perm in TET_PERMS:
            o1 = [0, 0, 0]
            o1[perm[0]] = 1
            o2 = list(o1)
            o2[perm[1]] = 1
            v1 = _corner(H, tuple(o1), zs)
            v2 = _corner(H, tuple(o2), zs)
            f = tet_fraction(np.stack([c000, v1, v2, c111], axis=-1))
            acc = f if acc is None else acc + f
        out[:, :, zs] = acc / 6.0
    return out


def subcell_fractions(phi):
    H = refine_half(phi)
    return subcell_fractions_2d(H) if H.ndim == 2 else subcell_fractions_3d(H)


def cv_mean(theta_padded, stagger, shape):
    """Mean of the 2^d sub-cells covering each control volume.

    ``theta_padded`` is the sub-cell array with one extra layer on every side
    (index shift +1).  Along an axis where the sample is cell-centred
    (stagger 1) the control volume of index i covers sub-cells 2i, 2i+1;
    on a grid line (stagger 0) it covers 2i-1, 2i."""
    d = len(stagger)

    def pick(offs):
        sl = []
        for a in range(d):
            first = 2 * 0 + (0 if stagger[a] == 1 else -1) + offs[a] + 1
            sl.append(slice(first, first + 2 * shape[a], 2))
        return theta_padded[tuple(sl)]

    if d == 2:
        return ((pick((0, 0)) + pick((1, 0))) + (pick((0, 1)) + pick((1, 1)))) * 0.25
    return (((pick((0, 0, 0)) + pick((1, 0, 0))) + (pick((0, 1, 0)) + pick((1, 1, 0))))
            + ((pick((0, 0, 1)) + pick((1, 0, 1))) + (pick((0, 1, 1)) + pick((1, 1, 1))))) * 0.125


def sample_weights(grid, phi_l, phi_s, w_min=1e-3):
    """W_L and W_F for every sample type of ``grid`` (dict keyed by stagger).

    Box walls are static solids: sub-cells outside the box are solid
    (theta_F = 0) and take the liquid fraction of their mirror image inside
    the box; faces on the box boundary get W_F = 0.  Weights strictly below
    w_min are snapped to 0."""
    th_l = subcell_fractions(phi_l)
    if phi_s is None:
        th_f = np.ones_like(th_l)
    else:
        th_f = 1.0 - subcell_fractions(phi_s)
    th_l = np.pad(th_l, 1, mode="edge")
    th_f = np.pad(th_f, 1, mode="constant", constant_values=0.0)
    staggers = [grid.cell] + grid.faces + [s for _, s in grid.samples if s != grid.cell]
    out = {}
    for st in staggers:
        if st in out:
            continue
        shp = grid.shape(st)
        wl = cv_mean(th_l, st, shp)
        wf = cv_mean(th_f, st, shp)
        wl = np.where(wl < w_min, 0.0, wl)
        wf = np.where(wf < w_min, 0.0, wf)
        if st in grid.faces:
            a = grid.faces.index(st)
            idx = [slice(None)] * grid.dim
            idx[a] = 0
            wf[tuple(idx)] = 0.0
            idx[a] = -1
            wf[tuple(idx)] = 0.0
        out[st] = (wl, wf)
    return out
