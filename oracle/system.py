"""The SPD (stress, pressure) system of one backward-Euler Stokes step.

Paper references (section / equation labels of the paper):
  * backward Euler step and its variational forms: Section 4,
    eqs. stokesequations1-3, stokesfreesurface, stokessolidwall;
  * combined free-surface + solid KKT: eq. stokesmixedsystem;
  * Schur complement on the velocity block -> SPD system:
    eq. stokesmixedsystemspd, in the factored form of Section 7
    ("Generalization and Further Factorization");
  * prescribed solid velocity right-hand side: Section 6.2;
  * prescribed traction on the free surface (p_BC, tau_BC): Section 6.1;
  * null-space elimination: Section 8;
  * body force: the fractional step of Section 10 (u* = u^n + dt g).

With the trace-free reduced stresses (see operators.py) the discrete
functional is
  1/2 (u-u*)^T P W_F W_L (u-u*) + dt p^T W_Lp G^T W_F u
      + dt tau^T W_Lt D W_F u - dt/2 tau^T C W_Ft W_Lt tau
where C is the compliance: 1/mu for tau_xx (2D) and every off-diagonal
stress, and (1/mu)[[1, 1/2], [1/2, 1]] on each 3D cell's (tau_xx, tau_yy)
pair (this reproduces the local relations tau_xx = mu(u_x - v_y) and
tau_xx + tau_yy/2 = mu(u_x - w_z) of Section 5).  Eliminating u gives

  A = dt B^T K B + Dg,   B = [G W_Lp | D^T W_Lt]   (faces x samples)
  K = diag(W_F / (rho W_L)) on faces with W_F > 0 and W_L > 0, else 0
  Dg = W_Ft W_Lt C on stresses, 0 on pressure
  b = B^T (W_F u* + W_S u_BC) - W_L W_S (B0^T u_BC),  B0 = [G | D^T]
  u = u* - dt (B x) / (rho W_L) on faces with K > 0; u_BC where W_F = 0.

Prescribed traction (Section 6.1).  With boundary values y = (tau_BC, p_BC)
given at the samples, the air-region integral of the boundary work adds
W_F [W_A^u B0 y - B0 (W_A y)] to the right-hand side of the velocity rows
(W_A = 1 - W_L), and every eliminated sample takes its boundary value y
instead of 0 (Section 8), which moves -W_F B0 (W_L y) of those samples to the
right-hand side too.  Together, with a = W_L * active,
  f = B0 (a y) - W_L^u (B0 y)
and eliminating u folds it into the input velocity on faces with K > 0:
  u*_eff = u* + dt f / (rho W_L).
Sign: the paper integrates with the normal pointing out of the air region,
and its right-hand side taken literally turns a uniform p_BC = p0 into a
liquid pressure shifted by -p0.  Here the work term has the sign for which a
prescribed pressure p_BC gives liquid pressure p = p_BC at the surface (the
uniform p0 shifts the pressure by +p0 and leaves the flow unchanged).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .grid import Grid
from .fractions import sample_weights
from .operators import b0 as build_b0


# ---------------------------------------------------------------------------
# (a1) body force
# ---------------------------------------------------------------------------
def body_force(u, g, dt):
    """u* = u^n + dt g on every face (the body-force half of the fractional
    step); advection is not part of this step."""
    return [np.asarray(u[a], dtype=np.float64) + dt * g[a] for a in range(len(u))]


# ---------------------------------------------------------------------------
# coefficient averaging
# ---------------------------------------------------------------------------
def cell_mean_at(grid, cell_values, stagger):
    """Mean of the in-box cells adjacent to each sample of ``stagger``.
    Along an axis where the sample lies on a grid line the neighbours are
    cells i-1 and i; along a cell-centred axis just cell i."""
    d = grid.dim
    pad = np.pad(np.asarray(cell_values, dtype=np.float64), 1, mode="constant",
                 constant_values=np.nan)
    shp = grid.shape(stagger)
    acc = np.zeros(shp)
    cnt = np.zeros(shp)
    offsets = [(-1, 0) if stagger[a] == 0 else (0,) for a in range(d)]
    for off in np.array(np.meshgrid(*offsets, indexing="ij")).reshape(d, -1).T:
        sl = tuple(slice(1 + off[a], 1 + off[a] + shp[a]) for a in range(d))
        v = pad[sl]
        ok = ~np.isnan(v)
        acc = acc + np.where(ok, v, 0.0)
        cnt = cnt + ok
    return acc / np.maximum(cnt, 1)


# ---------------------------------------------------------------------------
# assembly
# ---------------------------------------------------------------------------
@dataclass
class Assembly:
    grid: Grid
    dt: float
    W: dict                    # stagger -> (W_L, W_F)
    wl_s: np.ndarray           # W_L per sample (sample order)
    wf_s: np.ndarray           # W_F per sample
    wl_f: np.ndarray           # W_L per face (face order)
    wf_f: np.ndarray           # W_F per face, 0 on invalid faces
    invalid: np.ndarray        # per face: fluid face next to a zero-weight sample
    rho_f: np.ndarray
    mu_s: np.ndarray           # viscosity at stress samples (nan for p)
    K: np.ndarray              # per face
    bad: np.ndarray            # per face: W_F > 0 and W_L == 0
    active: np.ndarray         # per sample
    B0: sp.csr_matrix          # [G | D^T]
    B: sp.csr_matrix           # B0 diag(W_L * active)
    Dg: sp.csr_matrix          # compliance block (samples x samples), active only
    A_full: sp.csr_matrix      # dt B^T K B + Dg on all samples
    b_full: np.ndarray
    u_star: list               # input velocity (with the traction terms folded in)
    u_bc: np.ndarray           # per face (zero on box faces)
    act_idx: np.ndarray = field(default=None)
    u_star_in: list = field(default=None)    # u^n + dt g (before the traction terms)
    y_bc: np.ndarray = field(default=None)   # prescribed (tau, p) per sample, or None

    @property
    def A(self):
        return self.A_full[self.act_idx][:, self.act_idx].tocsc()

    @property
    def b(self):
        return self.b_full[self.act_idx]


def sample_is_stress(grid):
    return np.concatenate([np.full(grid.size(st), name != "p") for name, st in grid.samples])


def _concat(grid, per_stagger, which, staggers):
    return np.concatenate([grid.flat(per_stagger[s][which]) for s in staggers])


def compliance(grid, wl_s, wf_s, mu_s, active):
    """Dg = W_Ft W_Lt C on the active stress samples."""
    n = grid.n_samples()
    off = grid.sample_offsets()
    diag = np.zeros(n)
    rows, cols, vals = [], [], []
    for name, st in grid.samples:
        if name == "p":
            continue
        lo, hi = off[name]
        sl = slice(lo, hi)
        diag[sl] = wf_s[sl] * wl_s[sl] / mu_s[sl] * active[sl]
    if grid.dim == 3:
        lx, hx = off["txx"]
        ly, hy = off["tyy"]
        both = active[lx:hx] & active[ly:hy]
        c = 0.5 * wf_s[lx:hx] * wl_s[lx:hx] / mu_s[lx:hx] * both
        ix = np.arange(lx, hx)
        iy = np.arange(ly, hy)
        rows += [ix, iy]
        cols += [iy, ix]
        vals += [c, c]
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(diag)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def traction_samples(grid, case):
    """Prescribed boundary values (tau_BC, p_BC) in sample order (Section
    6.1), or None when the case prescribes none.  case["p_bc"]: cell array;
    case["tau_bc"]: the stress arrays in sample order after p (tau_xx, tau_xy
    in 2D; tau_xx, tau_yy, tau_xy, tau_xz, tau_yz in 3D), native shapes;
    either may be absent (zero)."""
    p_bc = case.get("p_bc")
    tau_bc = case.get("tau_bc")
    if p_bc is None and tau_bc is None:
        return None
    parts = []
    k = 0
    for name, st in grid.samples:
        if name == "p":
            src = p_bc
        else:
            src = None if tau_bc is None else tau_bc[k]
            k += 1
        parts.append(np.zeros(grid.size(st)) if src is None else grid.flat(src))
    return np.concatenate(parts)


def assemble(case, dt=None, w_min=1e-3):
    """Steps (a1)-(a4): body force, weights, coefficients, null-space
    elimination, A and b.  ``case`` is a dict from the ``cases`` module."""
    grid = Grid(case["n"], case["h"], case.get("origin"))
    dt = float(case["dt"] if dt is None else dt)
    d = grid.dim
    W = sample_weights(grid, case["phi_l"], case.get("phi_s"), w_min)
    sample_st = [s for _, s in grid.samples]
    wl_s = _concat(grid, W, 0, sample_st)
    wf_s = _concat(grid, W, 1, sample_st)
    wl_f = _concat(grid, W, 0, grid.faces)
    wf_f = _concat(grid, W, 1, grid.faces)

    rho_f = np.concatenate([grid.flat(cell_mean_at(grid, case["rho"], fs)) for fs in grid.faces])
    mu_s = np.concatenate([grid.flat(cell_mean_at(grid, case["mu"], st)) if name != "p"
                           else np.full(grid.size(st), np.nan) for name, st in grid.samples])

    B0 = build_b0(grid)
    S = (abs(B0) > 0).astype(np.float64).tocsr()
    # solid side of the null-space rule: a fluid face whose stencil holds a
    # sample of zero fluid weight is invalid and keeps its boundary value;
    # from here on it is treated exactly like a solid face (W_F := 0)
    invalid = (wf_f > 0.0) & ((S @ (wf_s == 0.0).astype(np.float64)) > 0)
    wf_f = np.where(invalid, 0.0, wf_f)

    kpos = (wf_f > 0.0) & (wl_f > 0.0)
    bad = (wf_f > 0.0) & (wl_f == 0.0)
    K = np.zeros_like(wf_f)
    K[kpos] = wf_f[kpos] / (rho_f[kpos] * wl_f[kpos])

    St = S.T.tocsr()
    touches_bad = (St @ bad.astype(np.float64)) > 0
    touches_k = (St @ kpos.astype(np.float64)) > 0
    # free-surface side: a sample of positive liquid weight that touches a
    # face of zero liquid weight (but positive fluid weight) is invalid;
    # a sample with no face of K > 0 in its stencil has an empty row
    active = (wl_s > 0.0) & ~touches_bad & touches_k

    a = wl_s * active
    B = (B0 @ sp.diags(a)).tocsr()
    Dg = compliance(grid, wl_s, wf_s, mu_s, active)
    A_full = (dt * (B.T @ sp.diags(K) @ B) + Dg).tocsr()

    u_star_in = body_force(case["u"], case["g"], dt)
    us = np.concatenate([grid.flat(q) for q in u_star_in])
    y_bc = traction_samples(grid, case)
    if y_bc is not None:
        f = B0 @ (a * y_bc) - wl_f * (B0 @ y_bc)
        us = us.copy()
        us[kpos] += dt * f[kpos] / (rho_f[kpos] * wl_f[kpos])
    u_star = split_faces(grid, us)
    if case.get("u_bc") is not None:
        ubc = np.concatenate([grid.flat(q) for q in case["u_bc"]])
    else:
        ubc = np.zeros(grid.n_faces())
    # box walls are static: no prescribed motion on box faces
    for fa, (lo, hi) in enumerate(grid.face_offsets()):
        fi = grid.index(grid.faces[fa])
        edge = np.zeros(grid.shape(grid.faces[fa]), dtype=bool)
        idx = [slice(None)] * d
        idx[fa] = 0
        edge[tuple(idx)] = True
        idx[fa] = -1
        edge[tuple(idx)] = True
        ubc[lo + fi[edge]] = 0.0
    ws_f = 1.0 - wf_f
    ws_s = 1.0 - wf_s
    b_full = a * (B0.T @ (wf_f * us + ws_f * ubc) - ws_s * (B0.T @ ubc))
    if y_bc is not None:
        # eliminated samples hold their boundary value: in 3D the compliance
        # couples a cell's tau_xx and tau_yy, so a fixed one moves its
        # coupling term to the right-hand side of the other
        fixed = y_bc * (~active)
        coupling = compliance(grid, wl_s, wf_s, mu_s, np.ones(grid.n_samples(), dtype=bool))
        b_full = b_full - active * (coupling @ fixed)

    asm = Assembly(grid=grid, dt=dt, W=W, wl_s=wl_s, wf_s=wf_s, wl_f=wl_f, wf_f=wf_f,
                   rho_f=rho_f, mu_s=mu_s, K=K, bad=bad, invalid=invalid, active=active, B0=B0, B=B,
                   Dg=Dg, A_full=A_full, b_full=b_full, u_star=u_star, u_bc=ubc,
                   u_star_in=u_star_in, y_bc=y_bc)
    asm.act_idx = np.flatnonzero(active)
    return asm


# ---------------------------------------------------------------------------
# solves and velocity recovery
# ---------------------------------------------------------------------------
def pressure_null_vector(asm):
    """Constant pressure on the active p samples (zero stress): the rank-1
    null vector of enclosed domains (Section 8, last paragraph)."""
    lo, hi = asm.grid.sample_offsets()["p"]
    c = np.zeros(asm.grid.n_samples())
    c[lo:hi] = 1.0
    c = c * asm.active
    return c[asm.act_idx]


def is_enclosed(asm, rtol=1e-12):
    A = asm.A
    c = pressure_null_vector(asm)
    if not c.any():
        return False
    r = A @ c
    scale = abs(A).sum(axis=1).max() * np.abs(c).max()
    return np.abs(r).max() <= rtol * scale


def solve_direct(asm):
    """Sparse direct solve of A x = b.  If the pressure is only determined up
    to a constant, the first active pressure is fixed to 0."""
    A = asm.A
    b = asm.b
    n = A.shape[0]
    x = np.zeros(n)
    keep = np.ones(n, dtype=bool)
    if n == 0:
        return np.zeros(asm.grid.n_samples())
    if is_enclosed(asm):
        keep[np.flatnonzero(pressure_null_vector(asm))[0]] = False
    Ak = A[keep][:, keep].tocsc()
    lu = spla.splu(Ak, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    x[keep] = lu.solve(b[keep])
    full = np.zeros(asm.grid.n_samples())
    full[asm.act_idx] = x
    return full


def recover_velocity(asm, x_full):
    """(a8) u = u* - dt (B x)/(rho W_L) where K > 0; u_BC where W_F = 0;
    0 on the remaining (air / eliminated) faces."""
    us = np.concatenate([asm.grid.flat(q) for q in asm.u_star])
    Bx = asm.B @ x_full
    kpos = asm.K > 0.0
    u = np.zeros_like(us)
    u[kpos] = us[kpos] - asm.dt * Bx[kpos] / (asm.rho_f[kpos] * asm.wl_f[kpos])
    solid = asm.wf_f == 0.0
    u[solid] = asm.u_bc[solid]
    return u


def split_faces(grid, vec):
    return [grid.unflat(vec[lo:hi], grid.faces[a]) for a, (lo, hi) in enumerate(grid.face_offsets())]


def split_samples(grid, vec):
    off = grid.sample_offsets()
    return {name: grid.unflat(vec[off[name][0]:off[name][1]], st) for name, st in grid.samples}


def step(case, dt=None, w_min=1e-3):
    """One full step with a direct solve: returns (assembly, x, u_faces)."""
    asm = assemble(case, dt, w_min)
    x = solve_direct(asm)
    u = recover_velocity(asm, x)
    return asm, x, u


def apply(asm, x_full):
    """y = A x on the full sample vector (inactive entries ignored, output 0)."""
    return asm.A_full @ (x_full * asm.active)


def true_relative_residual(asm, x_full):
    r = asm.b_full - apply(asm, x_full)
    nb = np.linalg.norm(asm.b_full)
    return np.linalg.norm(r[asm.active]) / nb if nb > 0 else np.linalg.norm(r[asm.active])


# ---------------------------------------------------------------------------
# the full (u, tau, p) KKT system, for tiny cross-checks
# ---------------------------------------------------------------------------
def kkt_dense(asm):
    """Dense KKT of eq. stokesmixedsystem (reduced stresses, scaled by 1/dt),
    restricted to faces with K > 0 and active samples:

      [ P W_F W_L / dt    W_F B  ] [u]   [ P W_F W_L u*/dt + W_F ... ]
      [ B^T W_F          -Dg     ] [x] = [ rhs of the constraint rows ]

    The prescribed-velocity terms of Section 6.2 enter the right-hand side
    of the stress/pressure rows; the velocity rows are unchanged.  Returns
    (matrix, rhs, face index, sample index)."""
    grid = asm.grid
    fidx = np.flatnonzero(asm.K > 0.0)
    sidx = asm.act_idx
    B = asm.B.toarray()[np.ix_(fidx, sidx)]
    wf = asm.wf_f[fidx]
    wl = asm.wl_f[fidx]
    m = asm.rho_f[fidx] * wf * wl / asm.dt
    Dg = asm.Dg.toarray()[np.ix_(sidx, sidx)]
    nf, ns = len(fidx), len(sidx)
    M = np.zeros((nf + ns, nf + ns))
    M[:nf, :nf] = np.diag(m)
    M[:nf, nf:] = wf[:, None] * B
    M[nf:, :nf] = (wf[:, None] * B).T
    M[nf:, nf:] = -Dg
    us = np.concatenate([grid.flat(q) for q in asm.u_star_in])
    rhs = np.zeros(nf + ns)
    rhs[:nf] = m * us[fidx]
    # constraint rows: B^T W_F u = -(B^T W_S u_BC - W_L W_S B0^T u_BC) on active rows
    a = asm.wl_s * asm.active
    ws_f = 1.0 - asm.wf_f
    ws_s = 1.0 - asm.wf_s
    corr = a * (asm.B0.T @ (ws_f * asm.u_bc) - ws_s * (asm.B0.T @ asm.u_bc))
    if asm.y_bc is not None:
        # Section 6.1's air-region work terms and the boundary values of the
        # eliminated samples, on the velocity rows (sign as read in the header)
        y = asm.y_bc
        wa_f = 1.0 - asm.wl_f
        wa_s = 1.0 - asm.wl_s
        fixed = asm.wl_s * (~asm.active) * y
        t = wa_f * (asm.B0 @ y) - asm.B0 @ (wa_s * y) - asm.B0 @ fixed
        rhs[:nf] += (asm.wf_f * t)[fidx]
        # a fixed sample's compliance coupling (3D tau_xx / tau_yy) on the
        # stress rows
        coupling = compliance(grid, asm.wl_s, asm.wf_s, asm.mu_s,
                              np.ones(grid.n_samples(), dtype=bool))
        corr = corr - coupling @ (y * (~asm.active))
    rhs[nf:] = -corr[sidx]
    return M, rhs, fidx, sidx
