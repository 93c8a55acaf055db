"""Learned preconditioner and flexible CG: plain CPU definitions (test
infrastructure only; the product path never imports this module).

The paper solves its SPD system with CG and an algebraic overlapping
multiplicative Schwarz preconditioner (Section 7 end, Section 9).  The
learned preconditioner is an addition to the method, not part of the paper;
each piece below is written from its published definition:

* U-Net style encoder/decoder (Ronneberger, Fischer and Brox 2015) on a
  cell-indexed 3D tensor, 3x3x3 convolutions, ReLU, 2x2x2 average pooling,
  nearest-neighbour upsampling and additive skips, no biases (so the network
  is positively homogeneous of degree one).
* Its gradient by the chain rule (reverse mode), written out layer by layer.
* Training loss: the A-norm error left after one exactly line-searched step
  along the network's direction f, relative to the A-norm error of doing
  nothing:  L(f) = 1 - (f.r)^2 / ((f.A f)(e.r)),  with A e = r.
  This is the quantity conjugate-gradient type methods reduce per step, it
  lies in [0, 1], is invariant to the scale of f and is 0 iff f is parallel
  to e.  Its gradient is  dL/df = (2a / (b E)) ((a / b) A f - r)  with
  a = f.r, b = f.A f, E = e.r.
* Adam (Kingma and Ba 2015) with bias correction.
* The preconditioner is a two-level step in the manner of multigrid: a
  Jacobi step with exact line search, d = D^-1 r, a1 = r.d / d.A d,
  smooths the residual to r1 = r - a1 A d; the network maps r1 to a
  direction n, used with an exact line search w = n.r1 / n.A n; the result
  is z = a1 d + w n.  The line searches make the step independent of the
  network's output scale, and the network only has to supply the smooth
  part of the error that the Jacobi step leaves.  Training pairs are
  transformed the same way: (r, e) -> (r1, e1 = e - a1 d), A e1 = r1.
* Flexible CG with the Polak-Ribiere form of beta (Golub and Ye 1999;
  Notay 2000), so that a non-linear preconditioner can be used; a direction
  that is not a descent direction (z.r <= 0 or not finite) is replaced by
  the Jacobi one.  Its truncated form (Notay 2000) makes each new direction
  A-orthogonal to the m previous ones instead of one, which keeps most of
  CG's acceleration when the preconditioner varies from step to step.

Everything is FP64.  ``bf16=True`` rounds to bfloat16 (round to nearest,
ties to even) exactly where the GPU path stores bfloat16: the input tensor,
the weights, every activation and every back-propagated activation
gradient; accumulations stay wide.

Tensor convention: channels last, shape (Z, Y, X, C), voxel (x, y, z) =
sample index (i, j, k) of every sample set (cell, face and edge samples
that share an index share a voxel).  Tensor extents are
roundup(n_axis + 1, 8) so that every sample of every set has a voxel and
three 2x2x2 poolings divide evenly.
Weights of a layer: shape (Cout, Cin, 3, 3, 3) indexed [co, ci, dz, dy, dx];
out[z, y, x, co] = sum_{ci, dz, dy, dx} W[co, ci, dz, dy, dx]
                   * in[z + dz - 1, y + dy - 1, x + dx - 1, ci]
(zero outside the tensor).  The flat parameter vector concatenates the
layers in LAYERS order, each in this (co, ci, dz, dy, dx) C order.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

# (name, cin, cout, level, relu).  Encoder: one conv per level, pooled input;
# bottleneck at level 3; decoder: upsampled coarser result plus the encoder
# activation of the same level (additive skip), one conv each.
LAYERS = (
    ("enc0", 16, 16, 0, True),
    ("enc1", 16, 32, 1, True),
    ("enc2", 32, 64, 2, True),
    ("enc3", 64, 128, 3, True),
    ("bott", 128, 64, 3, True),
    ("dec2", 64, 32, 2, True),
    ("dec1", 32, 16, 1, True),
    ("dec0", 16, 6, 0, False),
)
N_IN = 16          # input channels: 6 residual sets, 2 zero, 3 geometry, 5 zero
N_OUT = 6          # one correction channel per 3D sample set
GEOM = (8, 9, 10)  # W_L(cell), W_F(cell), log10(1 + dt mu / (rho h^2)) / 6


def layer_sizes():
    return [co * ci * 27 for (_, ci, co, _, _) in LAYERS]


def param_count():
    return int(sum(layer_sizes()))


def split_params(theta):
    """Flat parameter vector -> list of (Cout, Cin, 3, 3, 3) weight arrays."""
    out, o = [], 0
    for (_, ci, co, _, _), sz in zip(LAYERS, layer_sizes()):
        out.append(np.asarray(theta[o:o + sz], dtype=np.float64).reshape(co, ci, 3, 3, 3))
        o += sz
    return out


def tensor_dims(n):
    """(Z, Y, X) extents of the cell-indexed tensor of a grid of n cells."""
    r = lambda a: ((int(a) + 1 + 7) // 8) * 8
    return (r(n[2]), r(n[1]), r(n[0]))


# ---------------------------------------------------------------- rounding
def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    The FP64 value is first rounded to FP32 (the GPU rounds its FP32
    accumulators), then the low 16 bits of the FP32 pattern are rounded
    away.  NaN stays NaN."""
    a = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(a), np.nan, out)


def _rnd(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


# ------------------------------------------------------------- primitives
def _t(x):
    """(Z, Y, X, C) numpy -> (1, C, Z, Y, X) torch float64."""
    return torch.from_numpy(np.ascontiguousarray(np.moveaxis(x, -1, 0)))[None]


def _n(t):
    return np.ascontiguousarray(np.moveaxis(t[0].numpy(), 0, -1))


def conv3(x, w):
    """3x3x3 cross-correlation with zero padding 1 (same extents)."""
    return _n(F.conv3d(_t(x), torch.from_numpy(np.ascontiguousarray(w)), padding=1))


def conv3_input_grad(g, w):
    """Adjoint of conv3 with respect to its input."""
    return _n(F.conv_transpose3d(_t(g), torch.from_numpy(np.ascontiguousarray(w)), padding=1))


def conv3_weight_grad(x, g):
    """Adjoint of conv3 with respect to its weights: sum over voxels of
    g[v, co] * x[v + offset, ci]."""
    xt = _t(x)
    gt = _t(g)
    # correlate the input with the output gradient: batch <- ci, channels <- co
    wg = F.conv3d(xt.transpose(0, 1), gt.transpose(0, 1), padding=1)
    return wg.transpose(0, 1).numpy().copy()


def pool2(x):
    """2x2x2 mean."""
    Z, Y, X, C = x.shape
    return x.reshape(Z // 2, 2, Y // 2, 2, X // 2, 2, C).mean(axis=(1, 3, 5))


def up2(x):
    """Nearest-neighbour upsampling by 2 along each axis."""
    return x.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def sum2(x):
    """2x2x2 sum (adjoint of up2)."""
    Z, Y, X, C = x.shape
    return x.reshape(Z // 2, 2, Y // 2, 2, X // 2, 2, C).sum(axis=(1, 3, 5))


# ---------------------------------------------------------------- network
def forward(theta, x, bf16_mode=False):
    """Network output y (Z, Y, X, 6) and the activations kept for the
    gradient.  With bf16_mode the stored tensors are rounded to bfloat16."""
    r = lambda a: _rnd(a, bf16_mode)
    W = [r(w) for w in split_params(theta)]
    x = r(x)
    relu = lambda a: np.maximum(a, 0.0)
    c0 = r(relu(conv3(x, W[0])))
    p0 = r(pool2(c0))
    c1 = r(relu(conv3(p0, W[1])))
    p1 = r(pool2(c1))
    c2 = r(relu(conv3(p1, W[2])))
    p2 = r(pool2(c2))
    c3 = r(relu(conv3(p2, W[3])))
    d3 = r(relu(conv3(c3, W[4])))
    s2 = r(up2(d3) + c2)
    d2 = r(relu(conv3(s2, W[5])))
    s1 = r(up2(d2) + c1)
    d1 = r(relu(conv3(s1, W[6])))
    s0 = r(up2(d1) + c0)
    y = conv3(s0, W[7])                     # FP32 output on the GPU, not rounded
    cache = dict(W=W, x=x, c0=c0, p0=p0, c1=c1, p1=p1, c2=c2, p2=p2, c3=c3, d3=d3,
                 s2=s2, d2=d2, s1=s1, d1=d1, s0=s0)
    return y, cache


def backward(cache, gy, bf16_mode=False):
    """Gradient of <gy, y> with respect to the flat parameter vector, by the
    chain rule through forward(); activation gradients are rounded to
    bfloat16 where the GPU stores them, weight gradients stay wide."""
    r = lambda a: _rnd(a, bf16_mode)
    c = cache
    W = c["W"]
    mask = lambda a: (a > 0.0).astype(np.float64)
    gy = r(gy)
    gW = [None] * 8
    gW[7] = conv3_weight_grad(c["s0"], gy)
    g_s0 = r(conv3_input_grad(gy, W[7]))
    g_d1 = r(sum2(g_s0) * mask(c["d1"]))           # through up2 and d1's ReLU
    gW[6] = conv3_weight_grad(c["s1"], g_d1)
    g_s1 = r(conv3_input_grad(g_d1, W[6]))
    g_d2 = r(sum2(g_s1) * mask(c["d2"]))
    gW[5] = conv3_weight_grad(c["s2"], g_d2)
    g_s2 = r(conv3_input_grad(g_d2, W[5]))
    g_d3 = r(sum2(g_s2) * mask(c["d3"]))
    gW[4] = conv3_weight_grad(c["c3"], g_d3)
    g_c3 = r(conv3_input_grad(g_d3, W[4]) * mask(c["c3"]))
    gW[3] = conv3_weight_grad(c["p2"], g_c3)
    g_p2 = r(conv3_input_grad(g_c3, W[3]))
    # c2 feeds the pooled path (mean: gradient / 8 on each child) and the skip
    g_c2 = r((g_s2 + up2(g_p2) / 8.0) * mask(c["c2"]))
    gW[2] = conv3_weight_grad(c["p1"], g_c2)
    g_p1 = r(conv3_input_grad(g_c2, W[2]))
    g_c1 = r((g_s1 + up2(g_p1) / 8.0) * mask(c["c1"]))
    gW[1] = conv3_weight_grad(c["p0"], g_c1)
    g_p0 = r(conv3_input_grad(g_c1, W[1]))
    g_c0 = r((g_s0 + up2(g_p0) / 8.0) * mask(c["c0"]))
    gW[0] = conv3_weight_grad(c["x"], g_c0)
    return np.concatenate([g.ravel() for g in gW])


# ------------------------------------------------ samples <-> tensor (3D)
def _set_blocks(grid):
    """(offset, shape) of each sample set in the sample-order vector."""
    offs = grid.sample_offsets()
    return [(offs[name][0], grid.shape(st)) for name, st in grid.samples]


def geometry_channels(asm, case):
    """W_L and W_F of the cell samples and log10(1 + dt mu / (rho h^2)) / 6 at
    cells, as (nx, ny, nz) arrays."""
    g = asm.grid
    ncell = g.size(g.cell)
    wl = g.unflat(asm.wl_s[:ncell], g.cell)
    wf = g.unflat(asm.wf_s[:ncell], g.cell)
    mu = np.asarray(case["mu"], dtype=np.float64)
    rho = np.asarray(case["rho"], dtype=np.float64)
    lam = np.log10(1.0 + asm.dt * mu / (rho * g.h * g.h)) / 6.0
    return wl, wf, lam


def pack_input(asm, case, r_full, dinv_full):
    """Network input (Z, Y, X, 16) of a residual r (sample order, FP64) and
    the scale s: channel q at voxel (i, j, k) is s * sqrt(D^-1) r of set q's
    sample (i, j, k) (0 for inactive samples), with s = sqrt(n_active) /
    ||sqrt(D^-1) r|| (0 if that norm is 0); channels 8-10 hold geometry."""
    g = asm.grid
    Z, Y, X = tensor_dims(g.n)
    act = asm.active.astype(np.float64)
    rh = np.where(act > 0, np.asarray(r_full) * np.sqrt(np.maximum(dinv_full, 0.0)), 0.0)
    nrm = np.linalg.norm(rh)
    s = np.sqrt(act.sum()) / nrm if nrm > 0 else 0.0
    x = np.zeros((Z, Y, X, N_IN))
    for q, (o, shp) in enumerate(_set_blocks(g)):
        blk = (s * rh[o:o + int(np.prod(shp))]).reshape(shp, order="F")   # [i, j, k]
        x[:shp[2], :shp[1], :shp[0], q] = blk.transpose(2, 1, 0)
    wl, wf, lam = geometry_channels(asm, case)
    n = g.n
    for ch, arr in zip(GEOM, (wl, wf, lam)):
        x[:n[2], :n[1], :n[0], ch] = arr.transpose(2, 1, 0)
    return x, s


def unpack_output(asm, y, dinv_full, s):
    """Correction f (sample order) of a network output y: sqrt(D^-1) y / s
    on active samples, 0 elsewhere (0 everywhere when s = 0)."""
    g = asm.grid
    f = np.zeros(g.n_samples())
    if s == 0.0:
        return f
    for q, (o, shp) in enumerate(_set_blocks(g)):
        blk = y[:shp[2], :shp[1], :shp[0], q].transpose(2, 1, 0)
        f[o:o + int(np.prod(shp))] = blk.ravel(order="F")
    return np.where(asm.active, f * np.sqrt(np.maximum(dinv_full, 0.0)) / s, 0.0)


def unpack_adjoint(asm, g_f, dinv_full, s, dims):
    """Adjoint of unpack_output: the gradient with respect to y of a
    function of f, given its gradient g_f (sample order)."""
    g = asm.grid
    Z, Y, X = dims
    gy = np.zeros((Z, Y, X, N_OUT))
    if s == 0.0:
        return gy
    gv = np.where(asm.active, np.asarray(g_f) * np.sqrt(np.maximum(dinv_full, 0.0)) / s, 0.0)
    for q, (o, shp) in enumerate(_set_blocks(g)):
        blk = gv[o:o + int(np.prod(shp))].reshape(shp, order="F")
        gy[:shp[2], :shp[1], :shp[0], q] = blk.transpose(2, 1, 0)
    return gy


# ------------------------------------------------------------------ loss
def loss_and_grad(apply_A, f, r, e):
    """L(f) = 1 - (f.r)^2 / ((f.A f)(e.r)) and dL/df (all sample order; apply_A
    is y = A x on the same vectors).  L is undefined where f.A f = 0 (f = 0
    on the active samples); there the function returns L = 1 and a zero
    gradient."""
    q = apply_A(f)
    a = float(f @ r)
    b = float(f @ q)
    E = float(e @ r)
    if b <= 0.0 or E <= 0.0:
        return 1.0, np.zeros_like(f)
    L = 1.0 - a * a / (b * E)
    g = (2.0 * a / (b * E)) * ((a / b) * q - r)
    return L, g


# ------------------------------------------------------- two-level step
def smooth(apply_A, dinv, r):
    """Jacobi step with exact line search: (a1, d, A d, r1 = r - a1 A d)."""
    d = dinv * r
    qd = apply_A(d)
    dq = float(d @ qd)
    a1 = float(r @ d) / dq if dq > 0.0 else 0.0
    return a1, d, qd, r - a1 * qd


def smooth_pair(apply_A, dinv, r, e):
    """Training pair after the Jacobi step: (r1, e1) with A e1 = r1."""
    a1, d, qd, r1 = smooth(apply_A, dinv, r)
    return r1, e - a1 * d


def two_level(apply_A, dinv, r, net):
    """z = a1 d + w n with n = net(r1) and w = n.r1 / n.A n (w = 0 when
    n.A n <= 0 or a value is not finite)."""
    a1, d, qd, r1 = smooth(apply_A, dinv, r)
    n = net(r1)
    qn = apply_A(n)
    nq = float(n @ qn)
    w = float(n @ r1) / nq if nq > 0.0 and np.isfinite(nq) else 0.0
    if not np.isfinite(w):
        w = 0.0
    return a1 * d + w * n


# ------------------------------------------------------------------ Adam
def adam_step(theta, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------ flexible CG
def fcg(apply_A, b, precond, dinv, tol=1e-6, max_iter=10000):
    """Flexible CG from x0 = 0: z = M(r) (Jacobi z = D^-1 r where M gives no
    descent direction), beta = z.(r - r_prev) / (z_prev.r_prev) (Polak-
    Ribiere), p = z + beta p, alpha = p.r / p.A p.  Stops when ||r|| <= tol
    ||b|| (recursive residual).  Returns (x, iterations, history of
    ||r|| / ||b||, number of Jacobi fallbacks)."""
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, [0.0], 0
    hist = [1.0]
    p = z_prev = r_prev = None
    k = fallbacks = 0
    while k < max_iter and hist[-1] > tol:
        z = precond(r)
        zr = float(z @ r)
        if not np.isfinite(zr) or zr <= 0.0 or not np.all(np.isfinite(z)):
            z = dinv * r
            fallbacks += 1
        if p is None:
            p = z.copy()
        else:
            beta = float(z @ (r - r_prev)) / float(z_prev @ r_prev)
            p = z + beta * p
        q = apply_A(p)
        alpha = float(p @ r) / float(p @ q)
        x = x + alpha * p
        r_prev, z_prev = r, z
        r = r - alpha * q
        k += 1
        hist.append(np.linalg.norm(r) / nb)
    return x, k, hist, fallbacks


def fcg_truncated(apply_A, b, precond, dinv, m, tol=1e-6, max_iter=10000):
    """Truncated flexible CG from x0 = 0: p_k = z_k - sum over the m previous
    directions p_i of (z_k.A p_i / p_i.A p_i) p_i, alpha = p_k.r_k /
    p_k.A p_k; z_k = M(r_k), replaced by the Jacobi z when z_k.r_k <= 0 or
    not finite.  m = 1 is the Polak-Ribiere flexible CG of fcg().  Stops
    when ||r|| <= tol ||b||.  Returns (x, iterations, history, fallbacks)."""
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, [0.0], 0
    hist = [1.0]
    P, Q = [], []
    k = fallbacks = 0
    while k < max_iter and hist[-1] > tol:
        z = precond(r)
        zr = float(z @ r)
        if not np.isfinite(zr) or zr <= 0.0 or not np.all(np.isfinite(z)):
            z = dinv * r
            fallbacks += 1
        p = z.copy()
        for pi, qi in zip(P, Q):
            p = p - (float(z @ qi) / float(pi @ qi)) * pi
        q = apply_A(p)
        alpha = float(p @ r) / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        P.append(p)
        Q.append(q)
        if len(P) > m:
            P.pop(0)
            Q.pop(0)
        k += 1
        hist.append(np.linalg.norm(r) / nb)
    return x, k, hist, fallbacks

