"""Training data and training loop of the learned preconditioner.

Pairs (r, e) come from the method's own solves.  For an assembled 3D
problem with right-hand side b and solution x* (FP64 Jacobi PCG to a tight
tolerance), the iterate x_k after k PCG iterations gives the residual
r_k = b - A x_k and the exact correction e_k = x* - x_k (A e_k = r_k), so a
solve yields residuals of every roughness the preconditioner meets, from the
smooth right-hand side (k = 0) to the rough late residuals.

Training minimises the mean over pairs of
    L(f) = 1 - (f.r)^2 / ((f.A f)(e.r)),   f = network correction of r,
the A-norm error left after an exact line search along f, relative to that
of the exact correction (see vfs_unet_train_step in include/vfstokes.h).
Every numerical step (assembly, solves, the network's forward and backward
passes, the loss gradient and Adam) runs in the HIP library; this module only
orchestrates calls through the C ABI.
"""
from __future__ import annotations

import numpy as np

from . import vfstokes as V

# layer table of the network (Cin, Cout), in the order of the weight vector
LAYERS = ((16, 16), (16, 32), (32, 64), (64, 128), (128, 64), (64, 32), (32, 16), (16, 6))


def he_init(seed, last_scale=0.1):
    """He-normal weights (std sqrt(2 / (27 Cin))), the output layer scaled by
    last_scale; float32, layout of vfs_unet_set_weights."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (ci, co) in enumerate(LAYERS):
        std = np.sqrt(2.0 / (27 * ci)) * (last_scale if li == len(LAYERS) - 1 else 1.0)
        parts.append(rng.normal(0.0, std, size=co * ci * 27))
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == V.vfs_unet_param_count()
    return w


def make_pairs(ctx, dt, ks, tol=1e-10, max_iter=200000, device=None):
    """Residual/correction pairs of one problem: x* from an FP64 Jacobi-PCG
    solve to tol, then for each k in ks the iterate x_k of a k-iteration
    solve (x_0 = 0).  Returns a list of (r_k, e_k) in sample order (NumPy
    float64, or torch float64 tensors on `device`).  The context's solver
    settings are restored afterwards."""
    saved = getattr(ctx, "_solver", None)
    w_min = saved[4] if saved is not None else 1e-3
    ctx.vfs_set_solver(V.VFS_PRECOND_JACOBI, V.VFS_FP64, tol, max_iter, w_min)
    ctx.vfs_assemble(dt)
    b = ctx.vfs_get_rhs()
    xs = ctx.vfs_solve(b)
    pairs = []
    for k in ks:
        if k <= 0:
            xk = np.zeros_like(xs)
        else:
            ctx.vfs_set_solver(V.VFS_PRECOND_JACOBI, V.VFS_FP64, 1e-14, int(k), w_min)
            xk = ctx.vfs_solve(b, allow_unconverged=True)
        pairs.append(ctx.vfs_training_pair(xs, xk))
    if saved is not None:
        ctx.vfs_set_solver(*saved)
    if device is not None:
        import torch
        pairs = [(torch.from_numpy(r).to(device), torch.from_numpy(e).to(device)) for r, e in pairs]
    return pairs


def train(net, problems, steps, lr=1e-3, batch=4, seed=0, lr_final=None, log_every=0, log=print):
    """Adam on the mean loss of `batch` random pairs per step.  problems: list
    of (ctx, pairs), each ctx assembled and attached to nothing else that
    would re-assemble it meanwhile.  The learning rate decays geometrically
    to lr_final (default lr) over the steps.  Returns the per-step mean
    losses."""
    rng = np.random.default_rng(seed)
    index = [(p, q) for p, (_, pairs) in enumerate(problems) for q in range(len(pairs))]
    lr_final = lr if lr_final is None else lr_final
    hist = []
    for step in range(steps):
        rate = lr * (lr_final / lr) ** (step / max(1, steps - 1))
        losses = []
        pick = rng.choice(len(index), size=min(batch, len(index)), replace=False)
        for t in pick:
            p, q = index[t]
            ctx, pairs = problems[p]
            r, e = pairs[q]
            losses.append(net.vfs_unet_train_step(ctx, r, e))
        net.vfs_unet_adam(rate, grad_scale=1.0 / len(pick))
        hist.append(float(np.mean(losses)))
        if log_every and (step % log_every == 0 or step == steps - 1):
            log(f"step {step:5d} lr {rate:.2e} loss {hist[-1]:.4f}")
    return hist
