"""Plain Jacobi-preconditioned conjugate gradients on the explicit sparse A.

The paper solves its SPD system with preconditioned CG (Section 7 end,
Section 9 first paragraph); the preconditioner here is the diagonal of A,
the simplest choice.  This is the CPU timing baseline and a second solver
to cross-check the direct solve; it is written as the textbook algorithm
with x0 = 0 and stops on the recursively updated residual
||r||_2 / ||b||_2 <= tol or after max_iter iterations.
"""
from __future__ import annotations

import numpy as np


def jacobi_pcg(A, b, tol=1e-10, max_iter=100000, x0=None):
    """Returns (x, iterations, history of ||r||/||b||)."""
    n = A.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    d = A.diagonal()
    dinv = np.where(d > 0.0, 1.0 / np.where(d > 0.0, d, 1.0), 0.0)
    r = b - A @ x
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, [0.0]
    z = dinv * r
    p = z.copy()
    rz = r @ z
    hist = [np.linalg.norm(r) / nb]
    it = 0
    while it < max_iter and hist[-1] > tol:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = dinv * r
        rz_new = r @ z
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
        it += 1
        hist.append(np.linalg.norm(r) / nb)
    return x, it, hist


def fixed_iterations(A, b, iters):
    """Exactly ``iters`` Jacobi-PCG iterations (no convergence test); used to
    time the CPU baseline in DOF-iterations per second."""
    n = A.shape[0]
    x = np.zeros(n)
    d = A.diagonal()
    dinv = np.where(d > 0.0, 1.0 / np.where(d > 0.0, d, 1.0), 0.0)
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    for _ in range(iters):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x
