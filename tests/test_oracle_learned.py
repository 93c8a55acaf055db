"""Pins of the learned-preconditioner oracle (oracle/learned.py) against facts
fixed by mathematics, not by the oracle's own formulas: brute-force
convolution, adjoint identities, finite differences, exact reductions of
flexible CG to plain PCG and to a direct solve, closed forms of Adam and of
the loss, and bfloat16 rounding of hand-checked bit patterns."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import cases
from oracle import cg, learned, system


# ------------------------------------------------------------------ bf16
def test_bf16_rounding_bit_patterns():
    b = learned.bf16
    # representable values are unchanged
    for v in (1.0, -2.0, 0.5, 1.0 + 2.0 ** -7, 3.0 * 2.0 ** -130, 0.0):
        assert b(v) == v
    # ties go to the even neighbour
    assert b(1.0 + 2.0 ** -8) == 1.0
    assert b(1.0 + 3.0 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    # above the tie rounds up, below rounds down
    assert b(1.0 + 2.0 ** -8 + 2.0 ** -12) == 1.0 + 2.0 ** -7
    assert b(1.0 + 2.0 ** -8 - 2.0 ** -12) == 1.0
    assert b(-(1.0 + 2.0 ** -8 + 2.0 ** -12)) == -(1.0 + 2.0 ** -7)
    assert np.isnan(b(np.nan)) and b(np.inf) == np.inf
    # unit roundoff of an 8-bit significand: relative error <= 2^-8
    x = np.random.default_rng(0).normal(size=10000) * 10.0 ** np.random.default_rng(1).uniform(-5, 5, 10000)
    assert np.all(np.abs(b(x) - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-12))


# ------------------------------------------------------------ primitives
def test_conv3_matches_brute_force_loops():
    rng = np.random.default_rng(2)
    Z, Y, X, ci, co = 3, 4, 5, 2, 3
    x = rng.normal(size=(Z, Y, X, ci))
    w = rng.normal(size=(co, ci, 3, 3, 3))
    ref = np.zeros((Z, Y, X, co))
    for z in range(Z):
        for y in range(Y):
            for xx in range(X):
                for o in range(co):
                    s = 0.0
                    for c in range(ci):
                        for dz in range(3):
                            for dy in range(3):
                                for dx in range(3):
                                    zz, yy, x2 = z + dz - 1, y + dy - 1, xx + dx - 1
                                    if 0 <= zz < Z and 0 <= yy < Y and 0 <= x2 < X:
                                        s += w[o, c, dz, dy, dx] * x[zz, yy, x2, c]
                    ref[z, y, xx, o] = s
    assert np.allclose(learned.conv3(x, w), ref, rtol=0, atol=1e-12)


def test_conv3_adjoints():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(4, 6, 8, 3))
    w = rng.normal(size=(5, 3, 3, 3, 3))
    g = rng.normal(size=(4, 6, 8, 5))
    lhs = np.sum(learned.conv3(x, w) * g)
    assert np.isclose(lhs, np.sum(x * learned.conv3_input_grad(g, w)), rtol=1e-12)
    assert np.isclose(lhs, np.sum(w * learned.conv3_weight_grad(x, g)), rtol=1e-12)


def test_pool_up_sum_identities():
    rng = np.random.default_rng(4)
    a = rng.normal(size=(2, 3, 4, 5))
    b = rng.normal(size=(4, 6, 8, 5))
    assert np.allclose(learned.pool2(learned.up2(a)), a)
    assert np.isclose(np.sum(learned.up2(a) * b), np.sum(a * learned.sum2(b)), rtol=1e-12)
    assert np.allclose(learned.sum2(b), 8.0 * learned.pool2(b))
    assert learned.up2(a)[3, 5, 7, 2] == a[1, 2, 3, 2]


# ---------------------------------------------------------------- network
def _theta(seed, scale=1.0):
    """He-scaled random weights."""
    rng = np.random.default_rng(seed)
    ws = [rng.normal(size=sz) * scale * np.sqrt(2.0 / (ci * 27))
          for (_, ci, _, _, _), sz in zip(learned.LAYERS, learned.layer_sizes())]
    return np.concatenate(ws)


def test_param_count_and_layout():
    assert learned.param_count() == 27 * (16 * 16 + 16 * 32 + 32 * 64 + 64 * 128 + 128 * 64
                                          + 64 * 32 + 32 * 16 + 16 * 6)
    th = np.arange(learned.param_count(), dtype=np.float64)
    W = learned.split_params(th)
    assert W[0][0, 0, 0, 0, 1] == 1.0 and W[0][0, 1, 0, 0, 0] == 27.0 and W[0][1, 0, 0, 0, 0] == 27.0 * 16
    assert W[1][0, 0, 0, 0, 0] == 27.0 * 256


def test_network_is_positively_homogeneous():
    th = _theta(5)
    x = np.random.default_rng(6).normal(size=(16, 16, 16, 16))
    y1, _ = learned.forward(th, x)
    y2, _ = learned.forward(th, 3.5 * x)
    assert np.allclose(y2, 3.5 * y1, rtol=1e-12, atol=1e-12 * np.abs(y1).max())


def test_network_gradient_matches_finite_differences():
    """Directional derivative of <gy, y(theta)> along random directions,
    restricted to one layer at a time, against central differences."""
    rng = np.random.default_rng(7)
    th = _theta(8)
    x = rng.normal(size=(16, 16, 8, 16))
    gy = rng.normal(size=(16, 16, 8, 6))
    y, cache = learned.forward(th, x)
    grad = learned.backward(cache, gy)
    phi = lambda t: np.sum(learned.forward(t, x)[0] * gy)
    offs = np.cumsum([0] + learned.layer_sizes())
    for layer in range(8):
        d = np.zeros_like(th)
        d[offs[layer]:offs[layer + 1]] = rng.normal(size=offs[layer + 1] - offs[layer])
        eps = 1e-6
        fd = (phi(th + eps * d) - phi(th - eps * d)) / (2 * eps)
        an = float(grad @ d)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.abs(grad).max() * np.linalg.norm(d)), \
            (layer, fd, an)


def test_bf16_mode_is_close_to_fp64():
    rng = np.random.default_rng(9)
    th = _theta(10)
    x = rng.normal(size=(16, 8, 16, 16))
    y64, c64 = learned.forward(th, x)
    y16, c16 = learned.forward(th, x, bf16_mode=True)
    assert np.linalg.norm(y16 - y64) <= 0.03 * np.linalg.norm(y64)
    gy = rng.normal(size=y64.shape)
    g64 = learned.backward(c64, gy)
    g16 = learned.backward(c16, gy, bf16_mode=True)
    assert np.linalg.norm(g16 - g64) <= 0.05 * np.linalg.norm(g64)


# ------------------------------------------------ samples <-> tensor, loss
@pytest.fixture(scope="module")
def small3d():
    case = cases.pool3d(8, seed=11)
    asm = system.assemble(case)
    A = asm.A.tocsr()
    n = asm.grid.n_samples()
    idx = asm.act_idx
    dA = A.diagonal()
    dinv = np.zeros(n)
    dinv[idx] = 1.0 / dA
    lu = spla.splu(A.tocsc())

    def apply_full(v):
        out = np.zeros(n)
        out[idx] = A @ v[idx]
        return out

    def solve_full(v):
        out = np.zeros(n)
        out[idx] = lu.solve(v[idx])
        return out
    return case, asm, dinv, apply_full, solve_full


def test_pack_unpack_of_identity_network_is_jacobi(small3d):
    case, asm, dinv, apply_full, _ = small3d
    rng = np.random.default_rng(12)
    r = np.where(asm.active, rng.normal(size=asm.grid.n_samples()), 0.0)
    x, s = learned.pack_input(asm, case, r, dinv)
    assert x.shape == (16, 16, 16, 16)
    # the residual channels have unit RMS over active samples
    assert np.isclose(np.sum(x[..., :6] ** 2), asm.active.sum())
    f = learned.unpack_output(asm, x[..., :6], dinv, s)
    assert np.allclose(f, dinv * r, rtol=1e-12, atol=0)
    # geometry channels lie in [0, 1]; the unused channels are zero
    assert x[..., 8:11].min() >= 0.0 and x[..., 8:11].max() <= 1.0
    assert not x[..., 6:8].any() and not x[..., 11:].any()


def test_unpack_adjoint(small3d):
    case, asm, dinv, _, _ = small3d
    rng = np.random.default_rng(13)
    y = rng.normal(size=(16, 16, 16, 6))
    g = rng.normal(size=asm.grid.n_samples())
    s = 0.37
    lhs = np.sum(learned.unpack_output(asm, y, dinv, s) * g)
    rhs = np.sum(y * learned.unpack_adjoint(asm, g, dinv, s, (16, 16, 16)))
    assert np.isclose(lhs, rhs, rtol=1e-12)


def test_loss_closed_forms_and_gradient(small3d):
    case, asm, dinv, apply_full, solve_full = small3d
    rng = np.random.default_rng(14)
    r = np.where(asm.active, rng.normal(size=asm.grid.n_samples()), 0.0)
    e = solve_full(r)
    L, g = learned.loss_and_grad(apply_full, e, r, e)
    assert abs(L) < 1e-10 and np.abs(g).max() < 1e-8 * np.abs(r).max() / (e @ r) * 10
    L, _ = learned.loss_and_grad(apply_full, 2.5 * e, r, e)
    assert abs(L) < 1e-10
    # steepest descent (f = r): one exact line search along r
    rAr = r @ apply_full(r)
    L, _ = learned.loss_and_grad(apply_full, r, r, e)
    assert np.isclose(L, 1.0 - (r @ r) ** 2 / (rAr * (e @ r)), rtol=1e-12)
    # the loss of one exact step equals the remaining A-norm error fraction
    alpha = (r @ r) / rAr
    err = e - alpha * r
    assert np.isclose(L, (err @ apply_full(err)) / (e @ r), rtol=1e-10)
    # range and finite differences
    f = np.where(asm.active, rng.normal(size=r.size), 0.0)
    L, g = learned.loss_and_grad(apply_full, f, r, e)
    assert 0.0 <= L <= 1.0
    d = np.where(asm.active, rng.normal(size=r.size), 0.0)
    eps = 1e-6
    fd = (learned.loss_and_grad(apply_full, f + eps * d, r, e)[0]
          - learned.loss_and_grad(apply_full, f - eps * d, r, e)[0]) / (2 * eps)
    assert np.isclose(fd, g @ d, rtol=1e-6)
    # f = 0 on the active samples: defined as no progress
    L, g = learned.loss_and_grad(apply_full, np.zeros_like(r), r, e)
    assert L == 1.0 and not g.any()


def test_two_level_step_reductions(small3d):
    """With the exact coarse correction the two-level step is the exact
    inverse; with no network it is a multiple of the Jacobi direction; the
    smoothed pair keeps A e1 = r1 and the Jacobi step never increases the
    A-norm error."""
    case, asm, dinv, apply_full, solve_full = small3d
    rng = np.random.default_rng(15)
    r = np.where(asm.active, rng.normal(size=asm.grid.n_samples()), 0.0)
    e = solve_full(r)
    z = learned.two_level(apply_full, dinv, r, solve_full)
    assert np.linalg.norm(z - e) <= 1e-8 * np.linalg.norm(e)
    z0 = learned.two_level(apply_full, dinv, r, lambda v: np.zeros_like(v))
    a1 = (r @ (dinv * r)) / ((dinv * r) @ apply_full(dinv * r))
    assert np.allclose(z0, a1 * dinv * r, rtol=1e-12, atol=0)
    r1, e1 = learned.smooth_pair(apply_full, dinv, r, e)
    assert np.linalg.norm(apply_full(e1) - r1) <= 1e-8 * np.linalg.norm(r1)
    assert e1 @ r1 <= e @ r * (1 + 1e-12)
    # the network's output scale does not matter
    n = np.where(asm.active, rng.normal(size=r.size), 0.0)
    za = learned.two_level(apply_full, dinv, r, lambda v: n)
    zb = learned.two_level(apply_full, dinv, r, lambda v: -7.0 * n)
    assert np.allclose(za, zb, rtol=1e-10, atol=1e-12 * np.abs(za).max())


def test_fcg_with_exact_two_level_takes_one_iteration(small3d):
    case, asm, dinv, apply_full, solve_full = small3d
    bf = np.zeros(asm.grid.n_samples())
    bf[asm.act_idx] = asm.b
    pre = lambda r: learned.two_level(apply_full, dinv, r, solve_full)
    x, it, hist, fb = learned.fcg(apply_full, bf, pre, dinv, tol=1e-9)
    assert it == 1 and fb == 0


# ------------------------------------------------------------------- Adam
def test_adam_closed_form():
    g1 = np.array([0.3, -2.0, 1e-3, 0.0])
    g2 = np.array([-0.1, -2.0, 5e-3, 1.0])
    th = np.array([1.0, 2.0, 3.0, 4.0])
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    t1, m, v = learned.adam_step(th, 0 * th, 0 * th, g1, 1, lr, b1, b2, eps)
    # first step: the bias-corrected moments are g and g^2
    assert np.allclose(t1, th - lr * g1 / (np.abs(g1) + eps), rtol=0, atol=1e-15)
    t2, m, v = learned.adam_step(t1, m, v, g2, 2, lr, b1, b2, eps)
    mh = (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    vh = (b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    assert np.allclose(t2, t1 - lr * mh / (np.sqrt(vh) + eps), rtol=0, atol=1e-15)


# ------------------------------------------------------------- flexible CG
def test_fcg_with_jacobi_is_jacobi_pcg(small3d):
    case, asm, dinv, apply_full, _ = small3d
    A = asm.A.tocsr()
    b = asm.b
    x_ref, it_ref, hist_ref = cg.jacobi_pcg(A, b, tol=1e-10)
    bf = np.zeros(asm.grid.n_samples())
    bf[asm.act_idx] = b
    x, it, hist, fb = learned.fcg(apply_full, bf, lambda r: dinv * r, dinv, tol=1e-10)
    assert fb == 0
    assert abs(it - it_ref) <= 1
    assert np.linalg.norm(x[asm.act_idx] - x_ref) <= 1e-8 * np.linalg.norm(x_ref)
    # identical residual histories over the first iterations (rounding aside)
    k = min(20, it, it_ref)
    assert np.allclose(hist[:k], hist_ref[:k], rtol=1e-6)


def test_fcg_with_exact_inverse_takes_one_iteration(small3d):
    case, asm, dinv, apply_full, solve_full = small3d
    bf = np.zeros(asm.grid.n_samples())
    bf[asm.act_idx] = asm.b
    x, it, hist, fb = learned.fcg(apply_full, bf, solve_full, dinv, tol=1e-9)
    assert it == 1 and fb == 0
    assert hist[-1] < 1e-9


def test_fcg_replaces_non_descent_directions_by_jacobi(small3d):
    case, asm, dinv, apply_full, _ = small3d
    bf = np.zeros(asm.grid.n_samples())
    bf[asm.act_idx] = asm.b
    x1, it1, _, fb1 = learned.fcg(apply_full, bf, lambda r: -r, dinv, tol=1e-8)
    x2, it2, _, fb2 = learned.fcg(apply_full, bf, lambda r: dinv * r, dinv, tol=1e-8)
    assert fb1 == it1 and fb2 == 0 and it1 == it2
    assert np.allclose(x1, x2)


def test_truncated_fcg_reductions(small3d):
    """m = 1 is the Polak-Ribiere flexible CG; with a fixed SPD preconditioner
    the extra orthogonalisations vanish and every m gives PCG; with the exact
    inverse one iteration suffices."""
    case, asm, dinv, apply_full, solve_full = small3d
    bf = np.zeros(asm.grid.n_samples())
    bf[asm.act_idx] = asm.b
    rng = np.random.default_rng(16)
    n = np.where(asm.active, rng.normal(size=bf.size), 0.0)
    # a non-linear preconditioner: the two-level step with a fixed "network"
    pre = lambda r: learned.two_level(apply_full, dinv, r, lambda v: n * np.sign(v @ n + 1e-300))
    x1, k1, h1, _ = learned.fcg(apply_full, bf, pre, dinv, tol=1e-8, max_iter=200)
    x2, k2, h2, _ = learned.fcg_truncated(apply_full, bf, pre, dinv, 1, tol=1e-8, max_iter=200)
    kk = min(30, k1, k2)
    assert np.allclose(h1[:kk], h2[:kk], rtol=1e-6)
    jac = lambda r: dinv * r
    _, kj, hj = cg.jacobi_pcg(asm.A.tocsr(), asm.b, tol=1e-8)
    for m in (1, 3, 8):
        _, km, hm, fb = learned.fcg_truncated(apply_full, bf, jac, dinv, m, tol=1e-8)
        assert fb == 0 and abs(km - kj) <= 1 + 0.02 * kj   # rounding drift near convergence
        assert np.allclose(hm[:20], hj[:20], rtol=1e-6)
    _, k3, _, _ = learned.fcg_truncated(apply_full, bf, solve_full, dinv, 4, tol=1e-9)
    assert k3 == 1

