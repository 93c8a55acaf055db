"""Pins of the oracle's brick-local Schwarz preconditioners
(oracle/schwarz.py).

  * Same-colour samples never couple: A has no entry between two samples of
    one (type, parity) colour, on random 2D and 3D geometries -- what lets a
    colour be relaxed at once.
  * With one brick holding the whole grid and no overlap, the preconditioner
    is the textbook symmetric Gauss-Seidel operator (D + U)^-1 D (D + L)^-1
    of A in the colour ordering (dense triangular solves).
  * The preconditioner is symmetric positive definite for every brick size
    and overlap tried (dense operator, 2D and 3D), so plain PCG applies.
  * PCG with it converges to the direct solution, in fewer iterations than
    Jacobi PCG, and with the overlap (scaled by m^-1/2) in no more
    iterations than without it.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import cg, schwarz, system
from test_oracle_system import _box_case, _random_geometry


def _asm(dim, n, seed):
    rng = np.random.default_rng(seed)
    phi_l, phi_s = _random_geometry(dim, n, rng, solid=True)
    return system.assemble(_box_case(dim, n, phi_l, phi_s, rng))


def _dense_operator(asm, apply_m):
    act = asm.act_idx
    M = np.zeros((len(act), len(act)))
    for k, s in enumerate(act):
        e = np.zeros(asm.grid.n_samples())
        e[s] = 1.0
        M[:, k] = apply_m(e)[act]
    return M


@pytest.mark.parametrize("dim,n,seed", [(2, 9, 1), (2, 12, 2), (3, 5, 3), (3, 6, 4)])
def test_same_colour_samples_never_couple(dim, n, seed):
    asm = _asm(dim, n, seed)
    col = schwarz.colours(asm.grid)
    A = asm.A_full.tocoo()
    off = A.row != A.col
    same = col[A.row] == col[A.col]
    assert not np.any(off & same & (A.data != 0.0))


@pytest.mark.parametrize("dim,n,seed", [(2, 7, 5), (3, 4, 6)])
def test_single_brick_is_textbook_symmetric_gauss_seidel(dim, n, seed):
    asm = _asm(dim, n, seed)
    M = _dense_operator(asm, schwarz.preconditioner(asm, b=n + 1, overlap=0))
    A = asm.A.toarray()
    col = schwarz.colours(asm.grid)[asm.act_idx]
    order = np.argsort(col, kind="stable")
    Ap = A[np.ix_(order, order)]
    D = np.diag(np.diag(Ap))
    L = np.tril(Ap, -1)
    U = np.triu(Ap, 1)
    G = sla.solve_triangular(D + U, D @ sla.solve_triangular(D + L, np.eye(len(A)), lower=True))
    inv = np.empty_like(order)
    inv[order] = np.arange(len(order))
    want = G[np.ix_(inv, inv)]
    assert np.abs(M - want).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("dim,n,seed,b,overlap", [(2, 10, 7, 3, 0), (2, 10, 7, 3, 1), (2, 11, 8, 4, 2),
                                                   (3, 5, 9, 2, 0), (3, 5, 9, 2, 1), (3, 6, 10, 3, 1)])
def test_preconditioner_is_spd(dim, n, seed, b, overlap):
    asm = _asm(dim, n, seed)
    M = _dense_operator(asm, schwarz.preconditioner(asm, b, overlap))
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    assert ev[0] > 0.0


@pytest.mark.parametrize("dim,n", [(2, 24), (3, 10)])
def test_pcg_converges_to_the_direct_solution(dim, n):
    rng = np.random.default_rng(11)
    phi_l, phi_s = _random_geometry(dim, n, rng, solid=True)
    asm = system.assemble(_box_case(dim, n, phi_l, phi_s, rng, dt=0.05))
    x_direct = system.solve_direct(asm)
    if system.is_enclosed(asm):
        pytest.skip("enclosed: pressure constant")
    b = 4 if dim == 3 else 8
    its = {}
    _, its_j, _ = cg.jacobi_pcg(asm.A, asm.b, tol=1e-11)
    for overlap in (0, 1):
        x, its[overlap] = schwarz.pcg(asm, schwarz.preconditioner(asm, b, overlap), tol=1e-11)
        assert np.abs(x - x_direct).max() <= 1e-7 * np.abs(x_direct).max()
        assert its[overlap] < its_j, (overlap, its, its_j)
    # the scaled overlap helps rather than hurts
    assert its[1] <= its[0], its
