"""GPU parity of the batched persistent 2D solve (config-4 shaped problems)
against the oracle, through the C ABI."""
import numpy as np
import pytest

import cases
from gpu_util import expected_tile_samples, flat_faces, velocity_rel_linf
from oracle import system

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[batch] {msg}", flush=True)


def _problems(sizes, seed=7):
    return [cases.drop2d(n, seed * 100 + q) for q, n in enumerate(sizes)]


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5])
def test_batch_matches_oracle_every_tile_variant(variant):
    from paper_1010_2832_amd import vfstokes as V
    sizes = [24, 37, 64, 50, 33]
    probs = _problems(sizes)
    _banner(f"variant {variant} sizes {sizes}")
    b = V.batch_from_cases(probs, tol=1e-9)
    b.vfs_batch_set_tiles(variant, 2)
    b.vfs_batch_step(probs[0]["dt"])
    st = b.vfs_batch_get_stats()
    _banner(f"  stats {st}")
    assert st["graph_used"] == 1 and st["status"] == 0
    for i, c in enumerate(probs):
        asm, x, u = system.step(c)
        ug = flat_faces(asm.grid, b.vfs_batch_get_velocity(i))
        err = velocity_rel_linf(asm, ug, u)
        pr = b.vfs_batch_get_problem(i)
        assert pr["n_active"] == int(asm.active.sum())
        assert pr["rel_residual"] <= 1e-9
        assert system.true_relative_residual(asm, b.vfs_batch_get_solution(i)) <= 2e-9
        assert err <= 1e-4, (i, err)
    b.close()


def test_batch_items_are_the_active_tiles():
    """Work items are the tiles holding an active sample.  For every tile
    shape their count equals the count of tiles over the oracle's active set,
    an all-air problem keeps a single item and retires at once (its velocity
    equals the oracle's), a 3x3 problem smaller than one tile solves, and the
    others match the oracle.  Every step restarts from u^0."""
    from paper_1010_2832_amd import vfstokes as V
    probs = _problems([48, 64, 40, 3], seed=11)
    air = cases.drop2d(32, 1105)
    air["phi_l"] = np.ones_like(air["phi_l"])      # all air: no active sample
    probs.insert(2, air)
    ref = [system.step(c) for c in probs]
    b = V.batch_from_cases(probs, tol=1e-9)
    for variant in range(V.vfs_batch_num_variants()):
        bx, by = V.vfs_batch_variant_shape(variant)
        for i, c in enumerate(probs):
            b.vfs_batch_set_problem(i, c)
        b.vfs_batch_set_tiles(variant, 2)
        b.vfs_batch_step(probs[0]["dt"])
        st = b.vfs_batch_get_stats()
        tiles = [expected_tile_samples(asm, (bx, by)) // (bx * by * 3) for asm, _, _ in ref]
        want = sum(max(1, t) for t in tiles)
        _banner(f"variant {variant} ({bx}x{by}): active tiles {tiles}, items {st['n_items']}")
        assert st["status"] == 0
        assert st["n_items"] == want and st["n_tile_samples"] == want * bx * by * 3
        for i, (asm, x, u) in enumerate(ref):
            ug = flat_faces(asm.grid, b.vfs_batch_get_velocity(i))
            pr = b.vfs_batch_get_problem(i)
            assert pr["n_active"] == int(asm.active.sum())
            if pr["n_active"] == 0:
                assert pr["iterations"] == 0 and np.array_equal(ug, u), i
            else:
                assert velocity_rel_linf(asm, ug, u) <= 1e-4, (variant, i)
    b.close()


def test_batch_uneven_sizes_and_repeat_steps():
    """Uneven sizes (64..256), two consecutive steps (the velocity advances),
    second step compared with the oracle fed the first step's output."""
    from paper_1010_2832_amd import vfstokes as V
    sizes = [64, 96, 160, 256, 128, 64]
    probs = _problems(sizes, seed=9)
    b = V.batch_from_cases(probs, tol=1e-8)
    b.vfs_batch_step(probs[0]["dt"])
    u1 = [b.vfs_batch_get_velocity(i) for i in range(len(probs))]
    b.vfs_batch_step(probs[0]["dt"])
    st = b.vfs_batch_get_stats()
    _banner(f"  stats {st}")
    assert st["latency_p50_ms"] > 0 and st["latency_max_ms"] >= st["latency_p90_ms"] >= st["latency_p50_ms"]
    # problems retire independently: the 64^2 ones finish well before the 256^2 one
    lat = [b.vfs_batch_get_problem(i)["latency_ms"] for i in range(len(probs))]
    _banner(f"  per-problem latency ms {[round(v, 2) for v in lat]}")
    assert max(lat[0], lat[5]) < 0.5 * lat[3], lat
    for i, c in enumerate(probs):
        c2 = dict(c, u=u1[i])
        asm, x, u = system.step(c2)
        err = velocity_rel_linf(asm, flat_faces(asm.grid, b.vfs_batch_get_velocity(i)), u)
        assert err <= 1e-4, (i, err)
    b.close()


def test_autotuner_picks_a_valid_configuration(tmp_path):
    from paper_1010_2832_amd import autotune
    from paper_1010_2832_amd import vfstokes as V
    probs = _problems([64, 96, 128])
    b = V.batch_from_cases(probs, tol=1e-6)
    b.vfs_batch_step(probs[0]["dt"])
    res = autotune.tune(b, iterations=20, cache_path=str(tmp_path / "at.json"))
    _banner(f"  autotune {res['variant']} {res['blocks_per_cu']} {res['ms_per_iteration']:.4f} ms/iter")
    assert 0 <= res["variant"] < V.vfs_batch_num_variants()
    assert all(r["ms_per_iteration"] > 0 for r in res["table"])
    # every timed configuration can be resident at once (the grid barrier needs it)
    assert all(1 <= r["blocks_per_cu"] <= V.vfs_batch_max_blocks_per_cu(r["variant"])
               for r in res["table"])
    again = autotune.tune(b, cache_path=str(tmp_path / "at.json"))
    assert again["cached"] and again["variant"] == res["variant"]
    b.vfs_batch_step(probs[0]["dt"])
    st = b.vfs_batch_get_stats()
    assert st["status"] == 0
    assert st["blocks_per_cu"] == res["blocks_per_cu"]
    b.close()


def test_batch64_full_size():
    """64 problems with sizes drawn from {64, 96, ..., 512}^2, autotuned,
    mixed precision to 1e-6; oracle parity on the smallest, a middle and the
    largest problem; prints latency percentiles and aggregate DOF*iter/s."""
    from paper_1010_2832_amd import autotune
    from paper_1010_2832_amd import vfstokes as V
    probs = cases.batch64()
    sizes = [c["n"][0] for c in probs]
    _banner(f"batch64: {len(probs)} problems, sizes {min(sizes)}..{max(sizes)}")
    b = V.batch_from_cases(probs, tol=1e-6)
    b.vfs_batch_step(probs[0]["dt"])
    res = autotune.tune(b, iterations=20, use_cache=False, cache_path=None)
    _banner(f"  autotune: {res['variant']} {res['shape']} bpc {res['blocks_per_cu']} "
            f"{res['ms_per_iteration']:.4f} ms/iter")
    b.vfs_batch_step(probs[0]["dt"])     # second step starts from the first's velocity
    st = b.vfs_batch_get_stats()
    _banner(f"  stats {st}")
    _banner(f"  aggregate DOF*iter/s over the solve: {st['dof_iters'] / (st['t_solve_ms'] * 1e-3):.3e}")
    assert st["status"] == 0
    order = np.argsort(sizes)
    for i in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        pr = b.vfs_batch_get_problem(i)
        assert pr["rel_residual"] <= 1e-6
        _banner(f"  problem {i} n={sizes[i]} {pr}")
    b.close()
    # parity at the tolerance the benchmark reports (bench.BATCH_TOL): a fresh
    # batch, one step, against the oracle on three problems
    b = V.batch_from_cases(probs, tol=1e-9)
    b.vfs_batch_step(probs[0]["dt"])
    for i in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        asm, x, u = system.step(probs[i])
        err = velocity_rel_linf(asm, flat_faces(asm.grid, b.vfs_batch_get_velocity(i)), u)
        _banner(f"  parity problem {i} n={sizes[i]} velocity rel Linf {err:.2e}")
        assert err <= 1e-4
    b.close()
