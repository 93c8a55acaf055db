"""CPU checks of the batched-solve autotuner's host logic with the library
calls replaced by a table: it times every tile shape at each requested count
of workgroups per CU capped at the resident limit (each distinct count once),
applies the fastest, caches it under the device and problem-size multiset,
and replays the cache without timing."""
import types

from paper_1010_2832_amd import autotune

SHAPES = [(64, 4), (64, 8), (32, 8), (128, 2), (64, 12), (64, 16)]
CAPS = [4, 2, 4, 2, 2, 2]
# ms per CG iteration by (variant, workgroups per CU); 64x16 at 2 is the fastest
TIMES = {(v, b): 1.0 + 0.1 * v + (0.2 if b == 1 else 0.0) for v in range(6) for b in (1, 2, 4)}
TIMES[(5, 2)] = 0.5


class FakeBatch:
    def __init__(self, sizes):
        self.sizes = sizes
        self.timed = []
        self.applied = None

    def vfs_batch_time_variant(self, v, bpc, iterations):
        self.timed.append((v, bpc, iterations))
        return TIMES[(v, bpc)]

    def vfs_batch_set_tiles(self, v, bpc):
        self.applied = (v, bpc)


def fake_lib():
    return types.SimpleNamespace(
        vfs_batch_num_variants=lambda: len(SHAPES),
        vfs_batch_max_blocks_per_cu=lambda v: CAPS[v],
        vfs_batch_variant_shape=lambda v: SHAPES[v])


def test_sweep_caps_picks_and_caches(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "V", fake_lib())
    monkeypatch.setattr(autotune, "_device_name", lambda: "dev")
    cache = str(tmp_path / "at.json")
    b = FakeBatch([(64, 64), (96, 96)])
    res = autotune.tune(b, iterations=7, cache_path=cache)
    # every variant at each distinct capped count, with the requested iterations
    want = sorted((v, bpc) for v in range(6) for bpc in {min(x, CAPS[v]) for x in (1, 2, 4)})
    assert sorted((v, bpc) for v, bpc, _ in b.timed) == want
    assert all(it == 7 for _, _, it in b.timed)
    assert all(bpc <= CAPS[v] for v, bpc, _ in b.timed)
    assert (res["variant"], res["blocks_per_cu"]) == (5, 2) and b.applied == (5, 2)
    assert list(res["shape"]) == [64, 16] and res["ms_per_iteration"] == 0.5
    assert res["cached"] is False and len(res["table"]) == len(want)
    # same sizes in another order: the cache answers, nothing is timed
    b2 = FakeBatch([(96, 96), (64, 64)])
    again = autotune.tune(b2, cache_path=cache)
    assert again["cached"] is True and b2.timed == [] and b2.applied == (5, 2)
    # other sizes, or no cache: timed again
    b3 = FakeBatch([(64, 64)])
    assert autotune.tune(b3, cache_path=cache)["cached"] is False and b3.timed
    b4 = FakeBatch([(64, 64), (96, 96)])
    assert autotune.tune(b4, cache_path=cache, use_cache=False)["cached"] is False and b4.timed


def test_near_ties_go_to_the_larger_tile(tmp_path, monkeypatch):
    """Entries within 1% of the fastest probe: the largest tile area wins;
    beyond 1% the fastest wins."""
    monkeypatch.setattr(autotune, "V", fake_lib())
    monkeypatch.setattr(autotune, "_device_name", lambda: "dev")
    monkeypatch.setitem(TIMES, (4, 2), 0.5)            # 64x12, the fastest probe
    monkeypatch.setitem(TIMES, (5, 2), 0.5 * 1.005)    # 64x16, 0.5% slower: a tie
    b = FakeBatch([(64, 64)])
    res = autotune.tune(b, cache_path=None, use_cache=False)
    assert list(res["shape"]) == [64, 16] and b.applied == (5, 2)
    monkeypatch.setitem(TIMES, (5, 2), 0.5 * 1.02)     # 2% slower: 64x12 wins
    b2 = FakeBatch([(64, 64)])
    res2 = autotune.tune(b2, cache_path=None, use_cache=False)
    assert list(res2["shape"]) == [64, 12] and b2.applied == (4, 2)
