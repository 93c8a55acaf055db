"""Autotuner for the batched persistent 2D solve.

Sweeps every compiled tile shape (vfs_batch_variant_shape) and a range of
persistent workgroups per compute unit (capped at what can be resident,
vfs_batch_max_blocks_per_cu), timing a fixed number of CG
iterations of the persistent kernel on the batch's assembled problems
(vfs_batch_time_variant), and applies the fastest.  Results are cached as
JSON keyed by device name and the multiset of problem sizes, so a later
process with the same batch shape skips the sweep.
"""
from __future__ import annotations

import hashlib
import json
import os

from . import vfstokes as V

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "vfstokes", "autotune.json")


def _key(batch, device_name):
    sig = ",".join(f"{a}x{b}" for a, b in sorted(batch.sizes))
    return f"{device_name}|{hashlib.sha1(sig.encode()).hexdigest()[:16]}|{len(batch.sizes)}"


def _device_name():
    try:
        import torch
        return torch.cuda.get_device_name(0)
    except Exception:
        return "unknown"


def tune(batch, iterations=40, blocks_per_cu=(1, 2, 4), cache_path=DEFAULT_CACHE, use_cache=True,
         tie=0.01):
    """Pick (variant, blocks_per_cu) for `batch` (which must have been stepped
    once so that its problems are assembled).  Returns a dict with the choice
    and the timing table; applies the choice to the batch.

    The probes time iterations with every problem still iterating.  Among the
    entries within `tie` (relative) of the fastest, the largest tile wins:
    later in a solve, as problems retire, the larger tiles' smaller halo share
    tells (full 64-problem steps: 64x16 815 ms against 64x12 840 ms, with
    probes 0.5% apart)."""
    key = _key(batch, _device_name())
    cache = {}
    if use_cache and cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        best = cache[key]
        batch.vfs_batch_set_tiles(best["variant"], best["blocks_per_cu"])
        return dict(best, cached=True)
    table = []
    for v in range(V.vfs_batch_num_variants()):
        # only counts that can all be resident (larger requests are capped)
        cap = V.vfs_batch_max_blocks_per_cu(v)
        for bpc in sorted({min(b, cap) for b in blocks_per_cu}):
            ms = batch.vfs_batch_time_variant(v, bpc, iterations)
            table.append(dict(variant=v, shape=V.vfs_batch_variant_shape(v), blocks_per_cu=bpc,
                              ms_per_iteration=ms))
    fastest = min(r["ms_per_iteration"] for r in table)
    near = [r for r in table if r["ms_per_iteration"] <= fastest * (1.0 + tie)]
    best = min(near, key=lambda r: (-r["shape"][0] * r["shape"][1], r["ms_per_iteration"]))
    batch.vfs_batch_set_tiles(best["variant"], best["blocks_per_cu"])
    result = dict(variant=best["variant"], blocks_per_cu=best["blocks_per_cu"],
                  shape=list(best["shape"]), ms_per_iteration=best["ms_per_iteration"], table=table)
    if cache_path:
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            cache[key] = {k: result[k] for k in ("variant", "blocks_per_cu", "shape", "ms_per_iteration")}
            json.dump(cache, open(cache_path, "w"), indent=1)
        except OSError:
            pass
    return dict(result, cached=False)
