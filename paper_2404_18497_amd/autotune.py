"""Autotuner for the pilot search's launch shape.

The search places the buckets of one partition per wavefront. Its launch shape -- wavefronts per
workgroup, and either one wavefront per partition or a persistent grid of `groups_per_cu`
workgroups per compute unit pulling `items_per_grab` partitions at a time from an atomic queue --
changes only speed, never a result. The tuner times the search phase of real builds for every
candidate shape (best of `repeats`), installs the fastest with ``set_search_config`` and returns the
full table so callers can record it.
"""

from __future__ import annotations

import itertools

from . import binding

WAVES = (1, 2, 4, 8)
SCHEDULES = ((0, 1), (1, 1), (1, 4), (2, 1), (2, 4), (4, 1), (4, 4), (4, 16), (8, 4), (16, 4))


def candidates(waves=WAVES, schedules=SCHEDULES):
    return [dict(waves_per_group=w, groups_per_cu=g, items_per_grab=grab)
            for w, (g, grab) in itertools.product(waves, schedules)]


def _time_search(build, repeats: int) -> float:
    best = float("inf")
    for _ in range(repeats):
        handles = build()
        hs = [handles] if isinstance(handles, binding.MPHF) else handles
        best = min(best, hs[0].build_info()["search_ms"])
        for h in hs:
            h.close()
    return best


def tune(build, repeats: int = 2, cands=None, install: bool = True, log=None):
    """Times `build()` (returning a handle or a list of batch handles) under every candidate shape.

    Returns (best_shape, [(shape, search_ms), ...]); installs the best shape unless install=False."""
    cands = cands or candidates()
    before = binding.get_search_config()
    table = []
    try:
        for c in cands:
            binding.set_search_config(**c)
            ms = _time_search(build, repeats)
            table.append((c, ms))
            if log:
                log(f"{c} search {ms:.3f} ms")
    finally:
        binding.set_search_config(**before)
    best = min(table, key=lambda x: x[1])[0]
    if install:
        binding.set_search_config(**best)
    return best, table


def tune_batch(key_tensors, prm, repeats: int = 2, cands=None, install: bool = True, log=None):
    """Tunes the search shape on a batched build of the given key sets."""
    return tune(lambda: binding.build_batch_u64(key_tensors, prm), repeats, cands, install, log)


def tune_plain(keys, prm, repeats: int = 2, cands=None, install: bool = True, log=None):
    """Tunes the search shape on a plain build of one key set."""
    return tune(lambda: binding.build_u64(keys, prm), repeats, cands, install, log)
