"""Autotuning of the solver's kernel choices, with a persistent JSON cache.

Tunes the options that select kernel variants but not results (within the
parity bar): the banded kernels (register panels with lookahead vs the
wide-band kernels), the wide-band group size, and the COCG row blocking.
Candidates are timed on the caller's own workload (one warm-up and two timed
solves each, the fastest kept); the choice is stored under a key of the
workload's shape, so a later solve of the same shape reads it back instead
of timing again.  Every timed solve runs in the library; this module only
orders the candidates and keeps the cache.
"""
from __future__ import annotations

import json
import os
import time

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gepci_tune.json")

BAND_CANDIDATES = [{"band_kernels": "auto"}, {"band_kernels": "wide"}]
COCG_CANDIDATES = [{"rows_per_block": r, "row_group": g} for g in (4, 1) for r in (8, 16, 32)]


def shape_key(n_total, bw_max, nnz_per_row, columns, precision, solver, problems=1):
    """Cache key: the workload features the kernel choice depends on."""
    return (f"n{int(n_total)}_bw{int(bw_max)}_nnz{nnz_per_row:.1f}_w{int(columns)}_{precision}"
            f"_{solver}_p{int(problems)}")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, cache):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(solve, key, candidates, cache_path=DEFAULT_CACHE, repeats=2, log=None):
    """Return the fastest candidate option dict for `key`.

    solve(**opts) runs one solve with the candidate's options and returns
    its result (or list of results); the cache is consulted first and
    updated after timing.
    """
    cache = _load(cache_path)
    if key in cache:
        if log:
            log(f"autotune: cached choice for {key}: {cache[key]['opts']}")
        return dict(cache[key]["opts"])
    timings = []
    for opts in candidates:
        solve(**opts)                      # warm-up: kernels loaded, workspace kept
        best = None
        for _ in range(repeats):
            t0 = time.perf_counter()
            solve(**opts)
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        timings.append((best, opts))
        if log:
            log(f"autotune: {opts}: {best * 1e3:.1f} ms")
    best_t, best_opts = min(timings, key=lambda t: t[0])
    cache[key] = {"opts": best_opts, "ms": round(best_t * 1e3, 2),
                  "candidates": [{"opts": o, "ms": round(t * 1e3, 2)} for t, o in timings]}
    _store(cache_path, cache)
    return dict(best_opts)
