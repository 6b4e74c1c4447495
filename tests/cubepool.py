"""Run a function over slices of the exhaustive 2^24-colour cube in a process
pool and return the per-slice results (test helper)."""
import multiprocessing as mp
import os

import numpy as np

import synth

CHUNK = 1 << 21
WORKERS = min(8, os.cpu_count() or 1)


def _slice(start):
    return synth.cube_slice(start, CHUNK)


def cube_map(fn, *args):
    """fn(v8 (CHUNK, 3) uint8, *args) for every slice of the cube."""
    ctx = mp.get_context("fork")
    with ctx.Pool(WORKERS) as pool:
        return pool.starmap(_call, [(fn, s, args) for s in range(0, 1 << 24, CHUNK)])


def _call(fn, start, args):
    return fn(_slice(start), *args)


def mean_max(parts):
    """Combine per-slice (sum, max) pairs over the 2^24 cube."""
    s = sum(p[0] for p in parts)
    m = max(p[1] for p in parts)
    return s / float(1 << 24), m


def sum_max(d):
    d = np.asarray(d)
    return float(d.sum()), float(d.max())


_SHARED = {}


def cube_map_shared(fn, shared, *args):
    """Like cube_map, with `shared` (e.g. large GPU results as numpy arrays)
    inherited by the forked workers instead of pickled; fn(v8, start, shared, *args)."""
    _SHARED["v"] = shared
    ctx = mp.get_context("fork")
    try:
        with ctx.Pool(WORKERS) as pool:
            return pool.starmap(_call_shared, [(fn, s, args) for s in range(0, 1 << 24, CHUNK)])
    finally:
        _SHARED.clear()


def _call_shared(fn, start, args):
    return fn(_slice(start), start, _SHARED["v"], *args)
