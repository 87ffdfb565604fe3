"""Autotuner for the launch shape of the contact step.

Chooses, for a given workload, the detection work-item node size
(``tile_node_shift``: Z-order nodes of 2^shift cells), the detection
workgroup size (``tile_threads``), the LDS budget of a
detection tile (``tile_max_cells``, ``tile_max_stage``), the interval between
spatial re-sorts (``reorder_every``), the lanes per particle of the sweeps
(``pja_lanes``), the iteration blocking (one launch per sweep, or the fused
cooperative step, ``fused``) and then the hash-table size n_h (Eq. (6); Sec.
II-B's heuristic is n_h = 2 n), by timing each candidate through the C ABI
over a window that spans at least one re-sort.  The library's own defaults
are the first candidate, and another replaces the best so far only when it is
faster by a margin (2% by default), so timing noise does not trade a good
default for a worse shape.  These parameters change only memory layout, bucket
aliasing and work decomposition: partners are listed by (neighbour cell,
original index), never by bucket, and impulse sums keep list order, so every
output is bitwise identical across them (the GPU tests check this; the fused
step agrees to rounding) and the choice is free of numerical side effects.
The cell size is left at its default (c = 2 r_max (1 + 2^-10)) unless asked
for, because it changes which cell, and so which list position, a partner
falls in.

Results are cached in a JSON file keyed by device, particle count, particles
per cell and body count.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import gg

CACHE_ENV = "GG_AUTOTUNE_CACHE"


def _cache_path():
    return os.environ.get(CACHE_ENV, os.path.join(os.path.expanduser("~"), ".cache", "gg_autotune.json"))


def node_dims(shift):
    """Cells per axis of a Z-order node of 2^shift cells (x gets the extra bits)."""
    bx = (shift + 2) // 3
    by = (shift + 1) // 3
    bz = shift // 3
    return 1 << bx, 1 << by, 1 << bz


def particles_per_cell(x, radius):
    """Mean particles per occupied cell at the default cell size."""
    r = np.asarray(radius, np.float32)
    c = 2.0 * float(r.max()) * (1.0 + 2.0 ** -10)
    k = np.floor(np.asarray(x, np.float64) / c + 0.5).astype(np.int64)
    k -= k.min(axis=0)
    key = (k[:, 0] * 1_000_003 + k[:, 1]) * 1_000_033 + k[:, 2]
    return len(x) / max(1, len(np.unique(key)))


def candidates(ppc):
    """Launch shapes worth timing for ppc particles per occupied cell: for each
    workgroup size (64, 128, 256 threads), nodes holding roughly 0.3 to 1.4
    workgroups of particles, an LDS budget for the node's box plus a one-cell
    halo and one cell of drift, and three re-sort intervals.  (The library's
    defaults are timed before these.)"""
    out = []
    for tb in (64, 128, 256):
        for shift in range(2, 10):
            dx, dy, dz = node_dims(shift)
            per_node = ppc * dx * dy * dz
            if not 0.3 * tb <= per_node <= 1.4 * tb:
                continue
            cells = (dx + 3) * (dy + 3) * (dz + 3)
            stage = int(math.ceil(cells * (ppc + 0.6) * 1.1))
            if stage > 2048 or cells > 4096:
                continue
            for reorder in (8, 16, 32):
                out.append({"tile_node_shift": shift, "tile_max_cells": cells, "tile_max_stage": stage,
                            "tile_threads": tb, "reorder_every": reorder})
    return out


def hash_factors():
    """Table sizes tried, as multiples of the particle count (2 is the default)."""
    return (0.5, 1.0, 4.0, 8.0)


def key_of(n, ppc, n_bodies):
    try:
        import torch
        dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    except Exception:  # torch missing or no device
        dev = "unknown"
    return f"{dev}|n2^{int(round(math.log2(max(n, 1))))}|ppc{ppc:.1f}|bodies{n_bodies}"


def lane_counts():
    """Lanes per particle tried for the sweeps (results do not depend on it)."""
    return (1, 2, 4)


def cell_factors():
    """Cell sizes tried by ``tune(..., tune_cell=True)``, as multiples of the
    smallest admissible cell 2 r_max (1 + 2^-10)."""
    return (1.0, 1.125, 1.25)


def tune(x, v, radius, bodies, sim_kwargs=None, steps=32, warmup=8, use_cache=True, verbose=False,
         tune_cell=False, margin=0.02, record=None):
    """Return the fastest launch-shape parameters for this workload (a dict of
    gg.Sim keyword arguments).  With tune_cell the cell size is tuned too:
    a larger cell changes which cell, and so which list position, a partner
    falls in, hence the summation order and the rounding of the impulses
    (never the contact set); by default it stays at the smallest cell.
    record: a list that receives (candidate, ms per step or None) for every
    candidate timed, the library's defaults first."""
    sim_kwargs = dict(sim_kwargs or {})
    ppc = particles_per_cell(x, radius)
    key = key_of(len(x), ppc, len(bodies)) + ("|cell" if tune_cell else "")
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return dict(cache[key]["params"])

    def timed(cand):
        # wall time of `steps` steps after `warmup` (each step call returns
        # once its steps are done); no phase events, which would distort
        # launch-bound small beds
        kw = dict(sim_kwargs)
        kw.update(cand)
        try:
            sim = gg.Sim(x, v, radius, bodies, **kw)
            sim.step(warmup)
            t0 = time.perf_counter()
            sim.step(steps)
            t = (time.perf_counter() - t0) / steps
            st = sim.stats()
            sim.close()
        except gg.GGError as e:
            if verbose:
                print("autotune: candidate failed", cand, e)
            return None
        if verbose:
            print(f"autotune: {cand} -> {1e3 * t:.3f} ms/step, fallback items {st['detect_fallback']}")
        if record is not None:
            record.append((dict(cand), 1e3 * t))
        return t

    best, best_t = {}, timed({})     # the library's defaults
    if best_t is None:
        best_t = float("inf")

    def better(t):
        return t is not None and t < best_t * (1.0 - margin)
    for cand in candidates(ppc):
        t = timed(cand)
        if better(t):
            best, best_t = cand, t
    # then the lanes per particle of the sweeps, the iteration blocking (one
    # launch per sweep, or detection and all sweeps in one cooperative launch
    # with grid barriers), and the table size
    for lanes in lane_counts():
        cand = dict(best, pja_lanes=lanes)
        t = timed(cand)
        if better(t):
            best, best_t = cand, t
    if not sim_kwargs.get("differentiable"):
        cand = dict(best, fused=True)
        t = timed(cand)
        if better(t):
            best, best_t = cand, t
    n = len(x)
    for factor in hash_factors():
        cand = dict(best, hash_size=max(1, int(factor * n)))
        t = timed(cand)
        if better(t):
            best, best_t = cand, t
    if tune_cell:
        c0 = 2.0 * float(np.max(radius)) * (1.0 + 2.0 ** -10)
        for factor in cell_factors()[1:]:
            # a larger cell holds more particles: rescale the LDS budget
            cand = dict(best, cell_size=c0 * factor,
                        tile_max_stage=min(2048, int(best.get("tile_max_stage", 768) * factor ** 3) + 1))
            t = timed(cand)
            if better(t):
                best, best_t = cand, t
    if use_cache:
        cache[key] = {"params": best, "ms_per_step": 1e3 * best_t}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    return dict(best)
