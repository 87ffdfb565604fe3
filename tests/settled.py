"""The scoop bed's seeded-settling plan (scenes.SETTLE_*) run by the oracle, on
a small footprint: the settled random bed that parity tests start from.  The
state is produced by the oracle alone, so the oracle may take it as input."""
import functools
import math

import numpy as np

import oracle as O
from paper_2306_01369_amd import scenes

SIDE = 0.105          # 20 x 20 pour sites per layer at spacing 2.6 r (r = 2 mm)
N = 11200             # 28 full layers


def oracle_settle(scene):
    """Frictionless compaction, then settling with the scene's friction until
    all but scenes.settle_fast_allowed(n) grains are slower than SETTLE_VMAX
    (checked every SETTLE_CHECK_EVERY steps).  Returns (x, v, settle steps of
    the second phase, max speed), FP64."""
    kw = dict(dt=scene.dt, alpha=scene.alpha, gravity=scene.gravity, n_iters=scenes.SETTLE_ITERS)
    orc = O.Oracle(scene.x.astype(np.float64), scene.v.astype(np.float64), scene.radius, scene.bodies, mu=0.0,
                   **kw)
    for _ in range(scenes.SETTLE_COMPACT_STEPS):
        orc.step()
    orc = O.Oracle(orc.x, orc.v, scene.radius, scene.bodies, mu=scene.mu, **kw)
    steps, vmax = 0, math.inf
    while steps < scenes.SETTLE_MAX_STEPS:
        for _ in range(scenes.SETTLE_CHECK_EVERY):
            orc.step()
        steps += scenes.SETTLE_CHECK_EVERY
        speed = np.sqrt((orc.v ** 2).sum(1))
        vmax = float(speed.max())
        if int((speed >= scenes.SETTLE_VMAX).sum()) <= scenes.settle_fast_allowed(len(speed)):
            break
    return orc.x.copy(), orc.v.copy(), steps, vmax


@functools.lru_cache(maxsize=1)
def small_settled_bed():
    """(pour scene, x, v, settle steps, max speed) of the 11,200-grain bed."""
    pour = scenes.scoop_pour(n=N, side=SIDE)
    x, v, steps, vmax = oracle_settle(pour)
    return pour, x, v, steps, vmax


def bed_measures(x, r, side, pairs=None, n_pp=0):
    """Surface height (99th percentile of z + r), bulk packing fraction below it,
    and, with the contact list, the mean number of pair contacts of grains at
    least 3 diameters from the walls, the floor and the surface."""
    surface = scenes.surface_height(x, r)
    n = len(x)
    phi = n * (4.0 / 3.0) * math.pi * r ** 3 / (side * side * surface)
    out = {"surface": surface, "phi": phi}
    if pairs is not None:
        deg = np.bincount(np.asarray(pairs[:n_pp]).ravel(), minlength=n)
        m = 6 * r
        inner = ((x[:, 0] > m) & (x[:, 0] < side - m) & (x[:, 1] > m) & (x[:, 1] < side - m) &
                 (x[:, 2] > m) & (x[:, 2] < surface - m))
        out["coordination"] = float(deg[inner].mean())
        out["coordination_std"] = float(deg[inner].std())
        out["inner"] = int(inner.sum())
    return out
