"""The seeded-settling plan of the scoop bed, run by the oracle on a 11,200-grain
footprint: it must come to rest and give a random dense packing (not the
lattice it was poured from)."""
import numpy as np

import oracle as O
from paper_2306_01369_amd import scenes
from settled import SIDE, bed_measures, small_settled_bed


def test_settling_plan_reaches_rest_in_a_random_close_packing():
    pour, x, v, steps, vmax = small_settled_bed()
    r = float(pour.radius[0])
    assert vmax < scenes.SETTLE_VMAX and steps <= scenes.SETTLE_MAX_STEPS
    orc = O.Oracle(x, v, pour.radius, pour.bodies, dt=pour.dt, alpha=pour.alpha, mu=pour.mu,
                   n_iters=pour.n_iters)
    d = orc.step(detail=True)
    m = bed_measures(x, r, SIDE, d["pairs"], d["n_pp"])
    print(m, "settle steps", steps, "max speed", vmax)
    # random close packing of equal spheres: phi ~ 0.64 and about six
    # contacts per grain; the poured lattice (spacing 2.6 r) has phi = 0.24 and
    # no contacts, a settled simple-cubic stack 0.52 and exactly six, a
    # face-centred crystal 0.74 and twelve
    assert 0.58 <= m["phi"] <= 0.66, m
    assert 5.0 <= m["coordination"] <= 7.5, m
    assert m["coordination_std"] > 0.7, m          # contact numbers spread: no lattice
    assert m["inner"] > 2000
