"""Lanes per particle in the projected-Jacobi sweep (pja_lanes = 1, 2, 4):
every lane takes every L-th contact of its particle and the impulse sum keeps
list order, so all three give the same bits; and one step with four lanes
matches the FP64 oracle to the parity bar."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2306_01369_amd import gg, scenes

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _run(sc, steps, lanes, **kw):
    sim = gg.Sim(sc.x, sc.v, sc.radius, sc.bodies, dt=sc.dt, alpha=sc.alpha, mu=sc.mu, n_iters=sc.n_iters,
                 env_offsets=getattr(sc, "env_offsets", None), pja_lanes=lanes, diagnostics=True, **kw)
    tw = getattr(sc, "twists", None)
    sim.step(steps, twists=None if tw is None else tw[:steps])
    out = (sim.read("pos"), sim.read("vel"), sim.read("impulses"), sim.read("dv"), sim.stats())
    sim.close()
    return out


@pytest.mark.parametrize("case", ["drop", "batched", "fp64", "bed-with-tool"])
def test_lanes_per_particle_give_the_same_bits(case):
    kw = {}
    if case == "drop":
        sc, steps = scenes.drop_scene(), 40
    elif case == "batched":
        sc, steps = scenes.batched_scene(n_envs=4, lo=2000, hi=5000, n_steps=10), 10
    elif case == "fp64":
        sc, steps = scenes.drop_scene(), 20
        kw["precision"] = 1
    else:
        sc = scenes.column_scene(n=5000, r=0.004)
        side = float(sc.x[:, 0].max())
        sc.bodies = sc.bodies + [scenes.box_tool((side / 2, side / 2, float(sc.x[:, 2].max()) + 0.01),
                                                 (0.01, 0.02, 0.02), nu=(0.1, 0.0, -0.3))]
        steps = 20
    ref = _run(sc, steps, 1, **kw)
    assert ref[4]["pja_lanes"] == 1
    for lanes in (2, 4):
        got = _run(sc, steps, lanes, **kw)
        assert got[4]["pja_lanes"] == lanes
        say(case, "lanes", lanes, "contacts", len(got[2]), "max |dx|", float(np.abs(got[0] - ref[0]).max()))
        for a, b in zip(got[:4], ref[:4]):
            assert np.array_equal(a, b), (case, lanes)


def test_four_lanes_one_step_against_the_oracle():
    sc = scenes.column_scene(n=4000, r=0.004)
    side = float(sc.x[:, 0].max())
    bodies = sc.bodies + [scenes.capsule_tool((side / 2, side / 2, float(sc.x[:, 2].max()) + 0.005), 0.01, 0.02,
                                              nu=(0.0, 0.1, -0.2))]
    sim = gg.Sim(sc.x, sc.v, sc.radius, bodies, pja_lanes=4, diagnostics=True)
    orc = O.Oracle(sc.x.astype(np.float64), sc.v.astype(np.float64), sc.radius, bodies)
    sim.step(1)
    d = orc.step(detail=True)
    assert np.array_equal(sim.read("contacts"), d["pairs"])
    P = sim.read("impulses").astype(np.float64)
    err = np.abs(P - d["impulses"]).max() / np.abs(d["impulses"]).max()
    dv = sim.read("dv").astype(np.float64)
    errv = np.abs(dv - d["dv"]).max() / np.abs(d["dv"]).max()
    say("four lanes vs oracle: impulses", err, "dv", errv)
    assert err <= 1e-5 and errv <= 1e-5
    sim.close()


def test_lanes_give_the_same_gradients():
    sc = scenes.diff_scene(n=4096)
    rng = np.random.default_rng(4)
    steps = 6
    tw = np.zeros((steps, len(sc.bodies), 6), np.float32)
    tw[:, -1, :3] = (0.2, 0.0, -0.1)
    gx = rng.normal(size=(sc.n, 3)).astype(np.float32)
    gv = rng.normal(size=(sc.n, 3)).astype(np.float32)
    out = []
    for lanes in (1, 2, 4):
        sim = gg.Sim(sc.x, sc.v, sc.radius, sc.bodies, dt=sc.dt, alpha=sc.alpha, mu=sc.mu, n_iters=sc.n_iters,
                     differentiable=True, checkpoint_every=3, pja_lanes=lanes)
        sim.step(steps, twists=tw)
        res = (sim.read("pos"),) + tuple(sim.backward(gx, gv))
        sim.close()
        out.append(res)
    for lanes, res in zip((2, 4), out[1:]):
        say("gradients, lanes", lanes, "max |d dL/dx0|", float(np.abs(res[1] - out[0][1]).max()))
        for a, b in zip(res, out[0]):
            assert np.array_equal(a, b), lanes
