"""The fused step (GG_FLAG_FUSED: detection, sweeps and position update in one
cooperative launch, the fused kernel order of the Sec. II-D ablation) against
the split launches.  Both run the same device functions in the same
per-particle order; the compiler may still contract a multiply and an add
into a fused multiply-add differently in the two kernels, so binary32 states
agree to rounding (contact lists exactly) and the binary64 build bit for bit."""
import sys

import numpy as np
import pytest

from paper_2306_01369_amd import gg, scenes

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _run(scene, steps, fused, **kw):
    sim = gg.Sim(scene.x, scene.v, scene.radius, scene.bodies, dt=scene.dt, alpha=scene.alpha, mu=scene.mu,
                 n_iters=scene.n_iters, fused=fused, env_offsets=getattr(scene, "env_offsets", None), **kw)
    tw = getattr(scene, "twists", None)
    if tw is not None:
        sim.step(steps, twists=tw[:steps])
    else:
        sim.step(steps)
    out = sim.read("pos"), sim.read("vel"), sim.read("contacts"), sim.stats()
    sim.close()
    return out


@pytest.mark.parametrize("case", ["drop", "column-tools", "batched", "fp64"])
def test_fused_step_is_bitwise_the_split_step(case):
    kw = {}
    if case == "drop":
        sc, steps = scenes.drop_scene(), 60
    elif case == "column-tools":
        sc = scenes.column_scene(n=6000, r=0.004)
        side = float(sc.x[:, 0].max())
        sc.bodies = sc.bodies + [scenes.box_tool((side / 2, side / 2, float(sc.x[:, 2].max()) + 0.02),
                                                 (0.01, 0.02, 0.03), nu=(0.0, 0.0, -0.5))]
        steps = 30
    elif case == "batched":
        sc, steps = scenes.batched_scene(n_envs=5, lo=2000, hi=6000, n_steps=12), 12
    else:
        sc, steps = scenes.drop_scene(), 25
        kw["precision"] = 1
    say(case, "n =", sc.n, "steps", steps)
    xs, vs, cs, ss = _run(sc, steps, False, **kw)
    xf, vf, cf, sf = _run(sc, steps, True, **kw)
    say(case, "contacts", len(cs), "max |dx|", float(np.abs(xf - xs).max()), "max |dv|", float(np.abs(vf - vs).max()))
    assert sf["steps_done"] == ss["steps_done"] == steps
    # the split step's detection takes work items from queues, the fused one in fixed shares
    assert ss["detect_queues"] == 1 and sf["detect_queues"] == 0
    if case == "fp64":
        assert np.array_equal(xs, xf) and np.array_equal(vs, vf) and np.array_equal(cs, cf)
        assert sf["contacts_summed"] == ss["contacts_summed"]
    else:
        assert np.abs(xf - xs).max() <= 1e-6
        assert np.abs(vf - vs).max() <= 1e-4 * max(1.0, float(np.abs(vs).max()))
    # one step from the same state: the same contacts, impulses to rounding
    sim_s = gg.Sim(xs, vs, sc.radius, sc.bodies, dt=sc.dt, alpha=sc.alpha, mu=sc.mu, n_iters=sc.n_iters,
                   env_offsets=getattr(sc, "env_offsets", None), **kw)
    sim_f = gg.Sim(xs, vs, sc.radius, sc.bodies, dt=sc.dt, alpha=sc.alpha, mu=sc.mu, n_iters=sc.n_iters,
                   env_offsets=getattr(sc, "env_offsets", None), fused=True, **kw)
    sim_s.step(1)
    sim_f.step(1)
    assert np.array_equal(sim_s.read("contacts"), sim_f.read("contacts"))
    Ps, Pf = sim_s.read("impulses").astype(np.float64), sim_f.read("impulses").astype(np.float64)
    if len(Ps):
        err = np.abs(Pf - Ps).max() / np.abs(Ps).max()
        say(case, "one step: impulse rel diff", err)
        assert err <= 1e-5
    sim_s.close()
    sim_f.close()


def test_fused_step_reports_capacity_errors_like_the_split_step():
    # the failed step still reports the largest contact count its detection
    # saw (what a caller sizes the capacity from), the same in both forms
    sc = scenes.column_scene(n=3000, r=0.004)
    largest = []
    for fused in (False, True):
        sim = gg.Sim(sc.x, sc.v, sc.radius, sc.bodies, fused=fused, max_contacts=4)
        x0 = sim.read("pos")
        with pytest.raises(gg.CapacityError):
            sim.step(3)
        st = sim.stats()
        say("fused" if fused else "split", "steps done before the capacity error", st["steps_done"],
            "largest count", st["max_contacts"])
        assert st["steps_done"] == 0
        assert np.array_equal(sim.read("pos"), x0)   # the step was abandoned before integration
        largest.append(st["max_contacts"])
        sim.close()
    assert largest[0] == largest[1] > 4
