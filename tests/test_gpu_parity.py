"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars (from the method's definition and the reading of the paper):
  * cell indices and contact lists: bit-exact;
  * one step from the same state: world impulses and velocity changes within
    1e-5 of the largest impulse (resp. velocity change);
  * multi-step runs (chaotic): statistics within 1%.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2306_01369_amd import gg, scenes

pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _sim_from_state(x, v, r, bodies, **kw):
    return gg.Sim(np.asarray(x, np.float32), np.asarray(v, np.float32), np.asarray(r, np.float32), bodies, **kw)


def _oracle_from_state(x, v, r, bodies, **kw):
    return O.Oracle(np.asarray(x, np.float32).astype(np.float64), np.asarray(v, np.float32).astype(np.float64),
                    np.asarray(r, np.float32), bodies, **kw)


def _compare_one_step(x, v, r, bodies, label, env_offsets=None, **kw):
    """Run one step on both sides from the same binary32 state and compare."""
    say(label, "n =", len(x), "bodies =", len(bodies))
    sim = _sim_from_state(x, v, r, bodies, diagnostics=True, env_offsets=env_offsets, **kw)
    ok_kw = {k: kw[k] for k in ("dt", "alpha", "mu", "n_iters", "gravity", "mass_split", "hash_size", "cell_size",
                                "cyclic_z")
             if k in kw}
    if env_offsets is not None:
        ok_kw["env"] = np.repeat(np.arange(len(env_offsets) - 1), np.diff(env_offsets)).astype(np.int32)
        if "hash_size" not in ok_kw:
            say(label, "(per-environment tables)")
    orc = _oracle_from_state(x, v, r, bodies, **ok_kw)
    sim.step(1)
    d = orc.step(detail=True)
    pairs = sim.read("contacts")
    assert pairs.shape == d["pairs"].shape, (label, pairs.shape, d["pairs"].shape)
    np.testing.assert_array_equal(pairs, d["pairs"])
    st = sim.stats()
    assert st["n_pp"] == d["n_pp"] and st["n_pb"] == d["n_pb"]
    assert st["candidates"] == d["candidates"]
    P = sim.read("impulses").astype(np.float64)
    if len(P):
        scale = np.abs(d["impulses"]).max()
        err = np.abs(P - d["impulses"]).max() / scale
        say(label, "contacts", len(P), "impulse rel err", err)
        assert err <= TOL, (label, err)
    dv = sim.read("dv").astype(np.float64)
    dscale = max(np.abs(d["dv"]).max(), 1e-30)
    errv = np.abs(dv - d["dv"]).max() / dscale
    say(label, "dv rel err", errv)
    assert errv <= TOL, (label, errv)
    # the new state: v' = v + dt g + dv, x' = x + dt v'
    vel = sim.read("vel").astype(np.float64)
    vs = max(np.abs(orc.v).max(), 1e-30)
    assert np.abs(vel - orc.v).max() <= TOL * vs + 1e-7
    pos = sim.read("pos").astype(np.float64)
    assert np.abs(pos - orc.x).max() <= 1e-6 * max(1.0, np.abs(orc.x).max())
    sim.close()
    return d


# ------------------------------------------------------------------ cell index

@pytest.mark.parametrize("case", ["drop", "random-negative", "nonpow2", "table1"])
def test_cell_index_bit_exact(case):
    rng = np.random.default_rng(11)
    if case == "drop":
        s = scenes.drop_scene()
        x, r, kw = s.x, s.radius, {}
    elif case == "random-negative":
        x, r = scenes.random_spheres(5000, ((-1.2, 0.3), (-0.5, 0.9), (-2.0, -0.1)), 0.003, rng)
        kw = {}
    elif case == "nonpow2":
        x, r = scenes.random_spheres(3001, ((-0.2, 0.3), (0, 0.2), (0, 0.2)), 0.003, rng)
        kw = {"hash_size": 1000}
    else:
        x, r = scenes.random_spheres(700, ((0, 0.05), (0, 0.05), (0, 0.05)), 0.003, rng)
        kw = {"hash_size": 1}
    say("cell index", case, len(x))
    sim = gg.Sim(x, np.zeros_like(x), r, gravity=(0, 0, 0), **kw)
    sim.step(1)
    h = sim.read("cell_index")
    c, inv_c = O.default_cell(r)
    nh = kw.get("hash_size", 2 * len(x))
    _, h_ref = O.cell_index(x, inv_c, nh)
    np.testing.assert_array_equal(h, h_ref)


def test_cell_index_full_scoop_bed():
    s = scenes.scoop_scene()
    say("cell index scoop", s.n)
    sim = gg.scene_sim(s)
    sim.step(1)
    h = sim.read("cell_index")
    c, inv_c = O.default_cell(s.radius)
    _, h_ref = O.cell_index(s.x, inv_c, 2 * s.n)
    np.testing.assert_array_equal(h, h_ref)


# ------------------------------------------------------------------ one step

def test_one_step_drop_pile():
    s = scenes.drop_scene()
    orc = O.scene_oracle(s)
    for _ in range(45):       # the lattice has landed and piles up: dense contacts
        orc.step()
    x = orc.x.astype(np.float32)
    v = orc.v.astype(np.float32)
    d = _compare_one_step(x, v, s.radius, s.bodies, "drop-pile", dt=s.dt, alpha=s.alpha, mu=s.mu,
                          n_iters=s.n_iters)
    assert d["n_pp"] > 2000


@pytest.mark.parametrize("iters", [1, 2, 5, 20])
def test_one_step_random_cluster_iterations(iters):
    rng = np.random.default_rng(3)
    x, r = scenes.random_spheres(3000, ((0, 0.08), (0, 0.08), (0, 0.08)), 0.004, rng, r_jitter=0.25)
    v = (rng.normal(size=(3000, 3)) * 0.2).astype(np.float32)
    _compare_one_step(x, v, r, [], f"cluster-iters{iters}", gravity=(0, 0, 0), n_iters=iters, mu=0.3)


def test_one_step_bed_with_tools():
    # a resting bed with a box and a capsule pressed into it, moving and rotating
    s = scenes.column_scene(n=6000, r=0.004)
    rng = np.random.default_rng(5)
    top = float(s.x[:, 2].max())
    box = scenes.box_tool((0.02, 0.03, top - 0.004), (0.012, 0.02, 0.01), nu=(0.1, 0, -0.05),
                          omega=(0.3, -0.2, 1.0), R=scenes.random_rotation(rng))
    cap = scenes.capsule_tool((0.045, 0.04, top - 0.002), 0.008, 0.02, nu=(-0.1, 0.05, 0),
                              omega=(0, 2.0, 0), R=scenes.random_rotation(rng))
    bodies = s.bodies + [box, cap]
    d = _compare_one_step(s.x, s.v, s.radius, bodies, "bed-tools", mu=0.5)
    assert d["n_pb"] > 100


def test_one_step_without_mass_splitting():
    # Without mass splitting the Jacobi sweep is expansive in dense packs (the
    # oracle alone shows iterates growing ~800x over 20 sweeps on this column and
    # diverging on the cluster), so binary32 and FP64 separate; three sweeps keep
    # the comparison well conditioned.
    s = scenes.column_scene(n=2000, r=0.005)
    _compare_one_step(s.x, s.v, s.radius, s.bodies, "plain-mass-column", mass_split=False, n_iters=3)
    rng = np.random.default_rng(3)
    x, r = scenes.random_spheres(3000, ((0, 0.08), (0, 0.08), (0, 0.08)), 0.004, rng, r_jitter=0.25)
    v = (rng.normal(size=(3000, 3)) * 0.2).astype(np.float32)
    _compare_one_step(x, v, r, [], "plain-mass-cluster", gravity=(0, 0, 0), n_iters=3, mu=0.3, mass_split=False)


def test_one_step_full_scoop_bed():
    s = scenes.scoop_scene()
    # the tool starts 1 cm above the bed: lower it into the bed for this check
    bodies = [dict(b) for b in s.bodies]
    bodies[-1] = dict(bodies[-1])
    bodies[-1]["t"] = np.asarray(bodies[-1]["t"]) - np.array([0.0, 0.0, 0.02])
    d = _compare_one_step(s.x, s.v, s.radius, bodies, "scoop-1M", dt=s.dt, alpha=s.alpha, mu=s.mu,
                          n_iters=s.n_iters)
    assert d["n_pp"] > 2.5 * s.n


def test_one_step_settled_bed_with_the_tool_in_it():
    # the scoop bed's recipe (pour from a loose lattice, frictionless
    # compaction, settling until max |v| < 1 mm/s) on a 11,200-grain
    # footprint, settled by the oracle; the tool follows its scoop path into
    # the bed for 130 steps (oracle), then one step from that state
    from settled import SIDE, small_settled_bed
    pour, x, v, steps, vmax = small_settled_bed()
    r = float(pour.radius[0])
    surface = scenes.surface_height(x, r)
    tool = scenes.scoop_tool(surface, x=0.03, y=SIDE / 2, half=(0.01, 0.02, 0.05))
    bodies = pour.bodies + [tool]
    kw = dict(dt=pour.dt, alpha=pour.alpha, mu=pour.mu, n_iters=pour.n_iters)
    say("settled bed: settle steps", steps, "max speed", vmax)
    orc = O.Oracle(x, v, pour.radius, bodies, **kw)
    tb = len(bodies) - 1
    for _ in range(120):
        orc.step()
    # the tool meets grains on and off (they are pushed ahead of it): take the
    # first state from which it starts a step with at least 20 contacts
    for k in range(80):
        state = (orc.x.copy(), orc.v.copy(), orc.body_pose(tb))
        d = orc.step(detail=True)
        if np.sum(d["pairs"][d["n_pp"]:, 1] == tb) >= 20:
            break
    xs, vs, (Rm, tm) = state
    say("settled bed: tool path step", 120 + k)
    moved = [dict(b) for b in bodies]
    moved[-1]["R"], moved[-1]["t"] = np.asarray(Rm, float), np.asarray(tm, float)
    d = _compare_one_step(xs, vs, pour.radius, moved, "settled-11k", **kw)
    pb = d["pairs"][d["n_pp"]:]
    assert d["n_pp"] > 2.5 * pour.n and np.sum(pb[:, 1] == tb) >= 20


def test_one_step_full_batched_beds():
    # all 256 environments (9.7M grains) in the launch configuration the
    # benchmark times, capsules lowered 1 cm into their beds
    s = scenes.batched_scene(n_steps=1)
    bodies = [dict(b) for b in s.bodies]
    for b in bodies:
        if b["shape"] == "capsule":
            b["t"] = np.asarray(b["t"]) - np.array([0.0, 0.0, 0.01])
    d = _compare_one_step(s.x, s.v, s.radius, bodies, "batched-256", env_offsets=s.env_offsets, dt=s.dt,
                          alpha=s.alpha, mu=s.mu, n_iters=s.n_iters)
    assert d["n_pb"] > 256 and d["n_pp"] > 2 * s.n


def test_one_step_large_polydisperse_bed():
    # 4,194,304 polydisperse grains, 64 sweeps, box and capsule tools pressed
    # into the bed; the start is the large bed's layered recipe with the layers
    # 5% closer than the sum of their largest radii, so vertically aligned
    # grains of adjacent layers overlap (a state built without simulating;
    # the layers float 2% above the floor, so body contacts are the tools');
    # the launch shape is the benchmark's
    s = scenes.large_scene(gap=0.95)
    x, v = s.x, s.v
    surface = float(np.percentile(x[:, 2] + s.radius, 99.5))
    bodies = [dict(b) for b in s.bodies]
    for b in bodies[-2:]:
        low = b["params"][2] if b["shape"] == "box" else b["params"][0]
        b["t"] = np.array([b["t"][0], b["t"][1], surface - 0.005 + low])
    d = _compare_one_step(x, v, s.radius, bodies, "large-4M", dt=s.dt, alpha=s.alpha, mu=s.mu,
                          n_iters=s.n_iters)
    assert d["n_pp"] > 0.02 * s.n and d["n_pb"] > 200


# ------------------------------------------------------------------ multi-step

def _stats(x, pairs, n):
    deg = np.bincount(np.asarray(pairs).ravel(), minlength=n) if len(pairs) else np.zeros(n)
    return {"com": x.mean(0), "coord": deg.mean()}


def test_drop_100_steps_statistics():
    s = scenes.drop_scene()
    say("drop 100 steps")
    sim = gg.scene_sim(s)
    sim.step(100)
    orc = O.scene_oracle(s)
    for _ in range(99):
        orc.step()
    d = orc.step(detail=True)
    xg = sim.read("pos").astype(np.float64)
    pg = sim.read("contacts")
    pp_g = pg[:sim.stats()["n_pp"]]
    pp_o = d["pairs"][:d["n_pp"]]
    sg, so = _stats(xg, pp_g, s.n), _stats(orc.x, pp_o, s.n)
    say("com gpu", sg["com"], "oracle", so["com"], "coord", sg["coord"], so["coord"])
    np.testing.assert_allclose(sg["com"], so["com"], rtol=0.01)
    assert abs(sg["coord"] - so["coord"]) <= 0.01 * so["coord"]


def _bed_statistics(x, x0, r, pairs, n_pp, side, surface, c):
    """Centre of mass, packing fraction of a central sub-box (3 cells from the
    walls, the floor and the surface), mean coordination number (pair contacts
    per grain) and the fraction of grains displaced by more than a radius."""
    lo = np.array([3 * c, 3 * c, 3 * c])
    hi = np.array([side - 3 * c, side - 3 * c, surface - 3 * c])
    inside = np.all((x >= lo) & (x <= hi), axis=1)
    vol = (4.0 / 3.0) * np.pi * np.sum(r[inside].astype(np.float64) ** 3)
    deg = np.bincount(np.asarray(pairs[:n_pp]).ravel(), minlength=len(x))
    moved = np.linalg.norm(x - x0, axis=1) > r
    return {"com": x.mean(0), "phi": vol / np.prod(hi - lo), "coord": deg.mean(), "displaced": moved.mean()}


def test_tool_in_bed_100_steps_statistics():
    # the scoop bed's recipe at 20,000 grains with a box tool ploughing 2 cm
    # into it: statistics after 100 chaotic steps within 1%
    template = scenes.Scene("scoop", np.zeros((1, 3), np.float32), np.zeros((1, 3), np.float32),
                            np.full(1, 0.002, np.float32))
    base = scenes.scaled(template, 20000)
    r = float(base.radius[0])
    side = max(0.05, np.sqrt(base.n / 10.0) * 2 * r)      # the recipe's footprint
    surface = scenes.surface_height(base.x, r)
    tool = scenes.box_tool((0.05, side / 2, surface + 0.002 + 0.1), (0.025, 0.05, 0.1),
                           nu=(0.3 * np.cos(np.pi / 4), 0.0, -0.3 * np.sin(np.pi / 4)))
    bodies = base.bodies + [tool]
    say("tool in bed 100 steps: n", base.n, "side", side)
    sim = gg.Sim(base.x, base.v, base.radius, bodies)
    sim.step(100)
    orc = O.Oracle(base.x.astype(np.float64), base.v.astype(np.float64), base.radius, bodies)
    for _ in range(99):
        orc.step()
    d = orc.step(detail=True)
    c, _ = O.default_cell(base.radius)
    x0 = base.x.astype(np.float64)
    sg = _bed_statistics(sim.read("pos").astype(np.float64), x0, base.radius, sim.read("contacts"),
                         sim.stats()["n_pp"], side, surface, c)
    so = _bed_statistics(orc.x, x0, base.radius, d["pairs"], d["n_pp"], side, surface, c)
    say("gpu", sg)
    say("oracle", so)
    np.testing.assert_allclose(sg["com"], so["com"], rtol=0.01)
    for k in ("phi", "coord", "displaced"):
        assert abs(sg[k] - so[k]) <= 0.01 * abs(so[k]), k
    assert so["displaced"] > 0.02 and d["n_pb"] > 0


def test_determinism_bitwise():
    s = scenes.drop_scene()
    say("determinism")
    outs = []
    for _ in range(2):
        sim = gg.scene_sim(s)
        sim.step(60)
        outs.append((sim.read("pos"), sim.read("vel"), sim.read("impulses")))
        sim.close()
    for a, b in zip(outs[0], outs[1]):
        assert a.tobytes() == b.tobytes()


def test_pair_impulse_copies_are_equal_and_opposite():
    # momentum: g = 0, no bodies, the total momentum is conserved to binary32 rounding
    rng = np.random.default_rng(9)
    x, r = scenes.loose_lattice(4000, 0.005, (0, 0, 0), rng, spacing_factor=2.0, jitter_frac=0.1)
    v = (rng.normal(size=(4000, 3))).astype(np.float32)
    say("momentum")
    sim = gg.Sim(x, v, r, gravity=(0, 0, 0), mu=0.4)
    m = 2500 * 4 / 3 * np.pi * r.astype(np.float64) ** 3
    p0 = (m[:, None] * v).sum(0)
    sim.step(5)
    v1 = sim.read("vel").astype(np.float64)
    p1 = (m[:, None] * v1).sum(0)
    scale = (m[:, None] * np.abs(v)).sum()
    assert np.abs(p1 - p0).max() <= 1e-6 * scale
    assert sim.stats()["n_pp"] > 1000


# ------------------------------------------------------------------ edge cases

@pytest.mark.parametrize("n", [0, 1, 63, 65, 1000, 4097])
def test_small_and_ragged_sizes(n):
    say("ragged", n)
    rng = np.random.default_rng(n)
    x, r = scenes.loose_lattice(n, 0.004, (0.004, 0.004, 0.0039), rng)
    v = (rng.normal(size=(n, 3)) * 0.05).astype(np.float32)
    side = 0.004 * 2.02 * math.ceil(n ** (1 / 3)) if n else 0.05
    bodies = scenes.walled_box(0, side, 0, side)
    if n == 0:
        sim = gg.Sim(x, v, r, bodies)
        sim.step(3)
        assert sim.read("pos").shape == (0, 3)
        assert sim.stats()["steps_done"] == 3
        return
    _compare_one_step(x, v, r, bodies, f"ragged-{n}")


def test_capacity_overflow_aborts_before_integration():
    s = scenes.column_scene(n=1000, r=0.005)
    say("capacity")
    sim = gg.scene_sim(s, max_contacts=3)
    x0 = sim.read("pos")
    with pytest.raises(gg.CapacityError):
        sim.step(4)
    st = sim.stats()
    assert st["steps_done"] == 0 and st["last_status"] == gg.GG_ERR_CAPACITY
    np.testing.assert_array_equal(sim.read("pos"), x0)
    assert sim.read("contacts").shape == (0, 2)


def test_capacity_overflow_after_some_steps_keeps_completed_steps():
    # free fall into a floor: the first steps have no contacts, later ones do
    s = scenes.drop_scene()
    say("capacity-late")
    sim = gg.scene_sim(s, max_contacts=1)
    with pytest.raises(gg.CapacityError):
        sim.step(60)
    st = sim.stats()
    assert 0 < st["steps_done"] < 60
    orc = O.scene_oracle(s)
    for _ in range(st["steps_done"]):
        orc.step()
    assert np.abs(sim.read("pos") - orc.x).max() < 1e-5


def test_position_leaving_hash_range_is_reported():
    x = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]], np.float32)
    v = np.array([[0.0, 0.0, 0.0], [2e12, 0.0, 0.0]], np.float32)
    r = np.full(2, 0.005, np.float32)
    say("nonfinite")
    sim = gg.Sim(x, v, r, gravity=(0, 0, 0))
    with pytest.raises(gg.GGError) as e:
        sim.step(3)
    assert e.value.status == gg.GG_ERR_NONFINITE
    assert sim.stats()["steps_done"] == 1


def test_multi_env_contacts_and_buckets():
    rng = np.random.default_rng(21)
    counts = [300, 1, 0, 700, 455]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    xs = []
    for e, c in enumerate(counts):
        xe, _ = scenes.loose_lattice(c, 0.004, (0.004, 0.004, 0.0039), rng, spacing_factor=2.0, jitter_frac=0.1)
        xs.append(xe)
    x = np.concatenate(xs).astype(np.float32)      # all envs overlap in space
    r = np.full(len(x), 0.004, np.float32)
    v = np.zeros_like(x)
    env = np.repeat(np.arange(len(counts)), counts).astype(np.int32)
    bodies = []
    for e in range(len(counts)):
        bodies += scenes.walled_box(0, 0.08, 0, 0.08, env=e)
    say("multi-env", counts)
    sim = gg.Sim(x, v, r, bodies, env_offsets=off, diagnostics=True)
    sim.step(1)
    # buckets: env offset + Eq. (6) value in a table of 2 n_e buckets
    c, inv_c = O.default_cell(r)
    nh = np.array([max(1, 2 * cnt) for cnt in counts], np.int64)
    boff = np.concatenate([[0], np.cumsum(nh)[:-1]])
    _, h_ref = O.cell_index(x, inv_c, 1, bucket_offset=boff[env], env_n_h=nh[env])
    np.testing.assert_array_equal(sim.read("cell_index"), h_ref)
    orc = O.Oracle(x.astype(np.float64), v.astype(np.float64), r, bodies, env=env)
    d = orc.step(detail=True)
    np.testing.assert_array_equal(sim.read("contacts"), d["pairs"])
    P = sim.read("impulses")
    assert np.abs(P - d["impulses"]).max() <= TOL * np.abs(d["impulses"]).max()


def test_device_tensors_in_and_out():
    torch = pytest.importorskip("torch")
    s = scenes.drop_scene()
    say("device tensors")
    dev = torch.device("cuda:0")
    x = torch.from_numpy(s.x).to(dev)
    v = torch.from_numpy(s.v).to(dev)
    r = torch.from_numpy(s.radius).to(dev)
    stream = torch.cuda.current_stream().cuda_stream
    sim = gg.Sim(x, v, r, s.bodies, stream=stream)
    sim.step(30)
    out = torch.empty((s.n, 3), dtype=torch.float32, device=dev)
    sim.read("pos", out=out)
    ref = gg.scene_sim(s)
    ref.step(30)
    assert out.cpu().numpy().tobytes() == ref.read("pos").tobytes()


def test_twists_per_step_move_the_tool():
    s = scenes.column_scene(n=1500, r=0.005)
    top = float(s.x[:, 2].max())
    tool = scenes.box_tool((0.04, 0.04, top + 0.05), (0.01, 0.01, 0.01))
    bodies = s.bodies + [tool]
    say("twists")
    sim = gg.Sim(s.x, s.v, s.radius, bodies)
    tw = np.zeros((10, len(bodies), 6), np.float32)
    tw[:, -1, 2] = -5.0                      # tool moves down 5 cm in 10 steps, into the bed
    sim.step(10, twists=tw)
    orc = O.Oracle(s.x.astype(np.float64), s.v.astype(np.float64), s.radius, bodies)
    for k in range(10):
        orc.set_twists(tw[k])
        orc.step()
    assert np.abs(sim.read("pos") - orc.x).max() < 1e-4


# ------------------------------------------------- layout independence

def _run_bits(scene, steps, **kw):
    sim = gg.scene_sim(scene, **kw)
    sim.step(steps)
    out = (sim.read("pos").tobytes(), sim.read("vel").tobytes(), sim.read("contacts").tobytes(),
           sim.read("impulses").tobytes(), sim.read("cell_index").tobytes())
    st = sim.stats()
    sim.close()
    return out, st


@pytest.mark.parametrize("reorder", [1, 3, -1])
def test_results_independent_of_internal_order(reorder):
    # the Z-order re-sort changes only memory layout: every output is bitwise
    # the same for any re-sort interval, including never
    s = scenes.drop_scene()
    say("reorder", reorder)
    ref, _ = _run_bits(s, 50, reorder_every=8)
    got, _ = _run_bits(s, 50, reorder_every=reorder)
    assert got == ref


def test_tile_and_per_particle_detection_agree_bitwise():
    s = scenes.column_scene(n=5000, r=0.004)
    rng = np.random.default_rng(1)
    s.x = s.x[rng.permutation(s.n)]            # caller order not spatial
    say("tile vs fallback")
    tiled, st_t = _run_bits(s, 12)
    per_particle, st_f = _run_bits(s, 12, tile_max_cells=27)
    assert st_t["detect_fallback"] < st_f["detect_fallback"]
    assert st_f["detect_fallback"] == st_f["detect_items"] > 0
    assert tiled == per_particle


def test_larger_cell_keeps_contacts_and_parity():
    # the autotuner may grow the cell: same contact set, impulses within the
    # one-step bar of the oracle (only the summation order changes)
    s = scenes.column_scene(n=3000, r=0.004)
    c, _ = O.default_cell(s.radius)
    say("cell size x1.25")
    _compare_one_step(s.x, s.v, s.radius, s.bodies, "cell-x1.25", cell_size=float(np.float32(1.25 * c)))


def test_crowded_cells_one_step():
    # cells four times the default hold about 90 grains each: in the key
    # kernel runs of equal buckets span whole wavefronts (one atomic per run
    # of lanes), and detection takes the per-particle path; contacts exact,
    # impulses within the one-step bar of the oracle
    rng = np.random.default_rng(5)
    x, r = scenes.random_spheres(20000, ((0, 0.12), (0, 0.12), (0, 0.12)), 0.002, rng, r_jitter=0.25)
    v = (rng.normal(size=(20000, 3)) * 0.1).astype(np.float32)
    c, _ = O.default_cell(r)
    say("crowded cells: cell x4")
    d = _compare_one_step(x, v, r, [], "crowded-cells", gravity=(0, 0, 0), n_iters=5, mu=0.3,
                          cell_size=float(np.float32(4 * c)))
    assert d["n_pp"] > 10000


@pytest.mark.parametrize("threads,shift", [(64, 5), (64, 6), (256, 7)])
def test_detection_workgroup_size_keeps_results_bitwise(threads, shift):
    s = scenes.column_scene(n=5000, r=0.004)
    rng = np.random.default_rng(2)
    s.x = s.x[rng.permutation(s.n)]
    say("detection workgroup", threads, shift)
    ref, _ = _run_bits(s, 12)
    got, st = _run_bits(s, 12, tile_threads=threads, tile_node_shift=shift)
    assert got == ref
    assert st["detect_items"] > 0


def test_autotuned_launch_shape_keeps_results_bitwise(tmp_path, monkeypatch):
    from paper_2306_01369_amd import autotune
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "tune.json"))
    s = scenes.column_scene(n=6000, r=0.004)
    say("autotune")
    params = autotune.tune(s.x, s.v, s.radius, s.bodies, steps=2, warmup=1)
    again = autotune.tune(s.x, s.v, s.radius, s.bodies)      # from the cache
    assert again == params
    say("tuned", params)
    ref, _ = _run_bits(s, 15)
    # the tuned shape (the defaults when none beat them) and a candidate shape
    cand = autotune.candidates(autotune.particles_per_cell(s.x, s.radius))[0]
    for shape in (params, cand):
        got, st = _run_bits(s, 15, **shape)
        if shape.get("fused"):             # the fused step agrees to rounding
            pos_r = np.frombuffer(ref[0], np.float32)
            pos_g = np.frombuffer(got[0], np.float32)
            assert np.abs(pos_r - pos_g).max() <= 1e-6
            continue
        assert got[:4] == ref[:4], shape   # the bucket ids differ when n_h was tuned
        if "hash_size" not in shape:
            assert got == ref, shape


# ------------------------------------------------- graph replay, hash size

def _bits(sim):
    return sim.read("pos").tobytes(), sim.read("vel").tobytes()


def test_graph_replay_matches_direct_launches():
    # each call replays a captured launch sequence (captured on first use of a
    # step count / re-sort phase / buffer parity); every replay must equal the
    # direct launches bit for bit, with unrelated device work between replays
    torch = pytest.importorskip("torch")
    s = scenes.column_scene(n=3000, r=0.004)
    top = float(s.x[:, 2].max())
    tool = scenes.box_tool((0.03, 0.03, top + 0.02), (0.01, 0.01, 0.01))
    bodies = s.bodies + [tool]
    say("graph replay")
    direct = gg.Sim(s.x, s.v, s.radius, bodies, reorder_every=4)
    graphed = gg.Sim(s.x, s.v, s.radius, bodies, reorder_every=4, graph=True)
    junk = torch.zeros(1 << 20, device="cuda:0")
    calls = [(5, None), (5, None), (3, None), (5, None), (8, "tw"), (8, "tw"), (5, "bodies"), (5, None)]
    for k, (steps, what) in enumerate(calls):
        tw = None
        if what == "tw":
            tw = np.zeros((steps, len(bodies), 6), np.float32)
            tw[:, -1, 2] = -0.5
        if what == "bodies":
            moved = dict(tool, t=tool["t"] + np.array([0.005, 0.0, 0.0]))
            bodies2 = s.bodies + [moved]
            direct.set_bodies(bodies2)
            graphed.set_bodies(bodies2)
        direct.step(steps, twists=tw)
        graphed.step(steps, twists=tw)
        junk.add_(1.0)
        torch.cuda.synchronize()
        assert _bits(graphed) == _bits(direct), f"call {k}"
        assert graphed.stats()["n_pp"] == direct.stats()["n_pp"]
    assert float(junk[0]) == len(calls)


def test_graph_replay_after_the_pose_staging_grows():
    # a longer call reallocates the per-step body records; a later short call
    # must not replay a launch captured before that (it would read the old
    # records): without re-sorts every call has the same re-sort phase and
    # buffer parity, so only the allocation epoch tells the captures apart
    s = scenes.column_scene(n=2000, r=0.004)
    top = float(s.x[:, 2].max())
    tool = scenes.box_tool((0.03, 0.03, top + 0.004), (0.01, 0.01, 0.01))
    bodies = s.bodies + [tool]
    say("graph replay after staging growth")
    direct = gg.Sim(s.x, s.v, s.radius, bodies, reorder_every=-1)
    graphed = gg.Sim(s.x, s.v, s.radius, bodies, reorder_every=-1, graph=True)
    for k, steps in enumerate((1, 4, 1, 1)):
        tw = np.zeros((steps, len(bodies), 6), np.float32)
        tw[:, -1, 2] = -0.3 - 0.1 * k
        direct.step(steps, twists=tw)
        graphed.step(steps, twists=tw)
        assert _bits(graphed) == _bits(direct), f"call {k}"


def test_graph_replay_multi_env():
    rng = np.random.default_rng(5)
    counts = [500, 0, 1200, 64]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    x = np.concatenate([scenes.loose_lattice(c, 0.004, (0.004, 0.004, 0.0039), rng, spacing_factor=2.0,
                                             jitter_frac=0.1)[0] for c in counts]).astype(np.float32)
    r = np.full(len(x), 0.004, np.float32)
    v = np.zeros_like(x)
    bodies = []
    for e in range(len(counts)):
        bodies += scenes.walled_box(0, 0.08, 0, 0.08, env=e)
    say("graph multi-env")
    direct = gg.Sim(x, v, r, bodies, env_offsets=off)
    graphed = gg.Sim(x, v, r, bodies, env_offsets=off, graph=True)
    for k in range(4):
        direct.step(6)
        graphed.step(6)
        assert _bits(graphed) == _bits(direct), f"call {k}"


def test_batched_environments_equal_separate_simulations():
    # each environment of a batch, stepped on its own (one environment, its
    # own bodies and twists), gives the same bits: the batched form adds no
    # arithmetic, and the work queues of detection only distribute the work
    # items (which workgroup takes an item changes no result)
    sc = scenes.batched_scene(n_envs=3, lo=2000, hi=6000, n_steps=12)
    off = sc.env_offsets
    kw = dict(dt=sc.dt, alpha=sc.alpha, mu=sc.mu, n_iters=sc.n_iters)
    say("batched vs separate", np.diff(off).tolist())
    batch = gg.Sim(sc.x, sc.v, sc.radius, sc.bodies, env_offsets=off, **kw)
    batch.step(12, twists=sc.twists)
    xb, vb = batch.read("pos"), batch.read("vel")
    assert batch.stats()["detect_queues"] == 1
    batch.close()
    env_of_body = np.array([b.get("env", 0) for b in sc.bodies])
    for e in range(len(off) - 1):
        sl = slice(int(off[e]), int(off[e + 1]))
        idx = np.nonzero(env_of_body == e)[0]
        bodies = [dict(sc.bodies[b], env=0) for b in idx]
        one = gg.Sim(sc.x[sl], sc.v[sl], sc.radius[sl], bodies, **kw)
        one.step(12, twists=np.ascontiguousarray(sc.twists[:, idx]))
        assert np.array_equal(one.read("pos"), xb[sl]), e
        assert np.array_equal(one.read("vel"), vb[sl]), e
        one.close()


def test_detection_statistics_sum_over_workgroups_and_steps():
    # each detection workgroup stores its own counts and one small kernel sums
    # them: a call of several steps reports the last step's counts and the sum
    # over its steps, equal to the same steps taken one call at a time
    sc = scenes.column_scene(n=6000, r=0.004)
    side = float(sc.x[:, 0].max())
    bodies = sc.bodies + [scenes.box_tool((side / 2, side / 2, float(sc.x[:, 2].max()) + 0.01),
                                          (0.01, 0.02, 0.03), nu=(0.0, 0.0, -0.5))]
    kw = dict(dt=sc.dt, alpha=sc.alpha, mu=sc.mu, n_iters=sc.n_iters)
    say("statistics", sc.n)
    one = gg.Sim(sc.x, sc.v, sc.radius, bodies, **kw)
    per_step = []
    for _ in range(8):
        one.step(1)
        st = one.stats()
        assert st["contacts_summed"] == st["n_pp"] + st["n_pb"]
        per_step.append((st["n_pp"], st["n_pb"], st["candidates"], st["max_contacts"]))
    one.close()
    assert per_step[-1][0] > 1000 and per_step[-1][1] > 0
    many = gg.Sim(sc.x, sc.v, sc.radius, bodies, **kw)
    many.step(8)
    st = many.stats()
    many.close()
    assert (st["n_pp"], st["n_pb"], st["candidates"], st["max_contacts"]) == per_step[-1]
    assert st["contacts_summed"] == sum(a + b for a, b, _, _ in per_step)


def test_hash_table_size_changes_no_result():
    # partners are listed by (neighbour cell, original index), never by bucket,
    # so n_h (and with it bucket aliasing) changes only speed: outputs and the
    # candidate count are bitwise the same for any table size, down to n_h = 1
    s = scenes.drop_scene()
    say("hash size")
    ref, st_ref = _run_bits(s, 12)
    for nh in (1, 7, 4096, 3 * s.n + 1):
        got, st = _run_bits(s, 12, hash_size=nh)
        assert got[:4] == ref[:4], nh
        assert st["candidates"] == st_ref["candidates"], nh


# ------------------------------------------------- double build

def _f32(a):
    return float(np.float32(a))


def test_fp64_build_tracks_the_oracle_trajectory():
    # the double build computes what the FP64 oracle computes, up to FP64
    # rounding order: after 40 steps of a bed under a moving tool the binary32
    # readouts agree to their own rounding (the binary32 build drifts apart at
    # ~1e-5 m in the same run, since the dynamics amplify rounding)
    s = scenes.column_scene(n=2500, r=0.004)
    top = float(s.x[:, 2].max())
    tool = scenes.box_tool((0.03, 0.03, top + 0.011), (0.01, 0.01, 0.01), nu=(0.05, 0.0, -0.3))
    bodies = s.bodies + [tool]
    kw = dict(dt=_f32(1e-3), alpha=_f32(0.2), gravity=(0.0, 0.0, _f32(-9.81)))
    say("fp64 trajectory")
    sim = gg.Sim(s.x, s.v, s.radius, bodies, precision=1, diagnostics=True, **kw)
    orc = O.Oracle(s.x.astype(np.float64), s.v.astype(np.float64), s.radius, bodies, **kw)
    for k in range(40):
        sim.step(1)
        d = orc.step(detail=True)
        np.testing.assert_array_equal(sim.read("contacts"), d["pairs"], err_msg=f"step {k}")
    assert np.abs(sim.read("pos") - orc.x).max() <= 2e-8
    assert np.abs(sim.read("vel") - orc.v).max() <= 1e-6 * max(1.0, np.abs(orc.v).max())
    P = sim.read("impulses")
    assert np.abs(P - d["impulses"]).max() <= 1e-6 * np.abs(d["impulses"]).max()
    assert d["n_pb"] > 0


def test_fp64_build_multi_env_and_graph_replay():
    rng = np.random.default_rng(8)
    counts = [400, 900]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    x = np.concatenate([scenes.loose_lattice(c, 0.004, (0.004, 0.004, 0.0039), rng, spacing_factor=2.0,
                                             jitter_frac=0.1)[0] for c in counts]).astype(np.float32)
    r = np.full(len(x), 0.004, np.float32)
    v = np.zeros_like(x)
    bodies = scenes.walled_box(0, 0.08, 0, 0.08, env=0) + scenes.walled_box(0, 0.08, 0, 0.08, env=1)
    say("fp64 multi-env graph")
    direct = gg.Sim(x, v, r, bodies, env_offsets=off, precision=1)
    graphed = gg.Sim(x, v, r, bodies, env_offsets=off, precision=1, graph=True)
    for k in range(3):
        direct.step(9)
        graphed.step(9)
        assert _bits(graphed) == _bits(direct), f"call {k}"
    env = np.repeat(np.arange(2), counts).astype(np.int32)
    orc = O.Oracle(x.astype(np.float64), v.astype(np.float64), r, bodies, env=env, dt=_f32(1e-3),
                   alpha=_f32(0.2), gravity=(0.0, 0.0, _f32(-9.81)))
    sim = gg.Sim(x, v, r, bodies, env_offsets=off, precision=1, dt=_f32(1e-3), alpha=_f32(0.2),
                 gravity=(0.0, 0.0, _f32(-9.81)))
    for k in range(5):
        orc.step()
    sim.step(5)
    assert np.abs(sim.read("pos") - orc.x).max() <= 2e-8


# ------------------------------------------------- grid SDF bodies

def _bed_with_grid_tools(n=4000, seed=0):
    s = scenes.column_scene(n=n, r=0.004, seed=seed)
    top = scenes.surface_height(s.x, 0.004)
    rng = np.random.default_rng(seed + 7)
    bowl = scenes.grid_tool(scenes.bowl_grid(0.02, 0.004, 0.006, 512.0), (0.03, 0.03, top + 0.012),
                            R=scenes.random_rotation(rng), nu=(0.1, 0.0, -0.2), omega=(0.5, -1.0, 0.3))
    ball = scenes.grid_tool(scenes.ball_grid(0.01, 0.006, 512.0), (0.06, 0.05, top + 0.006),
                            nu=(0.0, 0.05, -0.1))
    return s, s.bodies + [bowl, ball]


def test_one_step_bed_with_grid_tools():
    s, bodies = _bed_with_grid_tools()
    d = _compare_one_step(s.x, s.v, s.radius, bodies, "grid tools")
    grid_contacts = int(np.sum(d["pairs"][d["n_pp"]:, 1] >= len(s.bodies)))
    say("grid-body contacts", grid_contacts)
    assert grid_contacts > 20


def test_grid_tools_over_steps_follow_the_oracle():
    # the double build tracks the oracle's contact sets and trajectory with
    # moving and spinning grid tools
    s, bodies = _bed_with_grid_tools(n=2500, seed=1)
    kw = dict(dt=float(np.float32(1e-3)), alpha=float(np.float32(0.2)), gravity=(0.0, 0.0, float(np.float32(-9.81))))
    say("grid tools, 25 steps, double build")
    sim = gg.Sim(s.x, s.v, s.radius, bodies, precision=1, **kw)
    orc = O.Oracle(s.x.astype(np.float64), s.v.astype(np.float64), s.radius, bodies, **kw)
    n_grid = 0
    for k in range(25):
        sim.step(1)
        d = orc.step(detail=True)
        np.testing.assert_array_equal(sim.read("contacts"), d["pairs"], err_msg=f"step {k}")
        n_grid += int(np.sum(d["pairs"][d["n_pp"]:, 1] >= len(s.bodies)))
    assert n_grid > 100
    assert np.abs(sim.read("pos") - orc.x).max() <= 2e-8


def test_grid_registration_is_validated():
    s, bodies = _bed_with_grid_tools(n=500)
    sim = gg.Sim(s.x, s.v, s.radius, bodies)
    good = bodies[-1]["grid"]
    bad = [dict(good, inv_spacing=0.0), dict(good, inv_spacing=float("nan")),
           dict(good, values=np.full((1, 4, 4), 0.1, np.float32)),
           dict(good, values=np.where(np.arange(good["values"].size).reshape(good["values"].shape) == 5, np.inf,
                                      good["values"]).astype(np.float32))]
    for g in bad:
        with pytest.raises(gg.GGError) as e:
            sim.set_grids([g])
        assert e.value.status == gg.GG_ERR_INVALID
    # a body naming a grid index that is not registered
    sim.set_grids([good])
    with pytest.raises(gg.GGError) as e:
        sim.set_bodies(s.bodies + [dict(bodies[-1], shape=3, params=[1.0, 0, 0, 0])])
    assert e.value.status == gg.GG_ERR_INVALID
    # the registered bodies still step
    sim.set_bodies(bodies)
    sim.step(2)



# ------------------------------------------------- many bodies, cyclic boundary

def test_one_step_gear_tower():
    # 16,384 grains flowing past 10 spinning grid gears in a grid tower: the
    # body boxes cull most SDF tests, and the contact list must still equal
    # the oracle's (which tests every body)
    s, cyc = scenes.gear_tower(n=16384, n_gears=10, seed=2)
    orc = O.Oracle(s.x.astype(np.float64), s.v.astype(np.float64), s.radius, s.bodies, cyclic_z=cyc)
    for _ in range(150):                 # develop the flow on the oracle
        orc.step()
    x = orc.x.astype(np.float32)
    v = orc.v.astype(np.float32)
    d = _compare_one_step(x, v, s.radius, s.bodies, "gear-tower", cyclic_z=cyc)
    per_body = np.bincount(d["pairs"][d["n_pp"]:, 1], minlength=len(s.bodies))
    say("gear-tower contacts per body", per_body.tolist())
    assert np.count_nonzero(per_body[1:]) >= 5


def test_cyclic_boundary_over_steps_follows_the_oracle():
    s, cyc = scenes.gear_tower(n=4096, n_gears=5, seed=3)
    kw = dict(dt=float(np.float32(1e-3)), alpha=float(np.float32(0.2)), gravity=(0.0, 0.0, float(np.float32(-9.81))))
    v0 = s.v.copy()
    v0[:, 2] = -1.5                      # start falling so grains cross the bottom cap
    say("cyclic boundary, double build")
    sim = gg.Sim(s.x, v0, s.radius, s.bodies, precision=1, cyclic_z=cyc, **kw)
    orc = O.Oracle(s.x.astype(np.float64), v0.astype(np.float64), s.radius, s.bodies, cyclic_z=cyc, **kw)
    for k in range(30):
        sim.step(1)
        d = orc.step(detail=True)
        np.testing.assert_array_equal(sim.read("contacts"), d["pairs"], err_msg=f"step {k}")
    x = sim.read("pos")
    assert np.abs(x - orc.x).max() <= 2e-8
    assert np.sum(orc.x[:, 2] > s.x[:, 2] + 0.1) > 10      # grains that crossed the bottom re-entered at the top


def test_body_poses_follow_the_twists():
    # the library advances poses in double (t += dt nu, R = Exp(dt [omega]x) R)
    # and reports them rounded once; the oracle's advance from the same binary32
    # pose, twists and step is the reference
    s = scenes.column_scene(n=500, r=0.004)
    Rm = scenes.random_rotation(np.random.default_rng(3))
    bodies = s.bodies + [scenes.capsule_tool((0.2, 0.2, 0.3), 0.02, 0.05, R=Rm)]
    sim = gg.Sim(s.x, s.v, s.radius, bodies)
    nb = len(bodies)
    rng = np.random.default_rng(1)
    tw = np.zeros((25, nb, 6), np.float32)
    tw[:, -1, :] = rng.uniform(-1, 1, (25, 6)).astype(np.float32)
    sim.step(25, twists=tw)
    got = sim.read("body_poses")
    assert got.shape == (nb, 3, 4)
    B = O.bodies_to_f32_pose(O.make_bodies(bodies), nb)
    lib = O.lib()
    dt = float(np.float32(1e-3))
    for k in range(25):
        for q in range(3):
            B[nb - 1].nu[q] = float(tw[k, -1, q])
            B[nb - 1].omega[q] = float(tw[k, -1, 3 + q])
        lib.ggo_advance_bodies(nb, B, dt)
    want = np.array([[[B[b].R[3 * r + c] for c in range(3)] + [B[b].t[r]] for r in range(3)] for b in range(nb)])
    say("body poses: max |diff|", float(np.abs(got - want).max()))
    assert np.abs(got - want).max() <= 1e-6
    assert np.array_equal(got[:-1], want[:-1].astype(np.float32))   # planes stay put
