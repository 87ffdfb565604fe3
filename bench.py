"""Throughput of the granular contact step on one MI355X.

Workload: 1,048,576 spheres (r = 2 mm) in a resting bed of a 1 x 1 m walled
box, a 0.05 x 0.1 x 0.2 m box tool moving at 0.2 m/s on a linear scoop path,
dt = 1 ms, 20 projected-Jacobi sweeps per step, mu = 0.5.  A step is one pass
of the whole hot path: cell keys, bucket sort, contact detection, 20 sweeps,
position update.  Inputs are resident in device memory before timing starts.

Prints one JSON line: particle-steps/s, the roofline of the dominant kernel
(one projected-Jacobi sweep) measured with HIP events on the library's stream,
and the FP64 oracle timed on this host's cores on a bounded sample.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (20 PJA iters) at 1M particles; batched & backward vs plain"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pja_traffic_scoop-1M.json")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pja_algorithmic_bytes(n, contacts):
    """Bytes one projected-Jacobi sweep must move: per contact its impulse
    read and written (12 + 12), both endpoint indices (8), normal (12),
    effective mass and bias (8) and the two endpoint iterates (12); per
    particle its iterate read and written (16 + 16)."""
    return 64.0 * contacts + 32.0 * n


def _code_only(text):
    """Source text without // comments and without blank space (comment and
    layout edits do not change the code the counters were taken on)."""
    import re
    text = re.sub(r"//[^\n]*", "", text)
    return re.sub(r"\s+", "", text)


def kernel_source_hash():
    """Hash of what sets k_pja's memory traffic: the kernel sources and the
    host function that launches the sweeps (its grid and arguments), code
    only."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2306_01369_amd/csrc/kernels.hip.h")) as f:
        h.update(_code_only(f.read()).encode())
    with open(os.path.join(ROOT, "paper_2306_01369_amd/csrc/gg.hip")) as f:
        host = f.read()
    a = host.index("void launch_sweeps(")
    h.update(_code_only(host[a:host.index("\n}\n", a)]).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per sweep from rocprofv3 FETCH_SIZE/WRITE_SIZE (scaled by a copy
    kernel's reading), if they were taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(scene, steps):
    import oracle as O
    orc = O.scene_oracle(scene)
    t0 = time.perf_counter()
    for _ in range(steps):
        orc.step()
    dt = time.perf_counter() - t0
    return {"value": scene.n * steps / dt, "unit": "particle-steps/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} steps of a 1,048,576-sphere resting bed of the same grains (r=2 mm, compressed "
                      "simple-cubic layers, ~3.1M contacts, 20 sweeps), FP64; the settled bed is the library's "
                      "output and is not given to the oracle"}


def copy_calibration(mib=512, reps=5):
    """A plain device copy of known size, for scaling rocprofv3 byte counters."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: {reps} copies of {mib} MiB")


def replay_ready(sim, steps, call):
    """Make calls of `steps` steps (call(steps)) until the next call starts in a
    re-sort phase and state-buffer parity already seen, so that it replays a
    graph captured earlier instead of capturing one inside a timed region.
    The library keys captures by (steps, re-sort phase, current state buffer);
    a re-sort at every step index divisible by the interval R swaps the buffers.
    Returns the number of steps made."""
    st = sim.stats()
    R, g0 = int(st["reorder_every"]), int(st["steps_total"])

    def state(g):
        return (0, 0) if R <= 0 else (g % R, ((g + R - 1) // R) % 2)
    seen, g = set(), g0
    while state(g) not in seen:
        seen.add(state(g))
        call(steps)
        g += steps
    return g - g0


def bench_batched(args, n_envs=256, steps=None, plain_steps=None):
    """n_envs (256) independent environments of U{8192..65536} spheres stepped
    in one launch sequence, against the same environments stepped one by one."""
    from paper_2306_01369_amd import gg, scenes
    import torch
    if steps is None:
        steps = args.steps if args.steps_given else 100
    if plain_steps is None:
        plain_steps = args.plain_steps
    log(f"generating {n_envs} batched environments")
    # the timed call (a multiple of twice the re-sort interval, 16 here, so every
    # call starts in the same re-sort phase and buffer parity) replays the graph
    # captured by the call before it; both the batched and the plain loop are
    # timed from step 128
    steps = 32 * max(1, steps // 32)
    sc = scenes.batched_scene(n_envs=n_envs, n_steps=128 + steps + max(8, plain_steps))
    n = sc.n
    tw = np.ascontiguousarray(sc.twists)
    kw = dict(dt=sc.dt, alpha=sc.alpha, mu=sc.mu, n_iters=sc.n_iters, env_offsets=sc.env_offsets)
    sim = gg.Sim(sc.x, sc.v, sc.radius, sc.bodies, graph=True, **kw)
    at = [0]

    def call(k):
        sim.step(k, twists=tw[at[0]:at[0] + k])
        at[0] += k
    while at[0] + steps < 128:
        call(32)
    call(steps)   # captures the graph the timed call replays (calls of multiples of
    warm = at[0]  # 32 steps all start in re-sort phase 0 with the same state buffer)
    prof = gg.Sim(sim.read("pos"), sim.read("vel"), sc.radius, sc.bodies, profile=True, **kw)
    torch.cuda.synchronize()
    log(f"batched: n={n}, timing {steps} steps (one graph launch)")
    t0 = time.perf_counter()
    call(steps)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    sim.close()
    # phase split from a profiled copy (events between phases; not the timed run)
    prof.step(5, twists=tw[at[0] - steps:at[0] - steps + 5])
    st = prof.stats()
    prof.close()
    # plain loop: every environment its own simulation, stepped in turn
    n_envs = len(sc.env_offsets) - 1
    plain_steps = max(1, min(steps, plain_steps))
    sims = []
    nb_env = len(sc.bodies) // n_envs
    for e in range(n_envs):
        a, b = int(sc.env_offsets[e]), int(sc.env_offsets[e + 1])
        bodies = [dict(bd, env=0) for bd in sc.bodies[e * nb_env:(e + 1) * nb_env]]
        sims.append((gg.Sim(sc.x[a:b], sc.v[a:b], sc.radius[a:b], bodies, dt=sc.dt, alpha=sc.alpha, mu=sc.mu,
                            n_iters=sc.n_iters, graph=True), np.ascontiguousarray(tw[:, e * nb_env:(e + 1) * nb_env])))
    # one-step calls: warm-up calls capture the graph of every re-sort phase and
    # state-buffer parity, so the timed calls replay
    made = []
    for sm, t in sims:
        pos = [0]

        def one(k, sm=sm, t=t, pos=pos):
            sm.step(k, twists=t[pos[0]:pos[0] + k])
            pos[0] += k
        for _ in range(warm):      # every (re-sort phase, buffer parity) is captured by step 64
            one(1)
        made.append(pos[0])
    torch.cuda.synchronize()
    log(f"plain loop: {n_envs} sims, timing {plain_steps} steps")
    t0 = time.perf_counter()
    for k in range(plain_steps):
        for (sm, t), m in zip(sims, made):
            sm.step(1, twists=t[m + k:m + k + 1])
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) * steps / plain_steps
    for sm, _ in sims:
        sm.close()
    value = n * steps / t_batched
    return {
        "metric": f"batched particle-steps/s ({n_envs} envs, 20 PJA iters)",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": 1e3 * t_batched / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched: {n_envs} walled beds of U{{8192..65536}} spheres r=3mm, capsule tools with "
                               "random piecewise-constant twists, dt=1 ms, 20 PJA sweeps",
                   "n": n, "n_envs": n_envs, "plain_loop_steps_timed": plain_steps,
                   "launch": "whole call as one captured HIP graph; the plain loop replays one graph per "
                             "environment and step"},
        "speedup_vs_plain_loop": t_plain / t_batched,
        "plain_loop_particle_steps_per_s": n * steps / t_plain,
        "phases_ms_per_step_profiled": {"keys_sort_detect": st["ms_detect"] / 5, "pja": st["ms_pja"] / 5,
                                        "integrate": st["ms_integrate"] / 5},
        "detect_fallback_items": st["detect_fallback"], "detect_items": st["detect_items"],
    }


def bench_drop(args):
    """4096 spheres dropped into a 0.2 m box (latency-bound).  value: the
    workload itself, 100 steps from rest, with direct launches (a first
    simulation warms the runtime up; a fresh one is timed).  Also: graph replay
    over 100 steps of the resting pile, once every launch sequence is captured,
    and launches per step."""
    from paper_2306_01369_amd import gg, scenes
    import torch
    steps = args.steps if args.steps_given else 100
    sc = scenes.drop_scene()
    warm = gg.scene_sim(sc)
    warm.step(steps)
    warm.close()
    sim = gg.scene_sim(sc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t_direct = (time.perf_counter() - t0) / steps
    st = sim.stats()
    sim.close()
    g = gg.scene_sim(sc, graph=True)
    for _ in range(4):                      # the pile lands
        g.step(steps)
    replay_ready(g, steps, g.step)
    start = g.stats()["steps_total"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / steps
    gst = g.stats()
    g.close()
    I = sc.n_iters
    launches = 6 + I + 1                     # keys, 3 scans, scatter, detect, sweeps, integrate
    resort = 1 + 4 * 5 + 1 + 11              # keys, 4 radix passes x 5, permute, work items
    return {
        "metric": "drop-pile step latency (4096 spheres, 20 PJA iters)",
        "value": 1e6 * t_direct, "unit": "us/step", "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": 1e3 * t_direct, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "drop: 4096 spheres r=5 mm from a 16^3 lattice into a 0.2 m walled box, "
                               "100 steps from rest (direct launches)", "n": sc.n},
        "contacts_last_step": st["n_pp"] + st["n_pb"],
        "us_per_step_graph_resting_pile": 1e6 * t_graph,
        "graph_window_first_step": start,
        "graph_window_contacts": gst["n_pp"] + gst["n_pb"],
        "launches_per_step": launches,
        "resort_launches": resort,
        "resort_every": st["reorder_every"],
        "pja_lanes": st["pja_lanes"],
    }


def bench_diff(args, precisions=(0, 1)):
    """32,768 grains, 50 steps with a capsule tool: plain forward, recorded
    (differentiable) forward and its backward (checkpoint every 10 steps),
    in the binary32 build and the double check build."""
    from paper_2306_01369_amd import gg, scenes
    import torch
    sc = scenes.diff_scene()
    steps = 50
    nb = len(sc.bodies)
    tw = np.zeros((steps, nb, 6), np.float32)
    tw[:, -1, :3] = sc.bodies[-1]["nu"]
    gx = np.zeros((sc.n, 3), np.float32)
    gx[:, 2] = 1.0 / sc.n
    res = {}
    for prec in precisions:
        kw = dict(dt=sc.dt, alpha=sc.alpha, mu=sc.mu, n_iters=sc.n_iters, precision=prec)
        t = {}
        for rep in range(2):                 # the first repetition warms up
            sim = gg.Sim(sc.x, sc.v, sc.radius, sc.bodies, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(steps, twists=tw)
            torch.cuda.synchronize()
            t["plain"] = time.perf_counter() - t0
            sim.close()
            dsim = gg.Sim(sc.x, sc.v, sc.radius, sc.bodies, differentiable=True, checkpoint_every=10, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            dsim.step(steps, twists=tw)
            torch.cuda.synchronize()
            t["recorded"] = time.perf_counter() - t0
            t0 = time.perf_counter()
            dsim.backward(gx, None)
            torch.cuda.synchronize()
            t["backward"] = time.perf_counter() - t0
            st = dsim.stats()
            dsim.close()
        res[prec] = dict(t, peak=st["device_bytes_peak"])
    f = res[0]
    return {
        "metric": "backward particle-steps/s (32,768 grains, 50 steps, 20 PJA iters)",
        "value": sc.n * steps / f["backward"], "unit": "particle-steps/s", "n_gpus": 1, "steps": steps,
        "warmup": 1, "ms_per_step": 1e3 * f["backward"] / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "differentiable: 32,768 spheres r=3mm resting in a 0.3x0.3 m footprint, capsule "
                               "tool, 50 steps, checkpoint every 10 steps, loss gradient w.r.t. x0 and twists",
                   "n": sc.n},
        "forward_plain_s": f["plain"], "forward_recorded_s": f["recorded"], "backward_s": f["backward"],
        "backward_over_plain_forward": f["backward"] / f["plain"],
        "forward_plus_backward_over_plain_forward": (f["recorded"] + f["backward"]) / f["plain"],
        "fp64_build": ({"forward_plain_s": res[1]["plain"], "forward_recorded_s": res[1]["recorded"],
                        "backward_s": res[1]["backward"]} if 1 in res else None),
        "device_bytes_peak": max(q["peak"] for q in res.values()),
    }


def bench_gears(args):
    """The many-body benchmark: helical gears (grid SDFs) spinning in a
    cylindrical tower with the cyclic vertical boundary; throughput for
    4,096 .. 65,536 particles and 0 .. 20 gears (plus the tower wall)."""
    from paper_2306_01369_amd import gg, scenes
    import torch
    steps = args.steps if args.steps_given else 64   # a multiple of twice the re-sort interval
    table = []
    for n in (4096, 16384, 65536):
        for nb in (0, 5, 10, 20):
            sc, cyc = scenes.gear_tower(n=n, n_gears=nb, seed=1)
            sim = gg.Sim(sc.x, sc.v, sc.radius, sc.bodies, dt=sc.dt, alpha=sc.alpha, mu=sc.mu,
                         n_iters=sc.n_iters, cyclic_z=cyc, graph=True)
            sim.step(steps)                 # the flow develops; the graph is captured
            replay_ready(sim, steps, sim.step)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(steps)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            st = sim.stats()
            sim.close()
            table.append({"particles": n, "gears": nb, "particle_steps_per_s": n * steps / t,
                          "us_per_step": 1e6 * t / steps, "contacts_pp": st["n_pp"], "contacts_pb": st["n_pb"]})
            log(f"gears n={n} bodies={nb}: {1e6 * t / steps:.1f} us/step")
    best = max(table, key=lambda r: r["particle_steps_per_s"])
    return {
        "metric": "gear-tower particle-steps/s (20 PJA iters) vs particles and gears",
        "value": table[-1]["particle_steps_per_s"], "unit": "particle-steps/s", "n_gpus": 1, "steps": steps,
        "warmup": steps, "ms_per_step": table[-1]["us_per_step"] / 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "gear tower: 65,536 spheres r=2 mm in a 0.1 m radius, 0.5 m tall cylindrical tower "
                               "(grid SDF wall) with 20 helical gears (grid SDFs) spinning at random rates, cyclic "
                               "vertical boundary, dt=1 ms, 20 PJA sweeps (value: the largest configuration)",
                   "n": 65536, "gears": 20},
        "table": table, "best": best,
    }


def bench_hash_sweep(args):
    """The paper's hash-table-size ablation: a column of grains at rest (the
    most collision candidates per grain), 1,024 .. 65,536 grains, table sizes
    n/4 .. 16n; speedup over real time = dt / (seconds per step)."""
    from paper_2306_01369_amd import gg, scenes
    import torch
    steps = args.steps if args.steps_given else 64   # a multiple of twice the re-sort interval
    factors = (0.25, 0.5, 1, 2, 4, 8, 16)
    table = []
    for n in (1024, 4096, 16384, 65536):
        sc = scenes.column_scene(n=n, r=0.004)
        row = {"particles": n}
        for f in factors:
            sim = gg.Sim(sc.x, sc.v, sc.radius, sc.bodies, dt=sc.dt, alpha=sc.alpha, mu=sc.mu,
                         n_iters=sc.n_iters, hash_size=max(1, int(f * n)), graph=True)
            replay_ready(sim, steps, sim.step)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(steps)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / steps
            sim.close()
            row[f"{f}n"] = sc.dt / t
        table.append(row)
        log(f"hash sweep n={n}: " + ", ".join(f"{k}={v:.1f}" for k, v in row.items() if k != "particles"))
    last = table[-1]
    return {
        "metric": "speedup over real time vs hash table size (column at rest)",
        "value": last["2n"], "unit": "x realtime (dt=1 ms)", "n_gpus": 1, "steps": steps, "warmup": steps,
        "ms_per_step": sc.dt / last["2n"] * 1e3, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "column at rest: 1,024..65,536 spheres r=4 mm packed in an 8x8-grain walled column, "
                               "20 PJA sweeps; table sizes n/4..16n (value: 65,536 grains at 2n)"},
        "table": table,
    }


def bench_passes(args):
    """The paper's kernel-order ablation on MI355X: detection and the impulse
    sweeps split across launches (the production path; also replayed from a
    captured graph) against one cooperative launch per step with grid-wide
    barriers (GG_FLAG_FUSED), on a column of grains at rest (1,024 .. 65,536
    grains) and on the 1M scoop bed; speedup over real time = dt / (s per step)."""
    from paper_2306_01369_amd import gg, scenes
    import torch
    steps = 8 * max(1, (args.steps if args.steps_given else 96) // 8)
    modes = (("split", {}), ("split+graph", {"graph": True}), ("fused", {"fused": True}))
    cases = [(f"column-{n}", scenes.column_scene(n=n, r=0.004)) for n in (1024, 4096, 16384, 65536)]
    cases.append(("scoop-1M", scenes.scoop_scene()))
    table = []
    for name, sc in cases:
        row = {"case": name, "particles": sc.n}
        for mode, kw in modes:
            sim = gg.Sim(sc.x, sc.v, sc.radius, sc.bodies, dt=sc.dt, alpha=sc.alpha, mu=sc.mu,
                         n_iters=sc.n_iters, **kw)
            k = steps if sc.n < 500000 else max(8, 8 * (steps // 40))
            replay_ready(sim, k, sim.step)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(k)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / k
            sim.close()
            row[mode] = {"us_per_step": 1e6 * t, "x_realtime": sc.dt / t}
        table.append(row)
        log(f"passes {name}: " + ", ".join(f"{m}={row[m]['us_per_step']:.0f} us" for m, _ in modes))
    last = table[-1]
    return {
        "metric": "kernel-order ablation: us/step, split launches vs one fused cooperative launch",
        "value": last["fused"]["us_per_step"] / last["split"]["us_per_step"], "unit": "fused/split time ratio (1M)",
        "n_gpus": 1, "steps": steps, "warmup": steps, "ms_per_step": last["fused"]["us_per_step"] / 1e3,
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "column at rest (1,024..65,536 spheres r=4 mm, 8x8 grains per layer, walled) and "
                               "the 1M scoop bed; 20 PJA sweeps; split launches (direct, graph) vs GG_FLAG_FUSED"},
        "table": table,
    }


def bench_gym(args):
    """The Gym-style bulldozing environment (Sec. III-A): 128 arenas of 8,192
    grains (1,048,576 in all), each action held for 5 steps of 10 ms, ego
    (64x48, perspective) and sky (64x64, orthographic) depth images and the
    goal-box reward after every environment step, uniform random actions."""
    from paper_2306_01369_amd.bulldozer import BulldozerEnv
    import torch
    steps = args.steps if args.steps_given else 40
    n_envs, per = 128, 8192
    env = BulldozerEnv(n_envs=n_envs, n_particles=per, device_obs=True)
    rng = np.random.default_rng(0)
    env.reset()
    log("gym: warm-up (graph capture)")
    for _ in range(5):
        env.step(rng.uniform(-1, 1, (n_envs, 2)))
    # every re-sort phase and buffer parity an environment step can start in
    replay_ready(env.sim, env.substeps, lambda k: env.step(rng.uniform(-1, 1, (n_envs, 2))))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        obs, rew, done, info = env.step(rng.uniform(-1, 1, (n_envs, 2)))
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    # phase split (each phase synchronised, so the sum exceeds the loop above)
    ph = {"sim_steps": 0.0, "render": 0.0, "reward": 0.0, "host_control": 0.0}
    k_ph = max(5, steps // 4)
    for _ in range(k_ph):
        ta = time.perf_counter()
        tw = env._twists(rng.uniform(-1, 1, (n_envs, 2)))
        tb = time.perf_counter()
        env.sim.step(env.substeps, tw)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        env.observe()
        torch.cuda.synchronize()
        td = time.perf_counter()
        env.sim.goal_reward(env.boxes)
        te = time.perf_counter()
        ph["host_control"] += tb - ta
        ph["sim_steps"] += tc - tb
        ph["render"] += td - tc
        ph["reward"] += te - td
    ph = {k: 1e3 * v / k_ph for k, v in ph.items()}
    st = env.sim.stats()
    env.close()
    n = n_envs * per
    log(f"gym: {1e3 * total / steps:.2f} ms per environment step; phases {ph}")
    return {
        "metric": "bulldozing environment steps/s (128 arenas, 5 x 10 ms sim steps + depth images + reward)",
        "value": n_envs * steps / total, "unit": "env-steps/s", "n_gpus": 1, "steps": steps, "warmup": 5,
        "ms_per_step": 1e3 * total / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "bulldozing: 128 walled 0.7 m arenas, each a 0.4 m pile of 8,192 spheres r=4 mm, a "
                               "goal box along the far side and a box blade under track steering; action held 5 "
                               "steps of 10 ms, 20 PJA sweeps; ego 64x48 + sky 64x64 depth images and goal-box "
                               "reward per environment step, uniform random actions",
                   "n": n, "n_envs": n_envs, "substeps": env.substeps},
        "particle_steps_per_s": n * env.substeps * steps / total,
        "phases_ms_per_env_step": ph,
        "contacts_last_step": st["n_pp"] + st["n_pb"],
    }


def bench_large(args):
    """4,194,304 polydisperse spheres, 64 sweeps, box + capsule tools: settle the
    layered start (untimed, 20 sweeps, tools still), time 80 forward steps, then a
    differentiable 20-step call and its backward (checkpoint every step,
    recompute); reports peak device memory."""
    from paper_2306_01369_amd import gg, scenes
    import torch
    log("generating the polydisperse bed")
    sc = scenes.large_scene()
    n = sc.n
    tile = {}
    still = [dict(b, nu=np.zeros(3), omega=np.zeros(3)) for b in sc.bodies]
    sim = gg.Sim(sc.x, sc.v, sc.radius, still, dt=sc.dt, alpha=sc.alpha, mu=sc.mu, n_iters=20, **tile)
    settle = args.settle_steps
    log(f"settling {settle} steps")
    t0 = time.perf_counter()
    for k in range(0, settle, 50):
        sim.step(min(50, settle - k))
        log(f"  settled {min(k + 50, settle)} steps, max |v| {np.abs(sim.read('vel')).max():.4f}")
    t_settle = time.perf_counter() - t0
    x = sim.read("pos")
    v = sim.read("vel")
    sim.close()
    rad = sc.radius
    surface = float(np.percentile(x[:, 2] + rad, 99.5))
    bodies = [dict(b) for b in sc.bodies]
    for b in bodies[-2:]:
        low = b["params"][2] if b["shape"] == "box" else b["params"][0]
        b["t"] = np.array([b["t"][0], b["t"][1], surface + 0.01 + low])
    kw = dict(dt=sc.dt, alpha=sc.alpha, mu=sc.mu, n_iters=sc.n_iters, profile=True, **tile)
    sim = gg.Sim(x, v, rad, bodies, **kw)
    sim.step(2)
    torch.cuda.synchronize()
    steps = 80
    log(f"timing {steps} forward steps (64 sweeps)")
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    st = sim.stats()
    x = sim.read("pos")
    v = sim.read("vel")
    sim.close()
    log("differentiable 20-step call and its backward")
    dsim = gg.Sim(x, v, rad, bodies, differentiable=True, checkpoint_every=1, **kw)
    t0 = time.perf_counter()
    dsim.step(20)
    torch.cuda.synchronize()
    t_fwd20 = time.perf_counter() - t0
    gx = np.zeros((n, 3), np.float32)
    gx[:, 2] = 1.0 / n      # d(mean height)/dx
    t0 = time.perf_counter()
    _, _, gtw = dsim.backward(gx, None)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    dst = dsim.stats()
    dsim.close()
    value = n * steps / t_fwd
    return {
        "metric": "large polydisperse particle-steps/s (64 PJA iters)",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": steps, "warmup": 2,
        "ms_per_step": 1e3 * t_fwd / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "large: 4,194,304 spheres, lognormal radii (median 2 mm, sigma 0.25, clipped "
                               "[1,4] mm), walled 2x2 m bed settled from stacked lattice layers, box + capsule tools, "
                               "64 PJA sweeps", "n": n, "settle_steps": settle, "settle_s": t_settle,
                   "bed_surface_m": surface, "contacts_last_step": st["n_pp"] + st["n_pb"],
                   "max_contacts_per_particle": st["max_contacts"], "capacity": st["capacity"]},
        "backward": {"steps": 20, "forward_s": t_fwd20, "backward_s": t_bwd, "backward_over_forward": t_bwd / t_fwd20,
                     "checkpoint_every": 1, "twist_grad_norm": float(np.linalg.norm(gtw))},
        "device_bytes_peak": max(st["device_bytes_peak"], dst["device_bytes_peak"]),
        "phases_ms_per_step": {"keys_sort_detect": st["ms_detect"] / steps, "pja": st["ms_pja"] / steps},
        "detect_fallback_items": st["detect_fallback"], "detect_items": st["detect_items"],
        "launch_shape": {k: st[k] for k in ("tile_threads", "tile_node_shift", "tile_max_cells", "tile_max_stage",
                                            "detect_workgroups", "reorder_every", "pja_lanes",
                                            "detect_queues")},
    }


def profiler_window(on):
    """Mark the start (on=True) or end of the timed steps in a profiler's
    kernel list: one short spin kernel (torch's `_sleep`, one thread) on the
    current stream, so a summary can keep only the dispatches between the two
    marks."""
    import torch
    torch.cuda._sleep(1000)
    torch.cuda.synchronize()


def _timed_bed(args, sim, n, pja_iters, workload, extra_config, traffic_measured=False):
    """W untimed steps, then K timed steps of `sim`; the bench line without the
    CPU baseline.  k_pja's duration comes from the library's HIP events on its
    own stream (profile=True)."""
    import torch
    log(f"n={n} warmup {args.warmup} steps")
    if args.warmup:
        sim.step(args.warmup)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    if args.profile_window:
        profiler_window(True)
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if args.profile_window:
        profiler_window(False)
    st = sim.stats()
    log(f"done: {elapsed:.3f} s, stats {st}")
    steps = args.steps
    launches = max(1, st["pja_launches"])
    pja_ms = st["ms_pja"] / launches
    contacts_avg = st["contacts_summed"] / max(1, st["steps_done"])
    algo = pja_algorithmic_bytes(n, contacts_avg)
    achieved = algo / (pja_ms * 1e-3) / 1e9
    # the counters were taken on the settled scoop bed only: another bed reports none
    traffic = measured_traffic() if traffic_measured else None
    out = {
        "metric": METRIC,
        "value": n * steps / elapsed,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": dict({"workload": workload, "n": n, "pja_iters": pja_iters, "contacts_per_step": contacts_avg,
                        "hit_rate": 2.0 * st["n_pp"] / max(1, st["candidates"])}, **extra_config),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_pja (one projected-Jacobi sweep)", "avg_launch_us": pja_ms * 1e3,
                     "algorithmic_bytes_per_launch": algo},
        "phases_ms_per_step": {"keys_sort_detect": st["ms_detect"] / steps, "pja": st["ms_pja"] / steps,
                               "integrate": st["ms_integrate"] / steps},
        "launch_shape": {k: st[k] for k in ("tile_threads", "tile_node_shift", "tile_max_cells", "tile_max_stage",
                                            "detect_workgroups", "reorder_every", "pja_lanes",
                                            "detect_queues")},
    }
    if traffic:
        # measured HBM bytes per sweep (rocprofv3 counters) over the live sweep duration
        gbs = traffic / (pja_ms * 1e-3) / 1e9
        out["hbm_measured"] = {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                               "bytes_per_launch": traffic}
    return out


def bench_lattice(args):
    """The 1,048,576-sphere bed built as compressed simple-cubic layers (six
    contacts per interior grain, no settling) with the scoop tool 1 cm above
    it: a secondary workload, the contact table's best case."""
    from paper_2306_01369_amd import gg, scenes
    import torch
    log("generating the lattice bed")
    scene = scenes.scoop_scene()
    stream = torch.cuda.current_stream(0).cuda_stream
    x = torch.from_numpy(scene.x).to("cuda:0")
    v = torch.from_numpy(scene.v).to("cuda:0")
    r = torch.from_numpy(scene.radius).to("cuda:0")
    sim = gg.Sim(x, v, r, scene.bodies, dt=scene.dt, alpha=scene.alpha, mu=scene.mu, n_iters=scene.n_iters,
                 gravity=scene.gravity, device=0, stream=stream, profile=True)
    del x, v, r
    out = _timed_bed(args, sim, scene.n, scene.n_iters,
                     "lattice bed: 1,048,576 spheres r=2mm in compressed simple-cubic layers (1x1 m walled box), "
                     "box tool 0.05x0.1x0.2 m at 0.2 m/s on a linear scoop path starting 1 cm above the bed, "
                     "dt=1 ms, 20 PJA sweeps, mu=0.5", {})
    sim.close()
    out["cpu_baseline"] = None if args.skip_cpu_baseline else cpu_baseline(scene, args.cpu_steps)
    return out


def settle_on_gpu(scene):
    """Seeded settling of a poured bed with the library (the plan of
    scenes.SETTLE_*): frictionless compaction, then settling with the bed's
    friction until all but scenes.settle_fast_allowed(n) grains are slower
    than SETTLE_VMAX (checked every SETTLE_CHECK_EVERY steps, at most
    SETTLE_MAX_STEPS).  Returns the state (caller order, binary32) and a record
    of the settling."""
    from paper_2306_01369_amd import gg, scenes
    t0 = time.perf_counter()
    kw = dict(dt=scene.dt, alpha=scene.alpha, gravity=scene.gravity, n_iters=scenes.SETTLE_ITERS, device=0)
    sim = gg.Sim(scene.x, scene.v, scene.radius, scene.bodies, mu=0.0, **kw)
    sim.step(scenes.SETTLE_COMPACT_STEPS)
    x, v = sim.read("pos"), sim.read("vel")
    sim.close()
    sim = gg.Sim(x, v, scene.radius, scene.bodies, mu=scene.mu, **kw)
    steps, vmax, fast = 0, float("inf"), scene.n
    allowed = scenes.settle_fast_allowed(scene.n)
    while steps < scenes.SETTLE_MAX_STEPS:
        sim.step(scenes.SETTLE_CHECK_EVERY)
        steps += scenes.SETTLE_CHECK_EVERY
        v = sim.read("vel").astype(np.float64)
        speed = np.sqrt((v * v).sum(1))
        vmax = float(speed.max())
        fast = int((speed >= scenes.SETTLE_VMAX).sum())
        if fast <= allowed:
            break
    x, v = sim.read("pos"), sim.read("vel")
    st = sim.stats()
    sim.close()
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(x, np.float32).tobytes())
    h.update(np.ascontiguousarray(v, np.float32).tobytes())
    rec = {"compaction_steps": scenes.SETTLE_COMPACT_STEPS, "settle_steps": steps, "max_speed": vmax,
           "grains_at_or_above_1mm_s": fast, "p999_speed": float(np.percentile(speed, 99.9)),
           "sweeps": scenes.SETTLE_ITERS, "contacts": st["n_pp"] + st["n_pb"], "seconds": time.perf_counter() - t0,
           "state_sha256": h.hexdigest()}
    log(f"settled: {rec}")
    return x, v, rec


SCOOP_PATH_STEPS = 200


def bench_scoop(args):
    """The scoop bed: 2^20 spheres poured and settled on the GPU, then the box
    tool's 200-step scoop path; the timed window is the path's last K steps
    (after W warm-up steps), where the tool is deepest in the bed."""
    from paper_2306_01369_amd import gg, scenes
    import torch
    log("pouring the scoop bed")
    pour = scenes.scoop_pour()
    n = pour.n
    x, v, settle = settle_on_gpu(pour)
    r0 = float(pour.radius[0])
    surface = scenes.surface_height(x, r0)
    tool = scenes.scoop_tool(surface)
    bodies = pour.bodies + [tool]
    approach = max(0, SCOOP_PATH_STEPS - args.warmup - args.steps)
    log("state to the device")
    stream = torch.cuda.current_stream(0).cuda_stream
    xd = torch.from_numpy(x).to("cuda:0")
    vd = torch.from_numpy(v).to("cuda:0")
    rd = torch.from_numpy(pour.radius).to("cuda:0")
    kw = dict(dt=pour.dt, alpha=pour.alpha, mu=pour.mu, n_iters=pour.n_iters, gravity=pour.gravity)
    sim = gg.Sim(xd, vd, rd, bodies, device=0, stream=stream, profile=True, **kw)
    del xd, vd, rd
    log(f"tool approach: {approach} untimed steps of the scoop path")
    for k in range(0, approach, 20):
        sim.step(min(20, approach - k))
    log("approach done")
    tuned = None
    if args.tune:
        # the launch shape for this bed, timed by the autotuner from the state
        # the window starts in (every candidate gives the same bits).  Off by
        # default: in this process, after torch's device work, the tuner has
        # stalled without progress (no cause found; the same tuning in a
        # process without the torch-stream simulation before it finishes in
        # about 5 s and gains about 2%)
        from paper_2306_01369_amd import autotune
        x1, v1, poses = sim.read("pos"), sim.read("vel"), sim.read("body_poses")
        sim.close()
        for q, b in enumerate(bodies):
            b["R"], b["t"] = poses[q][:, :3].astype(np.float64), poses[q][:, 3].astype(np.float64)
        t0 = time.perf_counter()
        table = []
        log("autotune from the approach state")
        params = autotune.tune(x1, v1, pour.radius, bodies, sim_kwargs=kw, use_cache=False, record=table)
        tuned = {"params": params, "seconds": time.perf_counter() - t0,
                 "default_ms_per_step": table[0][1] if table and table[0][1] else None,
                 "tuned_ms_per_step": min(t for _, t in table if t) if table else None}
        log(f"autotune: {tuned}")
        sim = gg.Sim(x1, v1, pour.radius, bodies, device=0, stream=stream, profile=True, **kw, **params)
    phi = n * (4.0 / 3.0) * math.pi * r0 ** 3 / (1.0 * 1.0 * surface)
    extra = {"bed": {"surface_m": surface, "packing_fraction": phi, **settle}, "autotune": tuned,
             "window": {"first_path_step": approach + args.warmup, "steps": args.steps,
                        "path_steps": SCOOP_PATH_STEPS}}
    out = _timed_bed(args, sim, n, pour.n_iters,
                     "scoop bed: 1,048,576 spheres r=2mm poured and settled (frictionless compaction, then mu=0.5 "
                     "until at most 10 grains move at 1 mm/s or more) in a 1x1 m walled box; box tool 0.05x0.1x0.2 m "
                     "starting 1 cm above "
                     "the surface, 0.2 m/s along (cos 30, 0, -sin 30); dt=1 ms, 20 PJA sweeps, mu=0.5; timed: the "
                     "last steps of the 200-step path", extra, traffic_measured=True)
    pairs = sim.read("contacts")
    out["config"]["tool_contacts_last_step"] = int(np.sum(pairs[sim.stats()["n_pp"]:, 1] == len(bodies) - 1))
    sim.close()
    if not args.skip_ratios:
        out.update(metric_ratios(args))
    if args.skip_cpu_baseline:
        out["cpu_baseline"] = None
    else:
        log(f"oracle on the host cores: {args.cpu_steps} steps")
        out["cpu_baseline"] = cpu_baseline(scenes.scoop_scene(), args.cpu_steps)
    return out


def metric_ratios(args):
    """The metric's other two numbers, on reduced and stated sizes so the run
    stays within minutes: the batched form against a loop of separate
    simulations (32 of the 256 environments), and the backward pass against
    the plain forward (the 32,768-grain differentiable bed, 50 steps)."""
    b = bench_batched(args, n_envs=32, steps=32, plain_steps=4)
    d = bench_diff(args, precisions=(0,))
    return {
        "batched_speedup_vs_plain": b["speedup_vs_plain_loop"],
        "backward_over_forward": d["backward_over_plain_forward"],
        "ratios_config": {
            "batched": "32 walled beds of U{8192..65536} spheres r=3mm (the first 32 of the 256-environment "
                       f"workload, {b['config']['n']} grains), 32 steps as one captured call vs 4 steps of 32 "
                       "separate simulations",
            "batched_particle_steps_per_s": b["value"],
            "backward": "32,768 grains r=3mm, 50 steps, capsule tool, checkpoint every 10 steps, binary32: "
                        "backward time over the plain forward's",
            "forward_recorded_over_plain": d["forward_recorded_s"] / d["forward_plain_s"],
        },
    }



def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", choices=["scoop", "lattice", "batched", "large", "drop", "diff", "gears", "hashsweep",
                                           "gym", "passes"],
                    default="scoop")
    ap.add_argument("--settle-steps", type=int, default=150, help="large workload: untimed settling steps")
    ap.add_argument("--profile-window", action="store_true",
                    help="scoop/lattice: bracket the timed steps with marker kernels for a profiler summary")
    ap.add_argument("--tune", action="store_true",
                    help="scoop: autotune the launch shape from the window's first state (default: the library's "
                         "default shape)")
    ap.add_argument("--skip-ratios", action="store_true",
                    help="scoop workload: leave out the batched and backward ratios")
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--calibrate-copy", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the workload is a single bed on one device; "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        copy_calibration()
        return
    args.steps_given = args.steps is not None
    if args.steps is None:
        args.steps = 50 if args.workload == "scoop" else 200
    if args.workload in ("batched", "large", "drop", "diff", "gears", "hashsweep", "gym", "passes"):
        out = {"batched": bench_batched, "large": bench_large, "drop": bench_drop, "diff": bench_diff,
               "gears": bench_gears, "hashsweep": bench_hash_sweep, "gym": bench_gym,
               "passes": bench_passes}[args.workload](args)
        print(json.dumps(out), flush=True)
        return

    if args.workload == "lattice":
        out = bench_lattice(args)
    else:
        out = bench_scoop(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
