"""gg_goal_reward_noalloc (no device allocation; its workspace is the
library's fixed per-GPU array) against gg_goal_reward through the C ABI: the
same bits on two calls in a row, the second with a smaller simulation, for
host and device outputs; a simulation beyond the workspace is rejected."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2306_01369_amd import gg, scenes

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _bed(n_envs, lo, hi, seed):
    s = scenes.batched_scene(seed=seed, n_envs=n_envs, lo=lo, hi=hi, n_steps=4)
    sim = gg.Sim(s.x, s.v, s.radius, s.bodies, env_offsets=s.env_offsets)
    sim.step(2, twists=s.twists[:2])
    return s, sim


def _boxes(s, rng):
    off = np.asarray(s.env_offsets)
    out = []
    for e in range(len(off) - 1):
        x = s.x[off[e]:off[e + 1]]
        # a box over part of the footprint, from below the floor to above the bed
        lo = x.min(0) + np.array([rng.uniform(0.0, 0.05), rng.uniform(0.0, 0.05), -0.01])
        hi = lo + np.array([rng.uniform(0.05, 0.2), rng.uniform(0.05, 0.2), 1.0])
        out.append(np.concatenate([lo, hi]))
    return np.asarray(out, np.float32)


def _device_call(fn, sim, boxes):
    torch = pytest.importorskip("torch")
    ne = boxes.shape[0]
    rew = torch.full((ne,), -1.0, dtype=torch.float64, device="cuda:0")
    ins = torch.full((ne,), -1, dtype=torch.int64, device="cuda:0")
    st = fn(sim._h, boxes.ctypes.data_as(C.c_void_p), C.c_void_p(rew.data_ptr()), C.c_void_p(ins.data_ptr()),
            gg.GG_MEM_DEVICE)
    assert st == gg.GG_OK, gg.lib().gg_error_detail()
    torch.cuda.synchronize()
    return rew.cpu().numpy(), ins.cpu().numpy()


def test_no_alloc_reward_matches_the_allocating_call_twice_the_second_smaller():
    rng = np.random.default_rng(5)
    L = gg.lib()
    for n_envs, lo, hi, seed in ((6, 20000, 40000, 1), (3, 1500, 4000, 2)):
        s, sim = _bed(n_envs, lo, hi, seed)
        bx = _boxes(s, rng)
        say("no-alloc reward: envs", n_envs, "grains", s.n)
        got, got_in = sim.goal_reward(bx, noalloc=True)
        want, want_in = sim.goal_reward(bx)
        assert got.tobytes() == want.tobytes() and np.array_equal(got_in, want_in)
        assert np.all(want_in > 0) and np.any(want_in < np.diff(s.env_offsets))
        dg, dgi = _device_call(L.gg_goal_reward_noalloc, sim, bx)
        dw, dwi = _device_call(L.gg_goal_reward, sim, bx)
        assert dg.tobytes() == dw.tobytes() == want.tobytes()
        assert np.array_equal(dgi, dwi) and np.array_equal(dgi, want_in)
        sim.close()


def test_no_alloc_reward_rejects_a_simulation_beyond_its_workspace():
    # 60,000 one-grain environments need 2.4 MB of workspace (40 bytes each)
    ne = 60000
    x = np.zeros((ne, 3), np.float32)
    x[:, 0] = np.arange(ne) * 0.01
    off = np.arange(ne + 1, dtype=np.int64)
    sim = gg.Sim(x, np.zeros_like(x), np.full(ne, 0.001, np.float32), [], env_offsets=off)
    bx = np.tile(np.array([[-1.0, -1.0, -1.0, 1.0, 1.0, 1.0]], np.float32), (ne, 1))
    with pytest.raises(gg.GGError) as e:
        sim.goal_reward(bx, noalloc=True)
    assert e.value.status == gg.GG_ERR_INVALID and "workspace" in str(e.value)
    rew, ins = sim.goal_reward(bx)           # the allocating call still serves it
    assert ins.sum() == np.sum(x[:, 0] <= np.float32(1.0)) and np.all(np.isfinite(rew))
    sim.close()
