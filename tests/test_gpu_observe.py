"""GPU parity of the observations of the Gym-style environment (Sec. III-A):
depth cameras and the goal-box reward through the C ABI, against the FP64
oracle on the state read back from the device.

Bars: depth images agree to 2 units in the last place of binary32 (hit
decisions are the same binary32 predicates on both sides, depths are FP64
rounded once); inside counts are exact; rewards agree to 1e-12 relative to
the sum of the magnitudes of their terms (FP64 sums in different orders)."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2306_01369_amd import gg, scenes

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _close_images(got, want, label):
    assert got.shape == want.shape, label
    ulp = np.spacing(np.maximum(np.abs(want), np.float32(1e-30))).astype(np.float64)
    err = np.abs(got.astype(np.float64) - want.astype(np.float64)) / ulp
    say(label, "pixels", want.size, "max error (ulp)", float(err.max()),
        "hit pixels", int(np.sum(want < want.max())))
    assert err.max() <= 2.0, label


def _bed_cameras(x0, x1, y0, y1, top, env=0, size=(96, 80)):
    cx, cy = 0.5 * (x0 + x1), 0.5 * (y0 + y1)
    sky = scenes.sky_camera(x0, x1, y0, y1, 0.4, size[0], size[1], env=env)
    ego = scenes.perspective_camera((x0 + 0.05, cy - 0.02, top + 0.12), (cx, cy, top * 0.5), 70.0, 64, 48, 1.5,
                                    env=env)
    corner = scenes.perspective_camera((x1 + 0.2, y1 + 0.15, top + 0.3), (cx, cy, 0.0), 50.0, 80, 60, 3.0, env=env)
    return [sky, ego, corner]


def _reward_terms_scale(x, boxes, off):
    """Sum of |term| per environment, the scale of the reward comparison."""
    out = []
    for e in range(len(off) - 1):
        p = np.asarray(x[off[e]:off[e + 1]], np.float64)
        lo, hi = boxes[e, :3].astype(np.float64), boxes[e, 3:].astype(np.float64)
        d = np.linalg.norm(p - np.clip(p, lo, hi), axis=1)
        n = max(len(p), 1)
        out.append((100.0 * len(p) + d.sum()) / n)
    return np.array(out)


@pytest.mark.parametrize("precision", [0, 1])
def test_depth_and_reward_of_a_moving_bed(precision):
    s = scenes.column_scene(n=3000, r=0.004)
    top = float(s.x[:, 2].max())
    side = float(s.x[:, 0].max()) + 0.004
    say("column bed 3000, precision", precision)
    v0 = np.zeros_like(s.x)
    v0[:, 0] = 0.3   # a sideways shove so that the state is not the lattice
    # the moved state comes from the oracle; both sides draw it from binary32
    orc = O.Oracle(s.x.astype(np.float64), v0.astype(np.float64), s.radius, s.bodies)
    for _ in range(7):
        orc.step()
    xs = orc.x.astype(np.float32)
    sim = gg.Sim(xs, orc.v.astype(np.float32), s.radius, s.bodies, precision=precision, reorder_every=2)
    x = sim.read("pos")
    assert np.array_equal(x, xs)
    r = sim.read("radius")
    cams = _bed_cameras(0.0, side, 0.0, side, top)
    got = sim.render_depth(cams)
    want = O.render_depth(x, r, cams, s.bodies)
    for k, (g, w) in enumerate(zip(got, want)):
        _close_images(g, w, f"camera {k}")
    assert np.array_equal(sim.render_depth(cams)[0], got[0])  # deterministic
    boxes = np.array([[side * 0.5, 0.0, 0.0, side, side, 0.05]], np.float32)
    rew, ins = sim.goal_reward(boxes)
    rw, iw = O.goal_reward(x, boxes)
    say("reward", rew, rw, "inside", ins, iw)
    assert np.array_equal(ins, iw)
    scale = _reward_terms_scale(x, boxes, [0, len(x)])
    assert np.all(np.abs(rew - rw) <= 1e-12 * scale)
    rew2, _ = sim.goal_reward(boxes)
    assert np.array_equal(rew, rew2)
    sim.close()


def test_depth_and_reward_per_environment():
    s = scenes.batched_scene(n_envs=6, lo=1500, hi=4000, n_steps=10)
    say("batched 6 envs", s.n)
    orc = O.Oracle(s.x.astype(np.float64), s.v.astype(np.float64), s.radius, s.bodies,
                   env=np.repeat(np.arange(6), np.diff(s.env_offsets)).astype(np.int32))
    for k in range(3):
        orc.set_twists(s.twists[k])
        orc.step()
    xs = orc.x.astype(np.float32)
    sim = gg.Sim(xs, orc.v.astype(np.float32), s.radius, s.bodies, env_offsets=s.env_offsets)
    x = sim.read("pos")
    assert np.array_equal(x, xs)
    r = sim.read("radius")
    off = np.asarray(s.env_offsets)
    cams = []
    grid = int(np.ceil(np.sqrt(6)))
    for e in (0, 3, 5, 3):
        gx, gy = (e % grid) * 0.5, (e // grid) * 0.5
        top = float(x[off[e]:off[e + 1], 2].max())
        cams += _bed_cameras(gx, gx + 0.3, gy, gy + 0.3, top, env=e, size=(48, 40))
    got = sim.render_depth(cams)
    want = O.render_depth(x, r, cams, s.bodies, env_offsets=off)
    for k, (g, w) in enumerate(zip(got, want)):
        _close_images(g, w, f"camera {k} env {cams[k]['env']}")
    boxes = []
    for e in range(6):
        gx, gy = (e % grid) * 0.5, (e // grid) * 0.5
        boxes.append([gx + 0.2, gy, 0.0, gx + 0.3, gy + 0.3, 0.03])
    boxes = np.asarray(boxes, np.float32)
    rew, ins = sim.goal_reward(boxes)
    rw, iw = O.goal_reward(x, boxes, env_offsets=off)
    assert np.array_equal(ins, iw)
    assert np.all(ins > 0) and np.all(ins < np.diff(off))
    assert np.all(np.abs(rew - rw) <= 1e-12 * _reward_terms_scale(x, boxes, off))
    sim.close()


def test_empty_environment_scores_zero_and_draws_only_planes():
    rng = np.random.default_rng(3)
    n = 500
    x = np.column_stack([rng.uniform(0.02, 0.18, n), rng.uniform(0.02, 0.18, n), rng.uniform(0.01, 0.05, n)])
    x = x.astype(np.float32)
    r = np.full(n, 0.004, np.float32)
    bodies = scenes.walled_box(0, 0.2, 0, 0.2, env=0) + scenes.walled_box(0, 0.2, 0, 0.2, env=2)
    sim = gg.Sim(x, np.zeros_like(x), r, bodies, env_offsets=[0, n, n, n])
    cams = [scenes.sky_camera(0, 0.2, 0, 0.2, 0.3, 32, 32, env=e) for e in (0, 1, 2)]
    got = sim.render_depth(cams)
    want = O.render_depth(x, r, cams, bodies, env_offsets=[0, n, n, n])
    for k, (g, w) in enumerate(zip(got, want)):
        _close_images(g, w, f"camera env {k}")
    assert np.all(got[1] == np.float32(0.3)) and np.all(got[2] == np.float32(0.3))
    boxes = np.tile(np.array([[0, 0, 0, 0.1, 0.2, 0.1]], np.float32), (3, 1))
    rew, ins = sim.goal_reward(boxes)
    rw, iw = O.goal_reward(x, boxes, env_offsets=[0, n, n, n])
    assert rew[1] == 0.0 and rew[2] == 0.0 and ins[1] == 0 and ins[2] == 0
    assert np.array_equal(ins, iw) and abs(rew[0] - rw[0]) <= 1e-12 * 100
    sim.close()


def test_camera_close_to_and_inside_particles():
    # spheres straddling the image border, one holding the camera, one behind it,
    # one whose footprint covers the whole image
    x = np.array([[0.0, 0.0, 0.5], [0.0, 0.0, 0.9], [0.02, 0.0, 0.45], [0.08, 0.05, 0.2],
                  [-0.1, 0.07, 0.1]], np.float32)
    r = np.array([0.05, 0.2, 0.01, 0.03, 0.02], np.float32)
    ground = [scenes.plane((0, 0, 0), (0, 0, 1))]
    sim = gg.Sim(x, np.zeros_like(x), r, ground, gravity=(0, 0, 0), max_contacts=8)
    cams = [scenes.perspective_camera((0, 0, 0.5), (0, 0, 0), 60.0, 40, 30, 3.0, up=(0, 1, 0)),
            scenes.perspective_camera((0.01, 0.0, 0.47), (0, 0, 0), 90.0, 33, 17, 3.0, up=(0, 1, 0)),
            scenes.sky_camera(-0.2, 0.2, -0.15, 0.15, 0.6, 41, 29)]
    got = sim.render_depth(cams)
    want = O.render_depth(x, r, cams, ground)
    for k, (g, w) in enumerate(zip(got, want)):
        _close_images(g, w, f"near camera {k}")
    sim.close()


def test_device_destination_matches_host():
    torch = pytest.importorskip("torch")
    s = scenes.column_scene(n=2000, r=0.004)
    sim = gg.Sim(s.x, s.v, s.radius, s.bodies)
    side = float(s.x[:, 0].max())
    cams = _bed_cameras(0.0, side, 0.0, side, float(s.x[:, 2].max()))
    host = np.concatenate([im.ravel() for im in sim.render_depth(cams)])
    dev = torch.full((host.size + 5,), -1.0, dtype=torch.float32, device="cuda")
    sim.render_depth(cams, out=dev)
    torch.cuda.synchronize()
    d = dev.cpu().numpy()
    assert np.array_equal(d[:host.size], host) and np.all(d[host.size:] == -1.0)
    sim.close()


def test_full_scoop_bed_sampled_pixels():
    s = scenes.scoop_scene()
    say("scoop bed", s.n)
    orc = O.scene_oracle(s)
    for _ in range(2):
        orc.step()
    xs = orc.x.astype(np.float32)
    sim = gg.Sim(xs, orc.v.astype(np.float32), s.radius, s.bodies)
    x = sim.read("pos")
    assert np.array_equal(x, xs)
    r = sim.read("radius")
    top = float(x[:, 2].max())
    cams = [scenes.sky_camera(0.0, 1.0, 0.0, 1.0, 0.5, 256, 256),
            scenes.perspective_camera((0.2, 0.5, top + 0.15), (0.6, 0.5, 0.0), 70.0, 160, 120, 2.0)]
    got = np.concatenate([im.ravel() for im in sim.render_depth(cams)])
    rng = np.random.default_rng(0)
    pix = rng.choice(got.size, 1500, replace=False)
    want = O.render_depth(x, r, cams, s.bodies, pixels=pix)
    _close_images(got[pix], want, "scoop sampled pixels")
    # the sky camera sees the bed surface: heights between 0 and the top
    sky = got[:256 * 256]
    assert np.all(sky >= np.float32(0.5 - top - 0.002 - 1e-6)) and np.all(sky <= np.float32(0.5))
    boxes = np.array([[0.6, 0.0, 0.0, 1.0, 1.0, 0.2]], np.float32)
    rew, ins = sim.goal_reward(boxes)
    rw, iw = O.goal_reward(x, boxes)
    assert np.array_equal(ins, iw)
    assert abs(rew[0] - rw[0]) <= 1e-12 * _reward_terms_scale(x, boxes, [0, len(x)])[0]
    sim.close()
