"""Host-side logic of the Gym-style bulldozing environment (Sec. III-A): arena
layout, track steering and camera placement, without a device."""
import math

import numpy as np

from paper_2306_01369_amd.bulldozer import BulldozerEnv


def _env(**kw):
    e = BulldozerEnv(n_envs=3, n_particles=500, **kw)
    e.state = e.initial_state()
    return e


def test_layout_keeps_piles_blades_and_goals_apart():
    e = _env()
    assert e.x0.shape == (1500, 3) and list(e.offsets) == [0, 500, 1000, 1500]
    for k in range(3):
        gx, gy = e.origin(k)
        p = e.x0[e.offsets[k]:e.offsets[k + 1]]
        assert p[:, 0].min() >= gx and p[:, 0].max() <= gx + e.arena
        assert p[:, 1].min() >= gy and p[:, 1].max() <= gy + e.arena
        box = e.goal_box(k)
        assert np.all(p[:, 0] < box[0])                      # the goal starts empty
        blade = e.bodies[e.blade_index[k]]
        assert blade["t"][0] + e.blade[0] < p[:, 0].min()    # the blade starts clear of the pile
        assert blade["env"] == k
    # arenas do not overlap
    assert e.origin(1)[0] - e.origin(0)[0] > e.arena


def test_track_steering_twists():
    e = _env(substeps=4, dt=0.01, v_max=0.2, yaw_max=1.0)
    x0 = e.state.copy()
    tw = e._twists(np.array([[1.0, 0.0], [0.0, 1.0], [5.0, -5.0]]))
    assert tw.shape == (4, len(e.bodies), 6)
    blades = set(e.blade_index)
    for b in range(len(e.bodies)):
        if b not in blades:
            assert not tw[:, b].any()
    # env 0: straight ahead along +x; env 1: turn in place; env 2: clipped to (1, -1)
    assert e.state[0][0] - x0[0][0] == pytest_approx(4 * 0.01 * 0.2)
    assert e.state[0][2] == 0.0
    assert np.array_equal(e.state[1][:2], x0[1][:2]) and e.state[1][2] == pytest_approx(4 * 0.01 * 1.0)
    assert e.state[2][2] == pytest_approx(-4 * 0.01 * 1.0)
    b2 = e.blade_index[2]
    np.testing.assert_allclose(np.linalg.norm(tw[:, b2, :3], axis=1), 0.2, rtol=1e-6)
    np.testing.assert_allclose(tw[:, b2, 5], -1.0)
    # the heading used at substep k is the yaw reached after k substeps
    for k in range(4):
        th = -0.01 * k
        np.testing.assert_allclose(tw[k, b2, :2], [0.2 * math.cos(th), 0.2 * math.sin(th)], rtol=1e-6)


def test_ego_camera_rides_on_the_blade():
    e = _env()
    e.state[0, 2] = math.pi / 2
    pose = e._ego_poses()[0]
    R, t = pose[:, :3], pose[:, 3]
    np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-12)
    fwd = R[:, 2]
    assert fwd[1] > 0.5 and fwd[2] < 0           # looks along the heading (+y), downward
    assert t[2] > e.blade[2]                      # above the blade


def pytest_approx(v):
    import pytest
    return pytest.approx(v, rel=1e-6, abs=1e-12)   # twists are binary32


def test_blade_stops_short_of_the_walls_but_may_turn_and_back_off():
    e = _env(substeps=3, dt=0.01, v_max=0.2, yaw_max=1.0)
    m = math.hypot(e.blade[0], e.blade[1]) + 0.02
    gx, gy = e.origin(1)
    e.state[1] = (gx + e.arena - m - 1e-4, gy + 0.3, 0.0)   # facing the far wall, almost at the limit
    x_before = e.state[1, 0]
    tw = e._twists(np.array([[0.0, 0.0], [1.0, 0.5], [0.0, 0.0]]))
    b = e.blade_index[1]
    assert np.all(tw[:, b, 0] == 0.0) and np.all(tw[:, b, 5] == np.float32(0.5))   # turns, does not advance
    assert e.state[1, 0] == x_before
    e.state[1, 2] = 0.0
    tw = e._twists(np.array([[0.0, 0.0], [-1.0, 0.0], [0.0, 0.0]]))
    assert np.all(tw[:, b, 0] < 0)                                                  # backing off is allowed
