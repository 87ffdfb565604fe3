"""Pins of the finite-difference gradient reference on closed forms."""
import numpy as np

import oracle as O
from paper_2306_01369_amd import scenes
from gradcheck import TargetLoss, fd_directional, oracle_rollout


def test_fd_free_fall_is_linear_map():
    # no contacts: x_N = x0 + N dt v0 + const, so a linear loss has
    # dL/dx0 = c and dL/dv0 = N dt c exactly
    rng = np.random.default_rng(0)
    x0 = rng.uniform(0, 1, (5, 3)) + 10.0
    v0 = rng.normal(size=(5, 3))
    r = np.full(5, 0.01, np.float32)
    c = np.array([0.3, -1.2, 0.7])
    loss = lambda x, v: float(np.sum(x @ c))
    N, dt = 7, 1e-3
    tw = np.zeros((N, 0, 6))
    d = (rng.normal(size=x0.shape), rng.normal(size=v0.shape), np.zeros_like(tw))
    got, same = fd_directional(loss, x0, v0, r, [], tw, d, 1e-4, dt=dt)
    assert same
    expect = np.sum(d[0] @ c) + N * dt * np.sum(d[1] @ c)
    assert abs(got - expect) < 1e-9 * (1 + abs(expect))


def test_fd_moving_plane_twist():
    # a sphere resting on a plane that moves up with speed nu_z: after each step
    # the sphere moves with the plane, so dv_N/dnu_z = 1 (the last step's twist)
    r = float(np.float32(0.01))
    pl = scenes.plane((0, 0, 0), (0, 0, 1))
    N = 4
    tw = np.zeros((N, 1, 6))
    tw[:, 0, 2] = 0.05
    d_tw = np.zeros_like(tw)
    d_tw[-1, 0, 2] = 1.0
    loss = lambda x, v: float(v[0, 2])
    got, same = fd_directional(loss, np.array([[0.0, 0.0, r - 1e-7]]), np.zeros((1, 3)), np.array([r], np.float32),
                               [pl], tw, (np.zeros((1, 3)), np.zeros((1, 3)), d_tw), 1e-6, alpha=0.0)
    assert same
    assert abs(got - 1.0) < 1e-6


def test_target_loss_gradient_matches_fd():
    rng = np.random.default_rng(1)
    L = TargetLoss((0.0, 0.0, 0.0), (0.02, 0.02, 0.01), width=1e-3, vel_weight=(0.1, -0.2, 0.3))
    x = rng.uniform(-0.03, 0.03, (50, 3))
    v = rng.normal(size=(50, 3))
    gx, gv = L.grads(x, v)
    for _ in range(5):
        dx = rng.normal(size=x.shape)
        dv = rng.normal(size=v.shape)
        h = 1e-8
        fd = (L(x + h * dx, v + h * dv) - L(x - h * dx, v - h * dv)) / (2 * h)
        an = np.sum(gx * dx) + np.sum(gv * dv)
        assert abs(fd - an) < 1e-5 * (1 + abs(an))
