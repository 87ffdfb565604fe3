"""Pins of the oracle's forward-mode (dual-number) step: its value part is the
plain step bit for bit; its tangents match closed forms (free fall, the pose
update) and FP64 central differences on smooth runs."""
import numpy as np

import oracle as O
from paper_2306_01369_amd import scenes
from gradcheck import TargetLoss, fd_directional, jvp_directional


def _tool_bed(n=600, seed=0):
    s = scenes.column_scene(n=n, r=0.004, seed=seed)
    top = float(s.x[:, 2].max())
    tool = scenes.box_tool((0.03, 0.03, top + 0.006), (0.01, 0.01, 0.01), nu=(0.1, 0.0, -0.3),
                           omega=(0.5, 1.0, 0.2))
    return s, s.bodies + [tool]


def test_value_part_is_the_plain_step_bitwise():
    s, bodies = _tool_bed()
    a = O.Oracle(s.x.astype(np.float64), s.v.astype(np.float64), s.radius, bodies)
    b = O.Oracle(s.x.astype(np.float64), s.v.astype(np.float64), s.radius, bodies)
    b.start_tangents(np.random.default_rng(0).normal(size=(s.n, 3)), np.random.default_rng(1).normal(size=(s.n, 3)))
    for k in range(8):
        a.step()
        b.step_jvp()
        assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v), k
        assert np.array_equal(a.stats, b.stats)
    for q in range(len(bodies)):
        assert a.body_pose(q)[0].tobytes() == b.body_pose(q)[0].tobytes()
        assert a.body_pose(q)[1].tobytes() == b.body_pose(q)[1].tobytes()


def test_free_fall_tangents_closed_form():
    # no contacts: x_N = x0 + dt sum_k v_k, v_k = v0 + k dt g, so
    # dx_N = dx0 + N dt dv0 and dv_N = dv0
    rng = np.random.default_rng(3)
    n, N, dt = 50, 12, 1e-3
    x = rng.uniform(0, 1, (n, 3)) * 10.0
    v = rng.normal(size=(n, 3))
    orc = O.Oracle(x, v, np.full(n, 0.001, np.float32), [], dt=dt)
    dx, dv = rng.normal(size=(n, 3)), rng.normal(size=(n, 3))
    orc.start_tangents(dx, dv)
    for _ in range(N):
        orc.step_jvp()
    np.testing.assert_allclose(orc.dv, dv, rtol=0, atol=1e-15)
    np.testing.assert_allclose(orc.dx, dx + N * dt * dv, rtol=1e-13, atol=1e-15)


def test_pose_tangent_matches_differences_of_the_pose_update():
    # a body spun by omega (and one at rest, where Exp is expanded to first
    # order): the tangent of R and t after 5 steps against central differences
    # of the oracle's own Rodrigues update
    rng = np.random.default_rng(4)
    for omega in ((0.7, -1.1, 2.0), (0.0, 0.0, 0.0)):
        b = scenes.box_tool((0.1, 0.2, 0.3), (0.01, 0.02, 0.03), nu=(0.1, -0.2, 0.3), omega=omega,
                            R=scenes.random_rotation(rng))
        dtw = rng.normal(size=6)
        orc = O.Oracle(np.zeros((1, 3)) + 50.0, np.zeros((1, 3)), np.full(1, 0.001, np.float32), [b])
        orc.start_tangents()
        for _ in range(5):
            orc.set_twist_tangents([dtw])
            orc.step_jvp()
        h = 1e-7
        poses = []
        for sgn in (1.0, -1.0):
            arr = O.bodies_to_f32_pose(O.make_bodies([b]), 1)    # the oracle's starting pose
            for q in range(3):
                arr[0].nu[q] += sgn * h * dtw[q]
                arr[0].omega[q] += sgn * h * dtw[3 + q]
            for _ in range(5):
                O.lib().ggo_advance_bodies(1, arr, 1e-3)
            poses.append((np.array(arr[0].R[:]), np.array(arr[0].t[:])))
        fdR = (poses[0][0] - poses[1][0]) / (2 * h)
        fdt = (poses[0][1] - poses[1][1]) / (2 * h)
        np.testing.assert_allclose(np.array(orc.dB[0].R[:]), fdR, rtol=0, atol=1e-7)
        np.testing.assert_allclose(np.array(orc.dB[0].t[:]), fdt, rtol=0, atol=1e-8)


def _colliding(n=400, seed=7, steps=6):
    r = 0.004
    rng = np.random.default_rng(seed)
    x, rad = scenes.loose_lattice(n, r, (0.01, 0.01, 0.01), rng, spacing_factor=2.02, jitter_frac=0.06)
    v = (0.3 * rng.normal(size=(n, 3))).astype(np.float32)
    side = 0.01 + 2.02 * r * 8
    cap = scenes.capsule_tool((side / 2, side / 2, side / 2), 0.008, 0.015, R=scenes.random_rotation(rng))
    bodies = scenes.walled_box(0.0, side, 0.0, side) + [cap]
    tw = np.zeros((steps, len(bodies), 6))
    tw[:, -1, :3] = (0.2, -0.1, 0.1)
    tw[:, -1, 3:] = (2.0, 1.0, -1.0)
    loss = TargetLoss((side * 0.6, side * 0.6, side * 0.6), (0.015, 0.02, 0.015), width=2e-3,
                      vel_weight=(0.02, -0.01, 0.03))
    return x.astype(np.float64), v.astype(np.float64), rad, bodies, tw, loss


def test_dual_numbers_match_central_differences_on_colliding_grains():
    x, v, r, bodies, tw, loss = _colliding()
    rng = np.random.default_rng(11)
    for kind in ("x0", "v0", "twist", "all"):
        dx = rng.normal(size=x.shape) if kind in ("x0", "all") else np.zeros(x.shape)
        dv = rng.normal(size=v.shape) if kind in ("v0", "all") else np.zeros(v.shape)
        dtw = np.zeros_like(tw)
        if kind in ("twist", "all"):
            dtw[:, -1, :] = rng.normal(size=(tw.shape[0], 6))
        jv = jvp_directional(loss, x, v, r, bodies, tw, (dx, dv, dtw), gravity=(0.0, 0.0, 0.0))
        h = 1e-8 / max(np.abs(dx).max(), np.abs(dv).max(), np.abs(dtw).max())
        fd, same = fd_directional(loss, x, v, r, bodies, tw, (dx, dv, dtw), h, gravity=(0.0, 0.0, 0.0))
        assert same
        assert abs(jv - fd) <= 1e-5 * abs(fd), (kind, jv, fd)


def test_dual_numbers_with_plain_masses_and_relaxation():
    x, v, r, bodies, tw, loss = _colliding(n=250, seed=9, steps=4)
    rng = np.random.default_rng(12)
    dx, dv = rng.normal(size=x.shape), rng.normal(size=v.shape)
    dtw = np.zeros_like(tw)
    dtw[:, -1, :] = rng.normal(size=(tw.shape[0], 6))
    kw = dict(gravity=(0.0, 0.0, 0.0), mass_split=False, relax=0.7, n_iters=5)
    jv = jvp_directional(loss, x, v, r, bodies, tw, (dx, dv, dtw), **kw)
    h = 1e-8 / max(np.abs(dx).max(), np.abs(dv).max(), np.abs(dtw).max())
    fd, same = fd_directional(loss, x, v, r, bodies, tw, (dx, dv, dtw), h, **kw)
    assert same
    assert abs(jv - fd) <= 1e-5 * abs(fd), (jv, fd)


def test_dual_numbers_with_a_grid_body():
    # a spinning bowl sampled on a grid among colliding grains: the dual
    # numbers through the trilinear interpolant and its gradient
    x, v, r, bodies, tw, loss = _colliding(n=300, seed=13, steps=5)
    side = 0.01 + 2.02 * 0.004 * 8
    bowl = scenes.grid_tool(scenes.bowl_grid(0.012, 0.003, 0.006, 1024.0), (side / 2, side / 2, side / 2),
                            R=scenes.random_rotation(np.random.default_rng(5)))
    bodies = bodies[:-1] + [bowl]
    rng = np.random.default_rng(14)
    dx, dv = rng.normal(size=x.shape), rng.normal(size=v.shape)
    dtw = np.zeros_like(tw)
    dtw[:, -1, :] = rng.normal(size=(tw.shape[0], 6))
    kw = dict(gravity=(0.0, 0.0, 0.0))
    jv = jvp_directional(loss, x, v, r, bodies, tw, (dx, dv, dtw), **kw)
    h = 1e-8 / max(np.abs(dx).max(), np.abs(dv).max(), np.abs(dtw).max())
    fd, same = fd_directional(loss, x, v, r, bodies, tw, (dx, dv, dtw), h, **kw)
    assert same
    assert abs(jv - fd) <= 1e-5 * abs(fd), (jv, fd)


def test_separating_contact_with_zero_tangential_velocity_has_zero_derivative():
    # A sphere touching a ground plane that slides along x at 0.1 m/s; the
    # sphere moves with the plane along x (relative tangential velocity exactly
    # zero) and leaves it upward.  The normal part of y is negative, so the
    # projection maps y to zero on a whole neighbourhood: the step does not
    # depend on the plane's velocity, and central differences give zero.  The
    # tangential test alone (0 > 0 is false) would keep the tangent of y_t and
    # make the sphere follow a perturbed plane.
    r = 0.004
    ground = scenes.plane((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    ground["nu"] = np.array([0.1, 0.0, 0.0])
    x = np.array([[0.0, 0.0, r - 1e-6]])
    v = np.array([[0.1, 0.0, 0.5]])
    kw = dict(dt=1e-3, alpha=0.2, mu=0.5, gravity=(0.0, 0.0, 0.0))
    tw = np.array([[[0.1, 0.0, 0.0, 0.0, 0.0, 0.0]]])
    for comp in range(3):
        dtw = np.zeros_like(tw)
        dtw[0, 0, comp] = 1.0
        loss = TargetLoss((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), width=1e-3, vel_weight=(1.0, 1.0, 1.0))
        z = np.zeros((1, 3))
        ref = jvp_directional(loss, x, v, np.full(1, r, np.float32), [ground], tw, (z, z, dtw), **kw)
        fd, same = fd_directional(loss, x, v, np.full(1, r, np.float32), [ground], tw, (z, z, dtw), 1e-7, **kw)
        assert same
        assert abs(fd) < 1e-9, (comp, fd)
        assert ref == 0.0, (comp, ref)


def test_frictionless_contact_with_zero_tangential_velocity_ignores_the_body_sliding():
    # A sphere pressed onto a frictionless ground plane that slides along x,
    # moving with it (relative tangential velocity exactly zero).  Without
    # friction the plane's tangential velocity cannot act on the sphere: the
    # disk of radius mu y_n = 0 drops the tangential part on a neighbourhood,
    # so the derivative with respect to nu_x and nu_y is zero (central
    # differences agree), while nu_z (normal) acts.
    r = 0.004
    ground = scenes.plane((0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    ground["nu"] = np.array([0.1, 0.0, 0.0])
    x = np.array([[0.0, 0.0, r - 1e-5]])
    v = np.array([[0.1, 0.0, -0.05]])
    kw = dict(dt=1e-3, alpha=0.2, mu=0.0, gravity=(0.0, 0.0, -9.81))
    tw = np.array([[[0.1, 0.0, 0.0, 0.0, 0.0, 0.0]]])
    loss = TargetLoss((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), width=1e-3, vel_weight=(1.0, 1.0, 1.0))
    z = np.zeros((1, 3))
    for comp in range(3):
        dtw = np.zeros_like(tw)
        dtw[0, 0, comp] = 1.0
        ref = jvp_directional(loss, x, v, np.full(1, r, np.float32), [ground], tw, (z, z, dtw), **kw)
        fd, same = fd_directional(loss, x, v, np.full(1, r, np.float32), [ground], tw, (z, z, dtw), 1e-7, **kw)
        assert same
        if comp < 2:
            assert abs(fd) < 1e-9 and ref == 0.0, (comp, fd, ref)
        else:
            assert abs(ref - fd) <= 1e-6 * abs(fd) and abs(fd) > 0.1, (fd, ref)
