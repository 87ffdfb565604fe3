"""Pins of the oracle's observation functions (Sec. III-A, "Bulldozing"): depth
cameras and the goal-box reward.  Each check rests on geometry worked out
independently of the oracle's camera-frame arithmetic: closed forms for a
sphere seen along the optical axis or from above, constant depth of a plane
parallel to the image, hit points lying on the surface they hit, brute-force
sphere tracing of small scenes, and rewards of hand-placed particles."""
import numpy as np
import pytest

import oracle as O
from paper_2306_01369_amd import scenes


def _pixel_dirs(cam):
    """Camera-frame ray origin and direction of every pixel (float64), from the
    pixel-centre convention g = (idx + 1/2) * 2/size - 1."""
    W, H = cam["width"], cam["height"]
    gu = (np.arange(W) + 0.5) * (2.0 / W) - 1.0
    gv = (np.arange(H) + 0.5) * (2.0 / H) - 1.0
    p0, p1 = (float(np.float32(q)) for q in cam["params"][:2])   # the camera holds binary32
    a = p0 * gu[None, :] * np.ones((H, 1))
    b = p1 * gv[:, None] * np.ones((1, W))
    return a, b


def test_sky_camera_sees_a_sphere_on_the_ground_in_closed_form():
    cam = scenes.sky_camera(0.45, 0.55, 0.45, 0.55, 1.0, 64, 64)
    c = np.array([0.503, 0.497, 0.02], np.float32).astype(np.float64)
    r = float(np.float32(0.01))
    ground = [scenes.plane((0, 0, 0), (0, 0, 1))]
    img = O.render_depth(c[None], [r], [cam], ground)[0]
    # world point under each pixel centre (image rows run toward -y)
    a, b = _pixel_dirs(cam)
    X, Y = 0.5 + a, 0.5 - b
    rho2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2
    inside = rho2 < r * r * (1 - 1e-4)
    outside = rho2 > r * r * (1 + 1e-4)
    h = np.sqrt(np.maximum(r * r - rho2, 0))
    want = 1.0 - c[2] - h
    # output rounding plus the binary32 pixel coordinates (~1e-8 m) magnified
    # by the slope of the sphere's surface
    tol = 1.5e-7 + np.sqrt(rho2) / np.maximum(h, 1e-30) * 1e-8
    assert inside.sum() > 100
    assert np.all(np.abs(img[inside] - want[inside]) <= tol[inside])
    assert np.all(img[outside] == np.float32(1.0))


def test_perspective_camera_sees_a_sphere_on_its_axis_in_closed_form():
    eye, ctr, r = np.array([0.5, 0.5, 1.0]), np.array([0.5, 0.5, 0.2]), 0.05
    cam = scenes.perspective_camera(eye, ctr, 20.0, 96, 72, 5.0, up=(0, 1, 0))
    ground = [scenes.plane((0, 0, 0), (0, 0, 1))]
    img = O.render_depth(ctr[None], [r], [cam], ground)[0]
    a, b = _pixel_dirs(cam)
    cosb = 1.0 / np.sqrt(a * a + b * b + 1.0)
    sinb = np.sqrt(1.0 - cosb ** 2)
    L = 0.8
    alpha = np.arcsin(r / L)
    beta = np.arccos(np.clip(cosb, -1, 1))
    hit = beta < alpha * (1 - 1e-4)
    miss = beta > alpha * (1 + 1e-4)
    ell = L * cosb - np.sqrt(np.maximum(r * r - (L * sinb) ** 2, 0))
    assert hit.sum() > 200 and miss.sum() > 200
    np.testing.assert_allclose(img[hit], (ell * cosb)[hit], rtol=1e-6)
    # the ground is parallel to the image plane: camera-frame depth 1 everywhere
    np.testing.assert_allclose(img[miss], 1.0, rtol=1e-6)


def test_plane_hit_points_lie_on_the_plane_from_any_tilt():
    ground = [scenes.plane((0, 0, 0), (0, 0, 1))]
    for pitch in (10.0, 35.0, 60.0):
        eye = np.array([0.0, 0.0, 0.3])
        tgt = eye + np.array([np.cos(np.radians(pitch)), 0.0, -np.sin(np.radians(pitch))])
        cam = scenes.perspective_camera(eye, tgt, 50.0, 40, 30, 100.0)
        img = O.render_depth(np.zeros((0, 3)), np.zeros(0), [cam], ground)[0].astype(np.float64)
        a, b = _pixel_dirs(cam)
        R = np.asarray(cam["pose"], np.float32)[:, :3].astype(np.float64)
        d = np.stack([a, b, np.ones_like(a)], -1) @ R.T
        z = np.float32(eye[2]).astype(np.float64) + img * d[..., 2]
        reach = -0.3 / 100.0        # rays that meet the plane before `far`
        down = d[..., 2] < 1.01 * reach
        assert down.sum() > 100
        np.testing.assert_allclose(z[down], 0.0, atol=1e-6 * img[down].max())
        assert np.all(img[d[..., 2] > 0.99 * reach] == np.float32(100.0))


def _trace(o, d, centres, radii, planes, far):
    """Sphere tracing of one ray against spheres and half spaces."""
    dl = np.linalg.norm(d)
    dn = d / dl
    ell = 0.0
    for _ in range(20000):
        p = o + ell * dn
        f = np.min(np.linalg.norm(centres - p, axis=1) - radii) if len(radii) else np.inf
        for (n, q) in planes:
            f = min(f, float(np.dot(n, p - q)))
        if f < 1e-11:
            return ell / dl
        ell += f
        if ell / dl > far:
            return far
    raise AssertionError("sphere tracing did not converge")


@pytest.mark.parametrize("kind", ["ortho", "perspective"])
def test_depth_matches_sphere_tracing_on_a_small_scene(kind):
    rng = np.random.default_rng(5)
    n = 40
    centres = np.column_stack([rng.uniform(0.4, 0.6, n), rng.uniform(0.4, 0.6, n), rng.uniform(0.01, 0.08, n)])
    radii = rng.uniform(0.008, 0.02, n)
    centres = centres.astype(np.float32).astype(np.float64)
    radii = radii.astype(np.float32).astype(np.float64)
    wall = 0.37 if kind == "ortho" else 0.45     # every ray starts on the free side
    bodies = [scenes.plane((0, 0, 0), (0, 0, 1)), scenes.plane((wall, 0, 0), (1, 0, 0))]
    planes = [(np.array([0.0, 0, 1]), np.zeros(3)), (np.array([1.0, 0, 0]), np.array([wall, 0, 0]))]
    if kind == "ortho":
        cam = scenes.sky_camera(0.38, 0.62, 0.38, 0.62, 0.5, 24, 24, far=0.6)
    else:
        cam = scenes.perspective_camera((0.75, 0.3, 0.25), (0.5, 0.5, 0.03), 45.0, 24, 18, 2.0)
    img = O.render_depth(centres, radii, [cam], bodies)[0]
    pose = np.asarray(cam["pose"], np.float32).astype(np.float64)
    R, t = pose[:, :3], pose[:, 3]
    a, b = _pixel_dirs(cam)
    checked = 0
    for v in range(cam["height"]):
        for u in range(cam["width"]):
            if kind == "ortho":
                o, d = t + R @ np.array([a[v, u], b[v, u], 0.0]), R @ np.array([0.0, 0, 1])
            else:
                o, d = t, R @ np.array([a[v, u], b[v, u], 1.0])
            # skip rays grazing a sphere, where the binary32 decision may differ
            dn = d / np.linalg.norm(d)
            rel = centres - o
            s = rel @ dn
            perp = np.sqrt(np.maximum(np.sum(rel * rel, 1) - s * s, 0))
            if np.any((np.abs(perp - radii) < 1e-4 * radii) & (s > 0)):
                continue
            want = _trace(o, d, centres, radii, planes, cam["params"][2])
            assert abs(img[v, u] - want) <= 1e-6 * max(1.0, want), (v, u, img[v, u], want)
            checked += 1
    assert checked > 0.9 * cam["width"] * cam["height"]


def test_depth_is_independent_of_particle_order_and_separates_envs():
    rng = np.random.default_rng(2)
    n = 600
    x = np.column_stack([rng.uniform(0, 0.2, n), rng.uniform(0, 0.2, n), rng.uniform(0.005, 0.05, n)])
    r = rng.uniform(0.003, 0.006, n)
    cams = [scenes.sky_camera(0, 0.2, 0, 0.2, 0.3, 40, 32),
            scenes.perspective_camera((0.3, 0.25, 0.2), (0.1, 0.1, 0.02), 60.0, 32, 24, 1.0)]
    ground = [scenes.plane((0, 0, 0), (0, 0, 1))]
    base = O.render_depth(x, r, cams, ground)
    perm = rng.permutation(n)
    again = O.render_depth(x[perm], r[perm], cams, ground)
    for p, q in zip(base, again):
        assert np.array_equal(p, q)
    # two environments: each camera sees only its own particles and planes
    half = n // 2
    cams2 = [dict(c, env=e) for e in (0, 1) for c in cams]
    ground2 = [scenes.plane((0, 0, 0), (0, 0, 1), env=0), scenes.plane((0, 0, 0), (0, 0, 1), env=1)]
    both = O.render_depth(x, r, cams2, ground2, env_offsets=[0, half, n])
    first = O.render_depth(x[:half], r[:half], cams, ground)
    second = O.render_depth(x[half:], r[half:], cams, ground)
    for got, want in zip(both, first + second):
        assert np.array_equal(got, want)
    # a pixel subset returns exactly those entries
    flat = np.concatenate([im.ravel() for im in base])
    pix = rng.choice(flat.size, 97, replace=False)
    assert np.array_equal(O.render_depth(x, r, cams, ground, pixels=pix), flat[pix])


def test_camera_inside_a_sphere_or_behind_it_ignores_that_sphere():
    cam = scenes.perspective_camera((0, 0, 0.5), (0, 0, 0), 40.0, 8, 8, 3.0, up=(0, 1, 0))
    ground = [scenes.plane((0, 0, 0), (0, 0, 1))]
    x = np.array([[0.0, 0.0, 0.5],      # contains the camera
                  [0.0, 0.0, 0.9]])     # behind it
    img = O.render_depth(x, [0.05, 0.2], [cam], ground)[0]
    np.testing.assert_allclose(img, 0.5, rtol=1e-6)


def test_goal_reward_closed_forms():
    lo, hi = np.array([0.1, 0.2, 0.0]), np.array([0.3, 0.4, 0.1])
    box = np.concatenate([lo, hi])[None]
    rng = np.random.default_rng(0)
    x = rng.uniform(lo, hi, (50, 3))
    rew, ins = O.goal_reward(x, box)
    assert rew[0] == 100.0 and ins[0] == 50
    # particles on the faces and corners are inside (closed box)
    corners = np.array([[lo[0], lo[1], lo[2]], [hi[0], hi[1], hi[2]], [lo[0], hi[1], 0.05]], np.float32)
    rew, ins = O.goal_reward(corners, np.asarray(box, np.float32))
    assert ins[0] == 3 and rew[0] == 100.0
    # distances: along an axis, to an edge (3-4-5), to a corner (k sqrt 3)
    out = np.array([hi + [0.25, 0.0, 0.0] * np.array([1, 0, 0]) - [0, 0.1, 0.05],
                    [hi[0] + 0.03, hi[1] + 0.04, 0.05],
                    lo - 0.02])
    xs = np.vstack([x[:7], out]).astype(np.float32)
    d_axis = np.float64(xs[7, 0]) - np.float64(np.float32(hi[0]))
    d_edge = np.hypot(np.float64(xs[8, 0]) - np.float64(np.float32(hi[0])),
                      np.float64(xs[8, 1]) - np.float64(np.float32(hi[1])))
    d_corner = np.sqrt(np.sum((np.float64(np.float32(lo)) - xs[9].astype(np.float64)) ** 2))
    rew, ins = O.goal_reward(xs, np.asarray(box, np.float32))
    assert ins[0] == 7
    assert abs(d_edge - 0.05) < 1e-7 and abs(d_corner - 0.02 * np.sqrt(3)) < 1e-7
    assert rew[0] == pytest.approx((700.0 - d_axis - d_edge - d_corner) / 10, rel=1e-14)


def test_goal_reward_per_environment():
    lo, hi = np.zeros(3), np.full(3, 0.1)
    x = np.array([[0.05, 0.05, 0.05], [0.2, 0.05, 0.05], [0.05, 0.05, 0.05]])
    boxes = np.array([np.concatenate([lo, hi]), np.concatenate([lo, hi]), np.concatenate([lo + 1, hi + 1])])
    rew, ins = O.goal_reward(x, boxes, env_offsets=[0, 2, 2, 3])
    assert list(ins) == [1, 0, 0]
    assert rew[0] == pytest.approx((100.0 - (float(np.float32(0.2)) - float(np.float32(0.1)))) / 2, rel=1e-12)
    assert rew[1] == 0.0
    assert rew[2] == pytest.approx(-np.sqrt(3) * (1.0 - 0.05), rel=1e-6)
