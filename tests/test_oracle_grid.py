"""Pins of the oracle's grid SDF bodies (pre-computed SDF samples on a regular
grid with trilinear interpolation, Sec. II-C): exact for affine fields,
knot values reproduced, second-order convergence to a smooth field,
gradient against differences, outside points never in contact, and a grid
of a plane's distance behaving like the analytic plane in a step."""
import numpy as np

import oracle as O
from paper_2306_01369_amd import scenes


def _body(grid, center=(0.0, 0.0, 0.0)):
    return scenes.grid_tool(grid, center)


def test_affine_field_is_reproduced_exactly():
    n = np.array([0.3, -0.5, 0.81])
    n /= np.linalg.norm(n)
    g = scenes.affine_grid(n, 0.01, (-0.05, -0.04, -0.03), (0.05, 0.04, 0.03), 256.0)
    b = _body(g)
    rng = np.random.default_rng(0)
    vals = np.asarray(g["values"], np.float64)
    # the interpolant of binary32 knot values: affine in p up to the rounding
    # of the knot values (|error| <= max rounding of a knot)
    tol = np.abs(vals).max() * 2.0 ** -23
    for p in rng.uniform((-0.049, -0.039, -0.029), (0.049, 0.039, 0.029), size=(200, 3)):
        f, gr = O.sdf64_body_frame(b, p)
        assert abs(f - (p @ n - 0.01)) <= tol + 1e-15
        # gradient of an affine field is the normal (up to knot rounding / spacing)
        assert np.abs(gr / np.linalg.norm(gr) - n).max() <= 1e-5


def test_knot_values_are_reproduced():
    g = scenes.ball_grid(0.02, 0.01, 512.0)
    b = _body(g)
    v = np.asarray(g["values"], np.float64)
    o = np.asarray(g["origin"], np.float64)
    rng = np.random.default_rng(1)
    nz, ny, nx = v.shape
    for _ in range(100):
        a, c, e = rng.integers(0, nx), rng.integers(0, ny), rng.integers(0, nz)
        p = o + np.array([a, c, e]) / 512.0
        f, _ = O.sdf64_body_frame(b, p)
        assert f == v[e, c, a]


def test_second_order_convergence_to_a_smooth_field():
    # ball distance sampled at h, h/2, h/4: the interpolation error in the
    # shell around the surface shrinks ~4x per halving
    rng = np.random.default_rng(2)
    dirs = rng.normal(size=(300, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    pts = dirs * rng.uniform(0.015, 0.025, size=(300, 1))
    errs = []
    for ih in (256.0, 512.0, 1024.0):
        b = _body(scenes.ball_grid(0.02, 0.008, ih))
        e = max(abs(O.sdf64_body_frame(b, p)[0] - (np.linalg.norm(p) - 0.02)) for p in pts)
        errs.append(e)
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs
    assert errs[2] < 3e-5       # ~h^2 / (8 R) at h = 1/1024 m


def test_gradient_matches_differences_inside_a_cell():
    b = _body(scenes.bowl_grid(0.03, 0.005, 0.006, 512.0))
    rng = np.random.default_rng(3)
    h = 1e-7
    for p in rng.uniform(-0.03, 0.005, size=(100, 3)):
        f, g = O.sdf64_body_frame(b, p)
        fd = np.array([(O.sdf64_body_frame(b, p + h * e)[0] - O.sdf64_body_frame(b, p - h * e)[0]) / (2 * h)
                       for e in np.eye(3)])
        # a difference across a cell face mixes two cells; only compare inside
        u = (p - np.asarray(b["grid"]["origin"], np.float64)) * 512.0
        if np.any(np.abs(u - np.round(u)) < 1e-3):
            continue
        assert np.abs(fd - g).max() <= 1e-6 * max(1.0, np.abs(g).max())


def test_points_outside_the_grid_are_never_in_contact():
    g = scenes.ball_grid(0.02, 0.004, 256.0)
    b = _body(g)
    x = np.array([[0.0, 0.0, 0.03], [0.0, -0.05, 0.0], [0.1, 0.1, 0.1]], np.float32)
    for p in x:
        assert O.sdf32(b, p) > 1e30
    # just inside: the binary32 interpolant
    assert abs(O.sdf32(b, np.array([0.0, 0.0, 0.0239], np.float32)) - (0.0239 - 0.02)) < 2e-4


def test_grid_of_a_plane_distance_acts_like_the_plane():
    # a resting column on the analytic ground plane and on a grid holding the
    # same plane's distance: same contacts, impulses equal to the knot rounding
    s = scenes.column_scene(n=400, r=0.004)
    lo, hi = (-0.01, -0.01, -0.02), (0.09, 0.09, 0.02)
    grid = scenes.affine_grid((0.0, 0.0, 1.0), 0.0, lo, hi, 256.0)
    floor_grid = _body(grid)
    a = O.Oracle(s.x.astype(np.float64), s.v.astype(np.float64), s.radius, s.bodies)
    b = O.Oracle(s.x.astype(np.float64), s.v.astype(np.float64), s.radius, [floor_grid] + s.bodies[1:])
    da, db = a.step(detail=True), b.step(detail=True)
    np.testing.assert_array_equal(da["pairs"], db["pairs"])
    assert da["n_pb"] == db["n_pb"] > 0
    assert np.abs(da["impulses"] - db["impulses"]).max() <= 1e-9 * np.abs(da["impulses"]).max()
