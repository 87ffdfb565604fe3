"""Pins of the oracle's closed-form SDFs (Sec. II-C, Eq. (7)) against brute
force distances to densely sampled surfaces, inside tests and finite
differences; and of the binary32 decision SDF against the FP64 one."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2306_01369_amd import scenes


def _box_surface(h, k=60):
    pts = []
    g = np.linspace(-1, 1, k)
    U, V = np.meshgrid(g, g, indexing="ij")
    for a in range(3):
        b, c = [q for q in range(3) if q != a]
        for s in (-1, 1):
            P = np.zeros((k * k, 3))
            P[:, a] = s * h[a]
            P[:, b] = U.ravel() * h[b]
            P[:, c] = V.ravel() * h[c]
            pts.append(P)
    return np.concatenate(pts)


def _capsule_surface(R, h, k=80):
    th = np.linspace(0, 2 * math.pi, k, endpoint=False)
    zs = np.linspace(-h, h, k)
    T, Z = np.meshgrid(th, zs, indexing="ij")
    side = np.stack([R * np.cos(T.ravel()), R * np.sin(T.ravel()), Z.ravel()], 1)
    ph = np.linspace(0, math.pi / 2, k)
    T2, P2 = np.meshgrid(th, ph, indexing="ij")
    cap = np.stack([R * np.cos(T2.ravel()) * np.cos(P2.ravel()), R * np.sin(T2.ravel()) * np.cos(P2.ravel()),
                    R * np.sin(P2.ravel())], 1)
    top = cap + [0, 0, h]
    bot = cap * [1, 1, -1] - [0, 0, h]
    return np.concatenate([side, top, bot])


def test_box_sdf_matches_sampled_distance():
    h = (0.05, 0.03, 0.08)
    box = scenes.box_tool((0, 0, 0), h)
    surf = _box_surface(h)
    rng = np.random.default_rng(0)
    for _ in range(300):
        p = rng.uniform(-0.12, 0.12, size=3)
        f, g = O.sdf64_body_frame(box, p)
        inside = np.all(np.abs(p) < h)
        assert (f < 0) == inside
        dmin = np.min(np.linalg.norm(surf - p, axis=1))
        # the sample grid spacing bounds the sampling error
        assert abs(abs(f) - dmin) < 2.5e-3
        assert abs(np.linalg.norm(g) - 1) < 1e-12


def test_capsule_sdf_matches_sampled_distance():
    R, hl = float(np.float32(0.02)), float(np.float32(0.075))   # shape parameters are binary32
    cap = scenes.capsule_tool((0, 0, 0), R, hl)
    surf = _capsule_surface(R, hl)
    rng = np.random.default_rng(1)
    for _ in range(300):
        p = rng.uniform(-0.12, 0.12, size=3)
        f, g = O.sdf64_body_frame(cap, p)
        assert abs(abs(f) - np.min(np.linalg.norm(surf - p, axis=1))) < 2.5e-3
        # exact distance to the axis segment minus R
        z = min(max(p[2], -hl), hl)
        assert abs(f - (math.hypot(math.hypot(p[0], p[1]), p[2] - z) - R)) < 1e-15


@pytest.mark.parametrize("shape", ["box", "capsule", "plane"])
def test_sdf_gradient_matches_finite_differences(shape):
    body = {"box": scenes.box_tool((0, 0, 0), (0.05, 0.03, 0.08)),
            "capsule": scenes.capsule_tool((0, 0, 0), 0.02, 0.075),
            "plane": scenes.plane((0, 0, 0), (0, 0, 1))}[shape]
    rng = np.random.default_rng(2)
    eps = 1e-7
    for _ in range(200):
        p = rng.uniform(-0.12, 0.12, size=3)
        f, g = O.sdf64_body_frame(body, p)
        fd = np.array([(O.sdf64_body_frame(body, p + eps * e)[0] - O.sdf64_body_frame(body, p - eps * e)[0]) / (2 * eps)
                       for e in np.eye(3)])
        # skip points within eps of a crease, where the SDF is not differentiable
        if np.linalg.norm(fd) < 1 - 1e-4:
            continue
        np.testing.assert_allclose(g, fd, atol=1e-5)


def test_f32_decision_sdf_agrees_with_fp64_in_world_frame():
    rng = np.random.default_rng(3)
    bodies = [scenes.box_tool((0.1, 0.2, 0.3), (0.05, 0.03, 0.08), R=scenes.random_rotation(rng)),
              scenes.capsule_tool((0.1, 0.2, 0.3), 0.02, 0.075, R=scenes.random_rotation(rng)),
              scenes.plane((0.0, 0.0, 0.05), (0, 0, 1)), scenes.plane((0.3, 0, 0), (-1, 0, 0))]
    for b in bodies:
        Rf = np.asarray(b["R"], np.float32).astype(np.float64)
        tf = np.asarray(b["t"], np.float32).astype(np.float64)
        for _ in range(200):
            x = rng.uniform(-0.1, 0.4, size=3).astype(np.float32)
            f32 = O.sdf32(b, x)
            p = Rf.T @ (x.astype(np.float64) - tf)
            f64, _ = O.sdf64_body_frame(b, p)
            assert abs(f32 - f64) < 1e-6


def test_plane_contact_normal_and_body_velocity_in_step():
    # a sphere overlapping a tilted plane gets its impulse along the plane normal
    r = 0.01
    th = math.radians(15)
    nrm = np.array([-math.sin(th), 0.0, math.cos(th)])
    t1 = np.array([math.cos(th), 0.0, math.sin(th)])
    pl = scenes.plane((0, 0, 0), (0, 0, 1))
    pl["R"] = np.stack([t1, np.cross(nrm, t1), nrm], axis=1)
    x = (nrm * (r - 1e-4)).reshape(1, 3)
    o = O.Oracle(x, np.zeros((1, 3)), np.array([r], np.float32), [pl], gravity=(0, 0, 0), mu=0.5)
    d = o.step(detail=True)
    assert d["n_pb"] == 1
    np.testing.assert_allclose(d["normals"][0], nrm, atol=1e-6)   # pose is rounded to binary32
    np.testing.assert_allclose(d["psi"][0], -1e-4, atol=1e-8)
    P, n_c = d["impulses"][0], d["normals"][0]
    assert np.dot(P, n_c) > 0 and np.linalg.norm(np.cross(P, n_c)) < 1e-12 * np.linalg.norm(P)
