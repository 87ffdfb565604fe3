"""Pins of the oracle's contact detection (Sec. II-B, II-C, Eq. (7)).

The hash-grid contact list must equal the O(n^2) definition exactly, for any
table size and any admissible cell size; the binary32 predicate is pinned on
exact ties and against an FP64 evaluation away from ties."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2306_01369_amd import scenes


def _set(pairs):
    return set(map(tuple, np.asarray(pairs).tolist()))


def test_pair_predicate_exact_touch_and_next_float():
    r = np.float32(0.5)
    a = np.array([0.0, 0.0, 0.0], np.float32)
    b = np.array([1.0, 0.0, 0.0], np.float32)
    assert O.pair_touch(a, b, r, r)                    # distance exactly r_i + r_j: "<=" holds
    b2 = np.array([np.nextafter(np.float32(1.0), np.float32(2.0)), 0, 0], np.float32)
    assert not O.pair_touch(a, b2, r, r)
    b3 = np.array([np.nextafter(np.float32(1.0), np.float32(0.0)), 0, 0], np.float32)
    assert O.pair_touch(a, b3, r, r)


def test_pair_predicate_agrees_with_fp64_away_from_ties():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 0.02, size=(4000, 2, 3)).astype(np.float32)
    r = rng.uniform(0.002, 0.006, size=(4000, 2)).astype(np.float32)
    for k in range(4000):
        d2 = float(np.sum((x[k, 0].astype(np.float64) - x[k, 1]) ** 2))
        s2 = (float(r[k, 0]) + float(r[k, 1])) ** 2
        if abs(d2 - s2) < 1e-5 * s2:
            continue
        assert O.pair_touch(x[k, 0], x[k, 1], r[k, 0], r[k, 1]) == (d2 <= s2)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("n_h_kind", ["one", "seven", "2n", "pow2"])
def test_hashgrid_equals_bruteforce_random(seed, n_h_kind):
    rng = np.random.default_rng(seed)
    n = 600
    x, r = scenes.random_spheres(n, ((0, 0.06), (0, 0.06), (0, 0.06)), 0.004, rng, r_jitter=0.2)
    n_h = {"one": 1, "seven": 7, "2n": 2 * n, "pow2": 1 << 12}[n_h_kind]
    c, inv_c = O.default_cell(r)
    grid, cand = O.pp_hashgrid(x, r, inv_c, n_h)
    brute = O.pp_bruteforce(x, r)
    assert len(brute) > 50
    assert _set(grid) == _set(brute)
    assert len(grid) == len(_set(grid))            # no duplicates despite aliasing
    assert np.all(grid[:, 0] < grid[:, 1])
    assert cand >= 2 * len(brute)


def test_hashgrid_independent_of_cell_size():
    rng = np.random.default_rng(4)
    x, r = scenes.random_spheres(500, ((0, 0.05), (0, 0.05), (0, 0.05)), 0.004, rng)
    brute = _set(O.pp_bruteforce(x, r))
    for scale in (1.0, 1.3, 2.0, 3.7):
        c = float(np.float32(2 * 0.004 * (1 + 2 ** -10) * scale))
        inv_c = float(np.float32(1.0) / np.float32(c))
        for nh in (1, 97, 1000):
            assert _set(O.pp_hashgrid(x, r, inv_c, nh)[0]) == brute


def test_hashgrid_exactly_touching_lattice():
    # spacing exactly 2r in binary32 (r = 0.5, integers): every face pair touches
    # with D == S, diagonals do not.  Negative coordinates exercise kappa < q.
    g = np.arange(-3, 4, dtype=np.float32)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1).astype(np.float32)
    r = np.full(len(x), 0.5, np.float32)
    c, inv_c = O.default_cell(r)
    grid = _set(O.pp_hashgrid(x, r, inv_c, 2 * len(x))[0])
    brute = _set(O.pp_bruteforce(x, r))
    assert grid == brute
    assert len(brute) == 3 * 7 * 7 * 6      # face bonds of a 7^3 cubic lattice


def test_bruteforce_counts_on_known_configurations():
    # a chain of 5 spheres with gaps of 0, -1e-3 (overlap), +1e-3, 0
    r = np.float32(0.5)
    xs = [0.0, 1.0, 1.999, 3.0, 4.0]
    x = np.array([[v, 0, 0] for v in xs], np.float32)
    pairs = _set(O.pp_bruteforce(x, np.full(5, r, np.float32)))
    assert pairs == {(0, 1), (1, 2), (3, 4)}


def test_env_segments_never_collide():
    rng = np.random.default_rng(5)
    x, r = scenes.random_spheres(400, ((0, 0.04), (0, 0.04), (0, 0.04)), 0.004, rng)
    env = (np.arange(400) % 3).astype(np.int32)
    c, inv_c = O.default_cell(r)
    g = _set(O.pp_hashgrid(x, r, inv_c, 800, env=env)[0])
    b = _set(O.pp_bruteforce(x, r, env=env))
    assert g == b
    assert all(env[i] == env[j] for i, j in b)
    assert len(_set(O.pp_bruteforce(x, r))) > len(b)


def test_drop_scene_initially_contact_free_between_particles():
    s = scenes.drop_scene()
    c, inv_c = O.default_cell(s.radius)
    assert len(O.pp_hashgrid(s.x, s.radius, inv_c, 2 * s.n)[0]) == 0


def test_packed_bed_has_six_face_contacts_inside():
    # the resting-bed recipe: compressed cubic layers, every face pair overlaps
    rng = np.random.default_rng(0)
    side = 0.004 + 7 * 0.004 * (1 - 1e-3) + 1e-6        # room for exactly 8 x 8 per layer
    pos = scenes.packed_bed(8 * 8 * 8, 0.002, 0.0, side, 0.0, side, rng)
    x = pos.astype(np.float32)
    r = np.full(len(x), 0.002, np.float32)
    brute = O.pp_bruteforce(x, r)
    deg = np.bincount(brute.ravel(), minlength=len(x))
    assert deg.max() == 6
    assert len(brute) == 3 * 8 * 8 * 7       # all face bonds of the 8^3 block, no diagonals


def test_body_contacts_plane_and_box():
    r = np.float32(0.01)
    ground = scenes.plane((0, 0, 0), (0, 0, 1))
    wall = scenes.plane((0.5, 0, 0), (-1, 0, 0))
    box = scenes.box_tool((0.2, 0.2, 0.2), (0.05, 0.05, 0.05))
    x = np.array([[0.1, 0.1, 0.01],      # touching ground exactly
                  [0.1, 0.1, 0.0101],    # just above
                  [0.49, 0.3, 0.3],      # touching the wall x = 0.5 from inside
                  [0.26, 0.2, 0.2],      # 1 cm off the box face: touching
                  [0.2, 0.2, 0.2],       # inside the box
                  [0.2605, 0.2605, 0.2]],  # near an edge, outside by > r
                 np.float32)
    pb = _set(O.pb_contacts(x, np.full(len(x), r, np.float32), [ground, wall, box]))
    assert (0, 0) in pb and (1, 0) not in pb
    assert (2, 1) in pb
    assert (3, 2) in pb and (4, 2) in pb
    assert (5, 2) not in pb
