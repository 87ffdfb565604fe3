"""Host logic of the launch-shape autotuner."""
import numpy as np

from paper_2306_01369_amd import autotune, scenes


def test_node_dims_follow_morton_interleaving():
    # x takes bits 0, 3, 6, ...; y bits 1, 4, ...; z bits 2, 5, ...
    assert autotune.node_dims(0) == (1, 1, 1)
    assert autotune.node_dims(1) == (2, 1, 1)
    assert autotune.node_dims(2) == (2, 2, 1)
    assert autotune.node_dims(3) == (2, 2, 2)
    assert autotune.node_dims(6) == (4, 4, 4)
    assert autotune.node_dims(7) == (8, 4, 4)
    for s in range(12):
        dx, dy, dz = autotune.node_dims(s)
        assert dx * dy * dz == 2 ** s


def test_particles_per_cell_of_packed_bed():
    rng = np.random.default_rng(0)
    x = scenes.packed_bed(4000, 0.002, 0.0, 0.1, 0.0, 0.1, rng)
    ppc = autotune.particles_per_cell(x, np.full(len(x), 0.002, np.float32))
    assert 0.9 < ppc < 1.6


def test_candidates_fit_the_lds_budget():
    for ppc in (0.5, 1.2, 3.0, 7.0):
        cands = autotune.candidates(ppc)
        assert cands, ppc
        for c in cands:
            dx, dy, dz = autotune.node_dims(c["tile_node_shift"])
            assert c["tile_max_cells"] >= (dx + 2) * (dy + 2) * (dz + 2)
            lds = (2 * c["tile_max_cells"] + 1) * 4 + c["tile_max_stage"] * 24
            assert lds <= 64 * 1024
            assert c["tile_threads"] in (64, 128, 256)
            assert c["tile_max_stage"] <= 2048 and c["tile_max_cells"] <= 4096


def test_hash_sizes_tried_exclude_the_default_and_stay_positive():
    f = autotune.hash_factors()
    assert 2.0 not in f and all(x > 0 for x in f)


def test_cell_sizes_tried_start_at_the_smallest_admissible_cell():
    f = autotune.cell_factors()
    assert f[0] == 1.0 and all(b > a for a, b in zip(f, f[1:]))


def test_lane_counts_are_the_supported_ones():
    assert set(autotune.lane_counts()) == {1, 2, 4}
