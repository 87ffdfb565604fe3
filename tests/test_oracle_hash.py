"""Pins of the oracle's cell coordinates and spatial hash (Eq. (6), Sec. II-B)."""
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hash_eq6.txt")


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(tuple(int(t) for t in line.split()))
    return rows


@pytest.mark.parametrize("row", _golden())
def test_hash_golden(row):
    k0, k1, k2, nh, h = row
    assert O.spatial_hash((k0, k1, k2), nh) == h


def test_hash_origin_cell_is_zero_for_any_table():
    # kappa = (q, q, q) makes every product zero, so the XOR and the bucket are 0.
    for nh in (1, 2, 3, 7, 1000, 2 ** 21, 2 ** 31 - 1):
        assert O.spatial_hash((100, 100, 100), nh) == 0


def test_hash_single_axis_is_prime_multiple():
    # With two coordinates at q the hash is p_a*(k_a - q) mod n_h for the third.
    p = (73856093, 19349663, 83492791)
    nh = 1_000_003
    for a in range(3):
        for d in (-7, -1, 1, 5, 123):
            k = [100, 100, 100]
            k[a] += d
            assert O.spatial_hash(k, nh) == (p[a] * d) % nh


def test_hash_is_nonnegative_and_in_range():
    rng = np.random.default_rng(1)
    for _ in range(2000):
        k = rng.integers(-5000, 5000, size=3)
        nh = int(rng.integers(1, 10 ** 7))
        h = O.spatial_hash(k, nh)
        assert 0 <= h < nh


def test_hash_power_of_two_matches_32bit_wraparound():
    # For n_h = 2^m the bucket is the low m bits of the 64-bit two's-complement
    # XOR, which 32-bit modular arithmetic reproduces exactly.
    rng = np.random.default_rng(2)
    p = np.array([73856093, 19349663, 83492791], dtype=np.uint32)
    for m in (1, 5, 13, 21, 24, 31):
        nh = 1 << m
        for _ in range(300):
            k = rng.integers(-2 ** 20, 2 ** 20, size=3)
            d = (k - 100).astype(np.int64).astype(np.uint32)
            with np.errstate(over="ignore"):
                prod = d * p
            v = prod[0] ^ prod[1] ^ prod[2]
            assert O.spatial_hash(k, nh) == int(v) & (nh - 1)


def test_cell_coordinate_rounds_half_to_even():
    # kappa = round(x / c) with ties to even: inv_c = 1 makes x*inv_c exact.
    x = np.array([[0.5, 1.5, 2.5], [-0.5, -1.5, -2.5], [0.49999997, 1.4999999, 3.5000002]], np.float32)
    kappa, _ = O.cell_index(x, 1.0, 97)
    assert kappa.tolist() == [[0, 2, 2], [0, -2, -2], [0, 1, 4]]


def test_cell_coordinate_product_rounded_to_binary32():
    # x * inv_c is rounded once to binary32 before rounding to an integer:
    # 0.1f * 5.0f = 0.5000000074505806 in exact arithmetic but 0.5f in binary32.
    x = np.array([[0.1, 0.3, -0.1]], np.float32)
    kappa, _ = O.cell_index(x, 5.0, 97)
    assert float(np.float32(0.1) * np.float32(5.0)) == 0.5
    assert kappa.tolist() == [[0, 2, 0]]


def test_cell_index_matches_golden_through_positions():
    # cell (0,0,0) and (1,0,0) at c = 4 mm: positions at the cell centres.
    c = np.float32(0.004)
    inv_c = float(np.float32(1.0) / c)
    x = np.array([[0.0, 0.0, 0.0], [0.004, 0.0, 0.0], [1.0, 1.0, 0.1]], np.float32)
    kappa, h = O.cell_index(x, inv_c, 2 ** 21)
    assert kappa[0].tolist() == [0, 0, 0] and kappa[1].tolist() == [1, 0, 0]
    assert h[0] == 1726156 and h[1] == 1924457
    assert kappa[2].tolist() == [250, 250, 25] and h[2] == 976439


def test_segmented_bucket_offset():
    x = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0]], np.float32)
    _, h = O.cell_index(x, 1.0, 8192, bucket_offset=np.array([0, 10000]), env_n_h=np.array([8192, 8192]))
    assert h.tolist() == [5836, 15836]
