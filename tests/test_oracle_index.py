"""Pins of the oracle's block index (Sec. 3.2: collision-free, one-to-one map
from block coordinate to block index) against brute force: a Python dict for
first-occurrence indexing and a dense array over the bounding box."""
import numpy as np
import pytest


def _random_coords(rng, n, lo=-6, hi=6):
    return rng.integers(lo, hi, size=(n, 3)).astype(np.int32)


def test_build_first_occurrence_matches_dict(oracle_lib):
    rng = np.random.default_rng(11)
    coords = _random_coords(rng, 3000)  # many duplicates, negative coordinates
    blocks, idx = oracle_lib.build_grid(coords)
    seen = {}
    for c in map(tuple, coords):
        seen.setdefault(c, len(seen))
    assert blocks.shape == (len(seen), 3)
    assert [tuple(b) for b in blocks] == list(seen.keys())
    np.testing.assert_array_equal(idx, [seen[tuple(c)] for c in coords])


def test_lookup_matches_dense_array(oracle_lib):
    rng = np.random.default_rng(12)
    coords = _random_coords(rng, 700, -9, 7)
    blocks, _ = oracle_lib.build_grid(coords)
    lo = blocks.min(0) - 2
    hi = blocks.max(0) + 2
    dense = -np.ones(hi - lo + 1, np.int64)
    for i, b in enumerate(blocks):
        dense[tuple(b - lo)] = i
    grid = np.stack(np.meshgrid(*[np.arange(lo[a], hi[a] + 1) for a in range(3)],
                                indexing="ij"), -1).reshape(-1, 3).astype(np.int32)
    got = oracle_lib.lookup(blocks, grid)
    want = dense[tuple((grid - lo).T)]
    np.testing.assert_array_equal(got, want)


def test_lookup_extreme_coordinates(oracle_lib):
    lim = 1 << 20
    coords = np.array([[-lim, -lim, -lim], [lim - 1, lim - 1, lim - 1], [0, 0, 0],
                       [-lim, lim - 1, 0], [5, -7, 3]], np.int32)
    blocks, idx = oracle_lib.build_grid(coords)
    np.testing.assert_array_equal(idx, np.arange(5))
    q = np.concatenate([coords, [[lim, 0, 0], [0, -lim - 1, 0], [1, 0, 0]]]).astype(np.int32)
    np.testing.assert_array_equal(oracle_lib.lookup(blocks, q), [0, 1, 2, 3, 4, -1, -1, -1])


@pytest.mark.parametrize("bad", [[1 << 20, 0, 0], [0, -(1 << 20) - 1, 0], [0, 0, 2 ** 31 - 1]])
def test_build_rejects_out_of_range(oracle_lib, bad):
    coords = np.array([[0, 0, 0], bad], np.int32)
    with pytest.raises(ValueError):
        oracle_lib.build_grid(coords)


def test_neighbors_brute_force(oracle_lib):
    rng = np.random.default_rng(13)
    blocks, _ = oracle_lib.build_grid(_random_coords(rng, 400, -4, 4))
    nbr = oracle_lib.neighbors(blocks)
    pos = {tuple(b): i for i, b in enumerate(blocks)}
    for i, b in enumerate(blocks):
        for s in range(8):
            q = (b[0] + (s & 1), b[1] + ((s >> 1) & 1), b[2] + ((s >> 2) & 1))
            assert nbr[i, s] == pos.get(q, -1)


def test_sphere_block_count():
    """The sphere workload: blocks within a 4-voxel band of |x| = 0.5 m at
    h = 1/64 m.  494 is the count of the band rule, computed independently
    by brute force over every voxel of the [-1,1]^3 cube here."""
    from synth import workloads
    w = workloads.sphere_tiny()
    h = 1.0 / 64
    i = np.arange(-64, 64)
    X, Y, Z = np.meshgrid(i, i, i, indexing="ij")
    d = np.sqrt((X * h) ** 2 + (Y * h) ** 2 + (Z * h) ** 2) - 0.5
    near = np.abs(d) <= 4 * h
    blocks = {(x // 8, y // 8, z // 8) for x, y, z in zip(X[near], Y[near], Z[near])}
    assert len(blocks) == 494
    assert set(map(tuple, w["block_coords"])) == blocks
