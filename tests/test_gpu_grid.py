"""GPU grid build / lookup / neighbour table: bit-exact against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import dev, to_dev

pytestmark = pytest.mark.gpu


def _build(coords, return_index=True):
    import paper_2305_13220_amd as sg
    return sg.Grid(to_dev(coords, torch.int32), 0.02, (0.1, -0.2, 0.3), return_index=return_index)


@pytest.mark.parametrize("n,lo,hi,seed", [(1, -3, 3, 0), (50, -2, 2, 1), (3000, -6, 6, 2),
                                          (200000, -40, 40, 3)])
def test_build_matches_oracle(n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    coords = rng.integers(lo, hi, size=(n, 3)).astype(np.int32)
    g = _build(coords)
    blocks_or, idx_or = oracle.build_grid(coords)
    assert g.n_blocks == blocks_or.shape[0]
    np.testing.assert_array_equal(g.block_coords().cpu().numpy(), blocks_or)
    np.testing.assert_array_equal(g.index_of_input.cpu().numpy(), idx_or)
    np.testing.assert_array_equal(g.neighbors().cpu().numpy(), oracle.neighbors(blocks_or))
    # lookups over the bounding box plus a margin, and random far queries
    blo, bhi = blocks_or.min(0) - 2, blocks_or.max(0) + 2
    q = np.stack(np.meshgrid(*[np.arange(blo[a], bhi[a] + 1) for a in range(3)], indexing="ij"),
                 -1).reshape(-1, 3).astype(np.int32)
    q = np.concatenate([q, rng.integers(-2 ** 31, 2 ** 31 - 1, size=(1000, 3))]).astype(np.int32)
    np.testing.assert_array_equal(g.lookup(to_dev(q)).cpu().numpy(), oracle.lookup(blocks_or, q))
    g.destroy()


def test_extreme_coordinates_and_range_error():
    import paper_2305_13220_amd as sg
    lim = 1 << 20
    coords = np.array([[-lim, -lim, -lim], [lim - 1, lim - 1, lim - 1], [0, 0, 0],
                       [lim - 1, -lim, 5], [0, 0, 0]], np.int32)
    g = _build(coords)
    np.testing.assert_array_equal(g.index_of_input.cpu().numpy(), [0, 1, 2, 3, 2])
    q = np.array([[lim, 0, 0], [-lim - 1, 0, 0], [lim - 1, lim - 1, lim - 1]], np.int32)
    np.testing.assert_array_equal(g.lookup(to_dev(q)).cpu().numpy(), [-1, -1, 1])
    nb = g.neighbors().cpu().numpy()
    assert (nb[1] == [1, -1, -1, -1, -1, -1, -1, -1]).all()
    g.destroy()
    with pytest.raises(sg.SgridError, match="status -2"):
        _build(np.array([[0, 0, 0], [lim, 0, 0]], np.int32))


def test_sphere_grid_matches_oracle():
    from synth import workloads
    w = workloads.sphere_tiny()
    g = _build(w["block_coords"])
    np.testing.assert_array_equal(g.block_coords().cpu().numpy(), w["block_coords"])
    np.testing.assert_array_equal(g.index_of_input.cpu().numpy(), np.arange(494))
    np.testing.assert_array_equal(g.neighbors().cpu().numpy(), oracle.neighbors(w["block_coords"]))


@pytest.mark.parametrize("workload", ["sphere", "random"])
def test_dense_map_matches_brute_force(workload):
    """Map entry: index*256 + neighbour mask for allocated blocks, else minus
    the Chebyshev distance to the nearest allocated block, capped at 32."""
    from scipy import ndimage
    if workload == "sphere":
        from synth import workloads
        coords = workloads.sphere_tiny()["block_coords"]
    else:
        rng = np.random.default_rng(17)
        coords = rng.integers(-30, 40, size=(300, 3)).astype(np.int32)
    g = _build(coords, return_index=False)
    m, bmin = g.dense_map()
    assert m is not None
    m = m.cpu().numpy()
    blocks, _ = oracle.build_grid(coords)
    nbr = oracle.neighbors(blocks)
    lo = blocks.min(0)
    assert tuple(bmin) == tuple(lo)
    dims = blocks.max(0) - lo + 1
    assert m.shape == (dims[2], dims[1], dims[0])
    occ = np.zeros((dims[2], dims[1], dims[0]), bool)
    want = np.zeros(occ.shape, np.int64)
    for i, b in enumerate(blocks):
        z, y, x = b[2] - lo[2], b[1] - lo[1], b[0] - lo[0]
        occ[z, y, x] = True
        want[z, y, x] = i * 256 + sum(1 << s for s in range(8) if nbr[i, s] >= 0)
    d = ndimage.distance_transform_cdt(~occ, metric="chessboard")
    want[~occ] = -np.minimum(d[~occ], 32)
    np.testing.assert_array_equal(m, want)
    g.destroy()


def test_hash_only_grid_has_no_map():
    from synth import workloads
    import paper_2305_13220_amd as sg
    w = workloads.sphere_tiny()
    g = sg.Grid(to_dev(w["block_coords"], torch.int32), float(w["h"]), dense_map_max_cells=0)
    m, _ = g.dense_map()
    assert m is None
    g.destroy()


def test_extend_keeps_indices_and_appends_new_blocks():
    """Extending a grid equals building it from the concatenated input: the
    old blocks keep their indices, new ones follow in first-occurrence
    order; neighbours, the dense map and lookups follow."""
    rng = np.random.default_rng(31)
    a = rng.integers(-6, 6, size=(3000, 3)).astype(np.int32)
    b = rng.integers(-9, 9, size=(4000, 3)).astype(np.int32)
    g = _build(a)
    n_old = g.n_blocks
    old = g.block_coords().cpu().numpy()
    n = g.extend(to_dev(b))
    blocks_or, _ = oracle.build_grid(np.concatenate([a, b]))
    assert n == blocks_or.shape[0] > n_old
    got = g.block_coords().cpu().numpy()
    np.testing.assert_array_equal(got, blocks_or)
    np.testing.assert_array_equal(got[:n_old], old)
    np.testing.assert_array_equal(g.neighbors().cpu().numpy(), oracle.neighbors(blocks_or))
    q = rng.integers(-11, 11, size=(5000, 3)).astype(np.int32)
    np.testing.assert_array_equal(g.lookup(to_dev(q)).cpu().numpy(), oracle.lookup(blocks_or, q))
    assert g.dense_map()[0] is not None
    assert g.extend(to_dev(np.zeros((0, 3), np.int32))) == n
    g.destroy()
