"""Point query (Eq. 17-18 at arbitrary points) against the oracle.

Validity flags bit-exact; f and features within 1e-5 of sum_a r_a |theta_a|
(the oracle's query of |vox|, since r_a >= 0); the gradient within 1e-5 of
2 max|theta_sdf| / h (each edge difference is bounded by twice the largest
corner value) plus 1e-5 relative."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import make_grid, to_dev

pytestmark = pytest.mark.gpu


def _sg():
    import paper_2305_13220_amd as sg
    return sg


def _points(w, n, seed, lo, hi):
    rng = np.random.default_rng(seed)
    h = float(w["h"])
    pts = rng.uniform(lo, hi, size=(n, 3)).astype(np.float32)
    # points on voxel and block faces, and exactly on voxel centres
    grid_pts = (np.round(rng.uniform(lo, hi, size=(n // 4, 3)) / h) * h).astype(np.float32)
    block_pts = (np.round(rng.uniform(lo, hi, size=(n // 8, 3)) / (8 * h)) * 8 * h).astype(np.float32)
    odd = np.array([[np.nan, 0, 0], [0, np.inf, 0], [1e30, 0, 0], [-1e30, 5, 5]], np.float32)
    return np.concatenate([pts, grid_pts, block_pts, odd])


def _check(w, vox_np, C, pts, g=None, what="query"):
    g = g or make_grid(w)
    out = _sg().query(g, to_dev(vox_np), to_dev(pts))
    valid, f, grad, feat = oracle.query(w["block_coords"], vox_np, C, w["h"], w["origin"], pts)
    _, fm, _, featm = oracle.query(w["block_coords"], np.abs(vox_np.astype(np.float64)), C, w["h"],
                                   w["origin"], pts)
    np.testing.assert_array_equal(out["valid"].cpu().numpy().astype(bool), valid, err_msg=what)
    assert valid.sum() > len(pts) // 10, f"{what}: too few valid points to test"
    gf = out["f"].cpu().numpy()
    assert np.all(np.abs(gf - f) <= 1e-5 * fm + 1e-30), what
    gg = out["grad"].cpu().numpy()
    gscale = 2.0 * np.abs(vox_np[..., 0]).max() / float(w["h"])
    assert np.all(np.abs(gg - grad) <= 1e-5 * gscale + 1e-5 * np.abs(grad)), what
    if C:
        gc = out["feat"].cpu().numpy()
        assert np.all(np.abs(gc - feat) <= 1e-5 * featm + 1e-30), what
    for k in ("f", "grad", "feat"):
        assert not out[k].cpu().numpy()[~valid].any(), f"{what}: {k} of an invalid point"


def test_query_sphere():
    from synth import workloads
    w = workloads.sphere_tiny()
    _check(w, w["vox"], 3, _points(w, 40000, 1, -0.7, 0.7), what="sphere")


@pytest.mark.parametrize("C", [0, 19])
def test_query_feature_counts(C):
    from synth import scenes
    w = scenes.sphere_scene(h=1.0 / 32, radius=0.4, band_vox=3, seed=5, C=max(C, 1))
    vox = w["vox"][..., : 1 + C].copy()
    if C == 19:
        rng = np.random.default_rng(9)
        vox = np.concatenate([w["vox"][..., :2], rng.normal(size=w["vox"].shape[:2] + (18,))],
                             -1).astype(np.float32)
    _check(w, vox, C, _points(w, 20000, 2, -0.6, 0.6), what=f"C={C}")


@pytest.mark.parametrize("dense_map", [True, False])
def test_query_room(dense_map):
    from synth import workloads
    import paper_2305_13220_amd as sg
    w = workloads.room_2cm()
    g = sg.Grid(to_dev(w["block_coords"], torch.int32), float(w["h"]),
                tuple(float(x) for x in w["origin"]), dense_map_max_cells=-1 if dense_map else 0)
    pts = _points(w, 100000, 3, -0.2, 6.2)
    _check(w, w["vox"], 3, pts, g=g, what=f"room, dense map {dense_map}")


def test_query_at_sample_positions_matches_render_inputs():
    """A query at a lattice sample's float32 position is that sample: the
    oracle's sample list gives the points, all must be valid."""
    from synth import workloads
    w = workloads.sphere_tiny()
    ray = w["rays"][(w["H"] // 2) * w["W"] + w["W"] // 2]  # centre pixel, looks at the sphere
    s = oracle.ray_samples(w["block_coords"], w["h"], w["origin"], ray, w["params"])
    assert len(s["t"]) > 0
    pts = (ray[:3][None, :].astype(np.float32) + s["t"][:, None].astype(np.float32)
           * ray[3:][None, :].astype(np.float32)).astype(np.float32)
    out = _sg().query(make_grid(w), to_dev(w["vox"]), to_dev(pts))
    # positions rebuilt in world units may round across a face; most stay valid
    assert out["valid"].float().mean().item() > 0.9


def test_query_lattice_room_full_and_options():
    """The k^3 lattice of the timed query (k = 80 here), built on the device
    the same way, compared in full; the geometry-only call and buffer reuse
    give the same bits; zero points is a no-op."""
    from synth import workloads
    import paper_2305_13220_amd as sg
    w = workloads.room_2cm()
    g = make_grid(w)
    vox = to_dev(w["vox"])
    h = float(w["h"])
    bmin, bmax = w["block_coords"].min(0), w["block_coords"].max(0)
    k = 80
    ax = [torch.linspace(float(w["origin"][a]) + 8 * h * float(bmin[a]),
                         float(w["origin"][a]) + 8 * h * float(bmax[a] + 1), k, device="cuda")
          for a in range(3)]
    zz, yy, xx = torch.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    pts = torch.stack([xx.reshape(-1), yy.reshape(-1), zz.reshape(-1)], 1).contiguous()
    pts_np = pts.cpu().numpy()
    _check(w, w["vox"], 3, pts_np, g=g, what="lattice k=80")
    full = sg.query(g, vox, pts)
    geo = sg.query(g, vox, pts, features=False)
    assert "feat" not in geo
    again = sg.query(g, vox, pts, features=False, out=geo)
    for key in ("valid", "f", "grad"):
        assert torch.equal(full[key], geo[key]) and again[key] is geo[key]
    empty = sg.query(g, vox, torch.empty((0, 3), dtype=torch.float32, device="cuda"))
    assert empty["f"].numel() == 0
    with pytest.raises(ValueError):
        sg.query(g, vox, pts[:10], out={"f": torch.empty(11, device="cuda")})
