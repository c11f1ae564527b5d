"""Block allocation from depth (Sec. 3.4.1) and fusion (Sec. 3.4.2) on the
GPU against the oracle, on depth and colour frames of the analytic room.

Bars: allocated block coordinates bit-exact, in the same order; association
counts bit-exact (the decisions are float32 on both sides); fused SDF within
1e-5 of trunc and features within 1e-5 (float32 averages of at most F
values against float64); voxels without association exactly (trunc, 0)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


def _sg():
    import paper_2305_13220_amd as sg
    return sg


def _frames(F, W, H, n_sem=0):
    from synth import workloads
    fr = workloads.room_depth_frames(n_frames=F, W=W, H=H, n_sem=n_sem)
    depth = fr["depth"].copy()
    rng = np.random.default_rng(3)
    # invalid depths: NaN, zero, negative, beyond depth_max
    idx = rng.choice(depth.size, 64, replace=False)
    depth.reshape(-1)[idx[:16]] = np.nan
    depth.reshape(-1)[idx[16:32]] = 0.0
    depth.reshape(-1)[idx[32:48]] = -1.0
    depth.reshape(-1)[idx[48:]] = 50.0
    return fr, depth


@pytest.mark.parametrize("dilate", [0, 1, 2])
def test_alloc_blocks_matches_oracle(dilate):
    sg = _sg()
    fr, depth = _frames(3, 160, 120)
    got = sg.alloc_blocks(to_dev(fr["cams"]), to_dev(depth), float(fr["h"]), (0.0, 0.0, 0.0),
                          dilate=dilate, depth_max=20.0).cpu().numpy()
    want = oracle.alloc_blocks(fr["cams"], depth, fr["h"], fr["origin"], dilate=dilate,
                               depth_max=20.0)
    assert want.shape[0] > 100
    np.testing.assert_array_equal(got, want)


def _check_fuse(g_vox, g_wt, o_vox, o_wt, trunc, what):
    np.testing.assert_array_equal(g_wt, o_wt, err_msg=f"{what}: association counts")
    assert (o_wt > 0).mean() > 0.05, f"{what}: too few associated voxels"
    none = o_wt == 0
    assert (g_vox[none][:, 0] == np.float32(trunc)).all() and not g_vox[none][:, 1:].any()
    err_sdf = np.abs(g_vox[..., 0] - o_vox[..., 0])
    assert err_sdf.max() <= 1e-5 * trunc, f"{what}: sdf error {err_sdf.max()}"
    err_f = np.abs(g_vox[..., 1:] - o_vox[..., 1:])
    assert err_f.max() <= 1e-5, f"{what}: feature error {err_f.max()}"


@pytest.mark.parametrize("n_sem,dilate,mu_blocks", [(0, 1, None), (16, 1, None), (16, 2, 2)])
def test_fuse_matches_oracle(n_sem, dilate, mu_blocks):
    """trunc 6 cm, or the supplement's mu = L R (L = 8 h) at R = 2."""
    sg = _sg()
    fr, depth = _frames(3, 160, 120, n_sem=n_sem)
    blocks = oracle.alloc_blocks(fr["cams"], depth, fr["h"], fr["origin"], dilate=dilate,
                                 depth_max=20.0)
    g = sg.Grid(to_dev(blocks), float(fr["h"]), (0.0, 0.0, 0.0))
    trunc = 0.06 if mu_blocks is None else 8 * float(fr["h"]) * mu_blocks
    vox, wt = sg.fuse(g, to_dev(fr["cams"]), to_dev(depth), to_dev(fr["feat"]), trunc, n_sem=n_sem)
    o_vox, o_wt = oracle.fuse(blocks, fr["h"], fr["origin"], fr["cams"], depth, fr["feat"], trunc,
                              n_sem=n_sem)
    _check_fuse(vox.cpu().numpy(), wt.cpu().numpy(), o_vox, o_wt, trunc, f"n_sem={n_sem}")
    if n_sem:
        s = vox.cpu().numpy()[..., 4:]
        nrm = np.linalg.norm(s, axis=-1)
        assert np.allclose(nrm[o_wt > 0], 1.0, atol=1e-5)


def test_alloc_and_fuse_full_frames():
    """Ten 640x480 frames: the allocation compared in full, the fusion on 400
    seeded blocks of the allocated grid (and every association count)."""
    sg = _sg()
    from synth import workloads
    fr = workloads.room_depth_frames(n_frames=10, W=640, H=480)
    cams, depth = to_dev(fr["cams"]), to_dev(fr["depth"])
    got = sg.alloc_blocks(cams, depth, float(fr["h"]), (0.0, 0.0, 0.0), dilate=1)
    want = oracle.alloc_blocks(fr["cams"], fr["depth"], fr["h"], fr["origin"], dilate=1)
    np.testing.assert_array_equal(got.cpu().numpy(), want)
    g = sg.Grid(got, float(fr["h"]), (0.0, 0.0, 0.0))
    trunc = 0.06
    vox, wt = sg.fuse(g, cams, depth, to_dev(fr["feat"]), trunc)
    pick = np.sort(np.random.default_rng(5).choice(want.shape[0], 400, replace=False))
    o_vox, o_wt = oracle.fuse(want[pick], fr["h"], fr["origin"], fr["cams"], fr["depth"], fr["feat"],
                              trunc)
    _check_fuse(vox.cpu().numpy()[pick], wt.cpu().numpy()[pick], o_vox, o_wt, trunc, "640x480 x 10")


def test_fuse_invalid_arguments():
    sg = _sg()
    fr, depth = _frames(1, 32, 24)
    blocks = oracle.alloc_blocks(fr["cams"], depth, fr["h"], fr["origin"], dilate=0, depth_max=20.0)
    g = sg.Grid(to_dev(blocks), float(fr["h"]), (0.0, 0.0, 0.0))
    cams, dep, feat = to_dev(fr["cams"]), to_dev(depth), to_dev(fr["feat"])
    with pytest.raises(sg.SgridError):
        sg.fuse(g, cams, dep, feat, 0.0)
    with pytest.raises(sg.SgridError):
        sg.fuse(g, cams, dep, feat, 0.05, n_sem=4)
    with pytest.raises(sg.SgridError):
        sg.alloc_blocks(cams, dep, 0.02, dilate=9)
    empty = sg.alloc_blocks(cams, torch.full_like(dep, float("nan")), 0.02)
    assert empty.shape == (0, 3)


@pytest.mark.parametrize("radius,sigma,C", [(1, 1.0, 3), (2, 0.8, 0), (1, 1.5, 19), (2, 1.0, 19), (1, 1.0, 32), (0, 1.0, 19)])
def test_denoise_matches_oracle(radius, sigma, C):
    """Gaussian de-noising (Sec. 3.4.3) within 1e-5 of sum w|theta| / sum w."""
    sg = _sg()
    from synth import workloads, scenes
    from gpu_helpers import assert_close_mag, make_grid
    if C == 3:
        w = workloads.room_2cm()
        vox = scenes.perturb(w["vox"], w["h"], seed=2)
    else:
        w = workloads.sphere_tiny()
        rng = np.random.default_rng(8)
        vox = np.concatenate([w["vox"][..., :1], rng.normal(size=w["vox"].shape[:2] + (C,))],
                             -1).astype(np.float32)
    g = make_grid(w)
    out = sg.denoise(g, to_dev(vox), radius=radius, sigma=sigma).cpu().numpy()
    want, mag = oracle.denoise(w["block_coords"], vox, C, radius=radius, sigma=sigma, with_mag=True)
    assert_close_mag(out, want, mag, 1e-5, f"denoise r={radius} C={C}")


def test_denoise_invalid_arguments():
    sg = _sg()
    from synth import workloads
    from gpu_helpers import make_grid
    w = workloads.sphere_tiny()
    g = make_grid(w)
    vox = to_dev(w["vox"])
    for kw in ({"radius": 9}, {"sigma": 0.0}, {"out": vox}):
        with pytest.raises(sg.SgridError):
            sg.denoise(g, vox, **kw)


def test_denoise_wide_radius_direct_path():
    """radius 3 takes the kernel without the LDS tile (the tiled one covers
    radius <= 2): both against the oracle on the perturbed sphere."""
    sg = _sg()
    from synth import workloads, scenes
    from gpu_helpers import assert_close_mag, make_grid
    w = workloads.sphere_tiny()
    vox = scenes.perturb(w["vox"], w["h"], seed=6)
    g = make_grid(w)
    for radius, sigma in ((3, 1.2), (2, 1.0), (0, 1.0)):
        out = sg.denoise(g, to_dev(vox), radius=radius, sigma=sigma).cpu().numpy()
        want, mag = oracle.denoise(w["block_coords"], vox, 3, radius=radius, sigma=sigma,
                                   with_mag=True)
        assert_close_mag(out, want, mag, 1e-5, f"denoise r={radius}")


def test_grid_from_depth_is_alloc_then_build():
    """One call: the grid's block coordinates are the allocation's, in the
    same order (so the block indices are those sg_grid_build gives)."""
    sg = _sg()
    fr, depth = _frames(3, 160, 120)
    cams, dep = to_dev(fr["cams"]), to_dev(depth)
    g = sg.Grid.from_depth(cams, dep, float(fr["h"]), dilate=1, depth_max=20.0)
    want = oracle.alloc_blocks(fr["cams"], depth, fr["h"], fr["origin"], dilate=1, depth_max=20.0)
    np.testing.assert_array_equal(g.block_coords().cpu().numpy(), want)
    assert g.dense_map()[0] is not None
    with pytest.raises(sg.SgridError, match="valid depth"):
        sg.Grid.from_depth(cams, torch.full_like(dep, float("nan")), float(fr["h"]))
