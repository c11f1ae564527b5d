"""Pins of the oracle's block allocation from depth (Sec. 3.4.1) and of the
depth / colour / semantic fusion (Sec. 3.4.2).

Closed forms on planes seen by cameras whose rotation is a cyclic axis
permutation (exact in float32, and not symmetric, so using R for R^T fails):
* a constant depth map lifts every pixel onto one plane, so the allocated
  blocks are a box of blocks (grown by the dilation radius), the first one
  the dilation of the first pixel's block;
* fusing that depth map gives SDF = min(D - z, trunc) (z the depth of the
  voxel along the optical axis) wherever D - z >= -trunc (the truncation of
  the supplement's Volumetric Fusion: clipped in front of the surface,
  rejected behind it), the constant colour, the normalised semantic vector,
  and the truncation value with weight 0 elsewhere; two frames average.
"""
import numpy as np
import pytest

H_VOX = 1.0 / 16  # power-of-two voxel size: voxel positions are exact
# camera axes in world coordinates: x_cam = +y, y_cam = +z, z_cam = +x
R_PERM = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]], np.float64)


def _cam(R, t, fx, fy, cx, cy):
    c = np.zeros(16, np.float32)
    c[:4] = fx, fy, cx, cy
    M = np.concatenate([R, np.asarray(t, np.float64)[:, None]], 1)
    c[4:] = M.reshape(-1)
    return c


def test_alloc_constant_depth_is_a_box_of_blocks(oracle_lib):
    W, H, D = 32, 24, 2.0
    fx = fy = 16.0
    t = np.array([0.25, -0.5, 0.125])
    cam = _cam(R_PERM, t, fx, fy, W / 2, H / 2)
    depth = np.full((1, H, W), D, np.float32)
    for r in (0, 1, 2):
        got = oracle_lib.alloc_blocks(cam[None], depth, np.float32(H_VOX), np.zeros(3, np.float32),
                                      dilate=r)
        # camera point (x D, y D, D) -> world (D + tx, x D + ty, y D + tz)
        xs = (np.arange(W) + 0.5 - W / 2) / fx * D
        ys = (np.arange(H) + 0.5 - H / 2) / fy * D
        bs = 8 * H_VOX
        bx = np.floor((D + t[0]) / bs)
        by = np.unique(np.floor((xs + t[1]) / bs))
        bz = np.unique(np.floor((ys + t[2]) / bs))
        want = {(int(bx) + dx, int(y) + dy, int(z) + dz) for y in by for z in bz
                for dx in range(-r, r + 1) for dy in range(-r, r + 1) for dz in range(-r, r + 1)}
        assert {tuple(c) for c in got} == want
        assert len(got) == len(want), "duplicates in the output"
        # first occurrence: pixel (0,0), dilation offset (-r,-r,-r) first
        first = (int(bx) - r, int(np.floor((xs[0] + t[1]) / bs)) - r,
                 int(np.floor((ys[0] + t[2]) / bs)) - r)
        assert tuple(got[0]) == first


def test_alloc_skips_invalid_depths_and_single_pixel_dilation(oracle_lib):
    W, H = 4, 3
    cam = _cam(np.eye(3), [0, 0, 0], 4.0, 4.0, 2.5, 1.5)
    depth = np.full((2, H, W), np.nan, np.float32)
    depth[0, 0, 0] = -1.0
    depth[0, 1, 1] = 0.0
    depth[0, 2, 3] = 100.0  # beyond depth_max
    depth[1, 1, 2] = 1.0    # the only valid pixel: its centre ray is the optical axis
    got = oracle_lib.alloc_blocks(np.stack([cam, cam]), depth, np.float32(H_VOX),
                                  np.zeros(3, np.float32), dilate=1, depth_max=10.0)
    b = (0, 0, 2)  # camera point (0, 0, 1); a pixel corner instead of its centre gives -1
    want = [(b[0] + dx, b[1] + dy, b[2] + dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1)
            for dx in (-1, 0, 1)]
    assert [tuple(c) for c in got] == want
    empty = oracle_lib.alloc_blocks(cam[None], np.full((1, H, W), np.nan, np.float32),
                                    np.float32(H_VOX), np.zeros(3, np.float32))
    assert empty.shape == (0, 3)


def _slab_setup(t, D):
    """Blocks around the plane seen at depth D by the permuted camera at t:
    the world plane x = t_x + D, blocks covering x in [x0 - 0.5, x0 + 0.5]."""
    x0 = t[0] + D
    bs = 8 * H_VOX
    bx = np.arange(np.floor((x0 - 0.5) / bs), np.floor((x0 + 0.5) / bs) + 1)
    by = np.arange(-2, 2)
    bz = np.arange(-2, 2)
    g = np.stack(np.meshgrid(bx, by, bz, indexing="ij"), -1).reshape(-1, 3).astype(np.int32)
    return g


def _voxel_world(blocks):
    from synth.scenes import voxel_positions
    return voxel_positions(blocks, H_VOX, np.zeros(3))


def test_fuse_plane_closed_form(oracle_lib):
    t = np.array([-1.0, 0.0, 0.0])
    D0, D1, trunc = 2.0, 2.25, 0.3
    W = H = 256
    f = 32.0  # every voxel of the slab projects well inside the image
    cam = _cam(R_PERM, t, f, f, W / 2, H / 2)
    blocks = _slab_setup(t, D0)
    col = np.array([0.2, 0.5, 0.9, 3.0, 4.0], np.float32)  # RGB + 2 semantic logits
    depth = np.stack([np.full((H, W), D0, np.float32), np.full((H, W), D1, np.float32)])
    feat = np.broadcast_to(col, (2, H, W, 5)).copy()
    feat[1, ..., :3] = [0.4, 0.1, 0.3]
    feat[1, ..., 3:] = [0.0, 1.0]
    vox, wt = oracle_lib.fuse(blocks, np.float32(H_VOX), np.zeros(3, np.float32),
                              np.stack([cam, cam]), depth, feat, trunc, n_sem=2)
    X = _voxel_world(blocks)
    z = X[..., 0] - t[0]  # depth along the optical axis (+x)
    mu = float(np.float32(trunc))
    a0 = D0 - z >= -mu
    a1 = D1 - z >= -mu
    n = a0.astype(int) + a1.astype(int)
    np.testing.assert_array_equal(wt, n)
    assert (n == 2).any() and (n == 1).any() and (n == 0).any()
    assert (D0 - z > mu).any(), "no voxel far enough in front to be clipped"
    s0, s1 = np.minimum(D0 - z, mu), np.minimum(D1 - z, mu)
    sdf = np.where(n > 0, (a0 * s0 + a1 * s1) / np.maximum(n, 1), mu)
    np.testing.assert_allclose(vox[..., 0], sdf, rtol=0, atol=1e-12)
    rgb = (a0[..., None] * col[:3] + a1[..., None] * feat[1, 0, 0, :3]) / np.maximum(n, 1)[..., None]
    np.testing.assert_allclose(vox[..., 1:4], rgb, atol=1e-7)
    sem = (a0[..., None] * col[3:] + a1[..., None] * feat[1, 0, 0, 3:])
    nrm = np.linalg.norm(sem, axis=-1, keepdims=True)
    sem = np.where(nrm > 0, sem / np.where(nrm > 0, nrm, 1), 0)
    np.testing.assert_allclose(vox[..., 4:], sem, atol=1e-7)
    assert np.allclose(np.linalg.norm(vox[n > 0][:, 4:], axis=-1), 1.0)


def test_fuse_behind_camera_and_outside_image(oracle_lib):
    """Voxels behind the camera or projecting outside the image get nothing."""
    t = np.array([-1.0, 0.0, 0.0])
    W = H = 8
    cam = _cam(R_PERM, t, 4.0, 4.0, W / 2, H / 2)  # narrow field of view
    blocks = np.array([[-3, 0, 0], [1, 0, 0], [1, 8, 0]], np.int32)  # behind, inside, off to the side
    depth = np.full((1, H, W), 2.0, np.float32)
    feat = np.ones((1, H, W, 1), np.float32)
    vox, wt = oracle_lib.fuse(blocks, np.float32(H_VOX), np.zeros(3, np.float32), cam[None], depth,
                              feat, 10.0)
    assert wt[0].sum() == 0 and wt[2].sum() == 0
    assert (vox[0, :, 0] == 10.0).all() and (vox[0, :, 1] == 0).all()
    assert wt[1].sum() > 0
