"""Pins of the oracle's Eikonal regulariser (Eq. 16 with the gradient of
Eq. 18) and of its derivative with respect to the SDF voxels.

* Multilinear SDF fields are reproduced exactly by trilinear interpolation,
  so the loss at a point is weight * (|grad P(p)| - 1)^2 in closed form
  (checked with the polynomial's own gradient, written here).  A linear field
  of unit slope gives zero loss and zero gradient.
* The voxel gradient equals central differences of the summed loss in
  float64 (a dropped factor, a wrong sign or a transposed axis fails this).
* Invalid points contribute nothing; feature channels get no gradient.
"""
import numpy as np
import pytest

from synth.scenes import voxel_positions
from test_oracle_interp import _dense_blocks, _multilinear


def _setup(seed, C=0, field=None):
    rng = np.random.default_rng(seed)
    h = 1.0 / 16
    origin = np.zeros(3, np.float32)
    blocks = _dense_blocks((-2, -2, -2), (1, 1, 1))
    val, grad = field or _multilinear(rng)
    pos = voxel_positions(blocks, h, origin)
    vox = np.empty((blocks.shape[0], 512, 1 + C))
    vox[..., 0] = val(pos)
    vox[..., 1:] = rng.normal(size=vox.shape[:2] + (C,))
    pv = rng.integers(-15 * 64, 14 * 64, size=(500, 3)) / 64.0  # voxel units, exact in float32
    p = (pv * h).astype(np.float32)
    return rng, h, origin, blocks, vox, p, pv * h, grad


@pytest.mark.parametrize("weight", [1.0, 0.37])
def test_eikonal_loss_closed_form_multilinear(oracle_lib, weight):
    _, h, origin, blocks, vox, p, pw, grad = _setup(31, C=2)
    loss, gv = oracle_lib.eikonal(blocks, vox, 2, np.float32(h), origin, p, weight)
    want = weight * (np.linalg.norm(grad(pw), axis=-1) - 1.0) ** 2
    np.testing.assert_allclose(loss, want, rtol=1e-10, atol=1e-12)
    assert not gv[..., 1:].any(), "feature channels must get no gradient"
    assert np.abs(gv[..., 0]).sum() > 0


def test_unit_slope_linear_field_has_zero_loss_and_gradient(oracle_lib):
    a = np.array([0.36, -0.48, 0.8])  # |a| = 1
    field = (lambda q: q @ a + 0.25, lambda q: np.broadcast_to(a, q.shape))
    _, h, origin, blocks, vox, p, _, _ = _setup(32, field=field)
    loss, gv = oracle_lib.eikonal(blocks, vox, 0, np.float32(h), origin, p, 2.0)
    assert np.abs(loss).max() < 1e-24
    assert np.abs(gv).max() < 1e-10


def test_eikonal_gradient_matches_central_differences(oracle_lib):
    rng, h, origin, blocks, vox, p, _, _ = _setup(33, C=1)
    vox[..., 0] += 0.3 * rng.normal(size=vox.shape[:2]) * h  # not multilinear any more
    weight = 0.8
    _, gv = oracle_lib.eikonal(blocks, vox, 1, np.float32(h), origin, p, weight)
    touched = np.flatnonzero(np.abs(gv[..., 0]).ravel() > 0)
    assert touched.size > 100
    pick = rng.choice(touched, 40, replace=False)
    eps = 1e-6
    for flat in pick:
        b, v = divmod(int(flat), 512)
        hi, lo = vox.copy(), vox.copy()
        hi[b, v, 0] += eps
        lo[b, v, 0] -= eps
        lp = oracle_lib.eikonal(blocks, hi, 1, np.float32(h), origin, p, weight)[0].sum()
        lm = oracle_lib.eikonal(blocks, lo, 1, np.float32(h), origin, p, weight)[0].sum()
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - gv[b, v, 0]) <= 1e-6 * max(1.0, abs(fd)), (b, v, fd, gv[b, v, 0])


def test_invalid_points_contribute_nothing(oracle_lib):
    _, h, origin, blocks, vox, p, _, _ = _setup(34)
    bad = np.array([[np.nan, 0, 0], [5.0, 5.0, 5.0], [0, np.inf, 0]], np.float32)
    loss, gv = oracle_lib.eikonal(blocks, vox, 0, np.float32(h), origin, bad, 1.0)
    assert not loss.any() and not gv.any()
    # appending invalid points changes nothing
    l1, g1 = oracle_lib.eikonal(blocks, vox, 0, np.float32(h), origin, p, 1.0)
    l2, g2 = oracle_lib.eikonal(blocks, vox, 0, np.float32(h), origin, np.concatenate([p, bad]), 1.0)
    np.testing.assert_array_equal(l2[: len(p)], l1)
    np.testing.assert_array_equal(g2, g1)


def _axis_rays(rng, h, n=40):
    """Rays along +z (and -x) whose origins and samples are dyadic, so every
    float32 sample position equals o + t d exactly."""
    o = rng.integers(-14 * 16, 13 * 16, size=(n, 2)) / 16.0 * h
    rz = np.zeros((n, 6), np.float32)
    rz[:, 0], rz[:, 1], rz[:, 2], rz[:, 5] = o[:, 0], o[:, 1], -1.0, 1.0
    rx = np.zeros((n, 6), np.float32)
    rx[:, 1], rx[:, 2], rx[:, 0], rx[:, 3] = o[:, 0], o[:, 1], 1.0, -1.0
    return np.concatenate([rz, rx])


def test_ray_samples_eikonal_is_point_eikonal_at_the_samples(oracle_lib):
    rng, h, origin, blocks, vox, _, _, _ = _setup(35, C=1)
    vox[..., 0] += 0.3 * rng.normal(size=vox.shape[:2]) * h
    rays = _axis_rays(rng, h)
    params = {"step": h / 2, "t_near": 0.0, "t_far": 2.0, "beta": h, "max_samples": 200}
    loss_r, gv_r = oracle_lib.eikonal_rays(blocks, vox, 1, np.float32(h), origin, rays, params, 0.6)
    total = np.zeros_like(vox)
    n_s = 0
    for r, ray in enumerate(rays):
        s = oracle_lib.ray_samples(blocks, np.float32(h), origin, ray, params)
        pts = (ray[:3].astype(np.float64) + s["t"][:, None].astype(np.float64) * ray[3:]).astype(np.float32)
        assert np.array_equal(pts.astype(np.float64),
                              ray[:3].astype(np.float64) + s["t"][:, None] * ray[3:].astype(np.float64))
        l, g = oracle_lib.eikonal(blocks, vox, 1, np.float32(h), origin, pts, 0.6)
        np.testing.assert_allclose(loss_r[r], l.sum(), rtol=1e-12, atol=1e-15)
        total += g
        n_s += len(pts)
    assert n_s > 1000
    np.testing.assert_allclose(gv_r, total, rtol=1e-10, atol=1e-12)


def test_ray_samples_eikonal_gradient_matches_central_differences(oracle_lib):
    rng, h, origin, blocks, vox, _, _, _ = _setup(36)
    vox[..., 0] += 0.3 * rng.normal(size=vox.shape[:2]) * h
    rays = _axis_rays(rng, h, n=8)
    params = {"step": h / 2, "t_near": 0.0, "t_far": 2.0, "beta": h, "max_samples": 200}
    _, gv = oracle_lib.eikonal_rays(blocks, vox, 0, np.float32(h), origin, rays, params, 1.3)
    touched = np.flatnonzero(np.abs(gv[..., 0]).ravel() > 0)
    pick = rng.choice(touched, 30, replace=False)
    eps = 1e-6
    for flat in pick:
        b, v = divmod(int(flat), 512)
        hi, lo = vox.copy(), vox.copy()
        hi[b, v, 0] += eps
        lo[b, v, 0] -= eps
        lp = oracle_lib.eikonal_rays(blocks, hi, 0, np.float32(h), origin, rays, params, 1.3)[0].sum()
        lm = oracle_lib.eikonal_rays(blocks, lo, 0, np.float32(h), origin, rays, params, 1.3)[0].sum()
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - gv[b, v, 0]) <= 1e-6 * max(1.0, abs(fd)), (b, v, fd, gv[b, v, 0])


def test_splitmix64_reference_outputs(oracle_lib):
    """The generator's first two outputs from state 0 (the published sequence)."""
    assert oracle_lib.splitmix64(0) == 0xE220A8397B1DCDAF
    assert oracle_lib.splitmix64(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4


def test_uniform_points_cover_the_blocks(oracle_lib):
    rng = np.random.default_rng(0)
    blocks = np.unique(rng.integers(-5, 5, size=(40, 3)), axis=0).astype(np.int32)
    h = np.float32(0.02)
    origin = np.array([0.5, -0.25, 1.0], np.float32)
    n = 200000
    p = oracle_lib.uniform_points(blocks, h, origin, n, seed=12345)
    # every point lies in one of the blocks (cell coordinates in [8b, 8b+8))
    v = (p.astype(np.float64) - origin) / float(h)
    b = np.floor(v / 8.0).astype(np.int64)
    keys = {tuple(x) for x in blocks}
    inside = np.array([tuple(x) in keys for x in b[:5000]])
    assert inside.mean() > 0.999
    # blocks and positions inside them are uniform (5-sigma bounds)
    idx = {tuple(x): i for i, x in enumerate(blocks)}
    counts = np.bincount([idx.get(tuple(x), 0) for x in b], minlength=len(blocks))
    exp = n / len(blocks)
    assert np.abs(counts - exp).max() < 5 * np.sqrt(exp)
    frac = v / 8.0 - b
    for a in range(3):
        hist = np.histogram(frac[:, a], bins=10, range=(0, 1))[0]
        assert np.abs(hist - n / 10).max() < 5 * np.sqrt(n / 10)
    # reproducible, and the seed matters
    np.testing.assert_array_equal(p[:100], oracle_lib.uniform_points(blocks, h, origin, 100, 12345))
    assert not np.array_equal(p[:100], oracle_lib.uniform_points(blocks, h, origin, 100, 12346))
