"""Pins of the oracle's Gaussian de-noising (Sec. 3.4.3): against
scipy.ndimage's convolution of the masked dense grid (normalised by the
convolved mask), a closed-form impulse response, and invariance of
constant and (in the interior) linear fields."""
import numpy as np
import pytest
from scipy import ndimage

from synth.scenes import voxel_positions


def _kernel(radius, sigma):
    d = np.arange(-radius, radius + 1)
    g = np.exp(-(d[:, None, None] ** 2 + d[None, :, None] ** 2 + d[None, None, :] ** 2)
               / (2 * sigma ** 2))
    return g


def _dense(blocks, vox):
    """Dense [Z,Y,X,V] array over the blocks' box (+1 block margin) and mask."""
    lo = blocks.min(0) - 1
    dims = (blocks.max(0) - lo + 2) * 8
    V = vox.shape[-1]
    a = np.zeros((dims[2], dims[1], dims[0], V))
    m = np.zeros((dims[2], dims[1], dims[0]))
    l = np.arange(512)
    lx, ly, lz = l % 8, (l // 8) % 8, l // 64
    for b, c in enumerate(blocks):
        o = (c - lo) * 8
        a[o[2] + lz, o[1] + ly, o[0] + lx] = vox[b]
        m[o[2] + lz, o[1] + ly, o[0] + lx] = 1.0
    return a, m, lo


@pytest.mark.parametrize("radius,sigma", [(1, 1.0), (2, 0.8)])
def test_denoise_matches_masked_convolution(oracle_lib, radius, sigma):
    rng = np.random.default_rng(41)
    # a sparse, irregular set of blocks with holes
    cand = np.stack(np.meshgrid(np.arange(-2, 2), np.arange(-1, 2), np.arange(0, 3), indexing="ij"),
                    -1).reshape(-1, 3)
    blocks = cand[rng.random(len(cand)) < 0.6].astype(np.int32)
    vox = rng.normal(size=(len(blocks), 512, 3))
    out = oracle_lib.denoise(blocks, vox, 2, radius=radius, sigma=sigma)
    a, m, lo = _dense(blocks, vox)
    k = _kernel(radius, sigma)
    num = np.stack([ndimage.convolve(a[..., c] * m, k, mode="constant") for c in range(3)], -1)
    den = ndimage.convolve(m, k, mode="constant")
    l = np.arange(512)
    lx, ly, lz = l % 8, (l // 8) % 8, l // 64
    for b, c in enumerate(blocks):
        o = (c - lo) * 8
        want = num[o[2] + lz, o[1] + ly, o[0] + lx] / den[o[2] + lz, o[1] + ly, o[0] + lx][:, None]
        np.testing.assert_allclose(out[b], want, rtol=1e-12, atol=1e-12)


def test_denoise_impulse_constant_and_linear(oracle_lib):
    blocks = np.stack(np.meshgrid(np.arange(-1, 2), np.arange(-1, 2), np.arange(-1, 2),
                                  indexing="ij"), -1).reshape(-1, 3).astype(np.int32)
    centre = int(np.flatnonzero((blocks == 0).all(1))[0])
    pos = voxel_positions(blocks, 1.0, np.zeros(3))
    # constant -> unchanged everywhere (renormalised at the border of the grid)
    vox = np.full((len(blocks), 512, 1), 2.5)
    np.testing.assert_allclose(oracle_lib.denoise(blocks, vox, 0), vox, rtol=1e-14)
    # linear -> unchanged where the whole neighbourhood is allocated (symmetric kernel)
    lin = (0.3 * pos[..., 0] - 1.1 * pos[..., 1] + 0.7 * pos[..., 2] + 4.0)[..., None]
    out = oracle_lib.denoise(blocks, lin, 0, radius=1, sigma=1.3)
    np.testing.assert_allclose(out[centre], lin[centre], rtol=1e-12, atol=1e-12)
    # impulse at voxel (3,3,3) of the centre block -> the normalised kernel
    imp = np.zeros((len(blocks), 512, 1))
    imp[centre, 3 + 8 * 3 + 64 * 3, 0] = 1.0
    out = oracle_lib.denoise(blocks, imp, 0, radius=1, sigma=0.9)
    k = _kernel(1, 0.9)
    k /= k.sum()
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                v = (3 + dx) + 8 * (3 + dy) + 64 * (3 + dz)
                assert out[centre, v, 0] == pytest.approx(k[dz + 1, dy + 1, dx + 1], rel=1e-12)
    assert out[centre, 0, 0] == 0.0
