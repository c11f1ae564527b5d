"""Pins of the oracle's interpolation (Eq. 17-18), density (the Laplace-CDF
transform of Sec. 3.5.1) and sample selection.

* Trilinear interpolation reproduces every multilinear polynomial
  (span of 1, x, y, z, xy, yz, zx, xyz) exactly, and its closed-form gradient
  is the polynomial's gradient.  A dropped corner, a wrong sign in dr/du or a
  swapped axis fails this.
* sigma(f) = laplace.cdf(-f, scale=beta) / beta (scipy), and its derivative.
* The kept samples of a ray equal a brute-force float32 walk over the lattice
  written here with numpy and a Python set of blocks.
"""
import numpy as np
import pytest
from scipy import stats

from synth.scenes import voxel_positions


def _multilinear(rng):
    c = rng.normal(size=8)

    def val(p):
        x, y, z = p[..., 0], p[..., 1], p[..., 2]
        return (c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * y * z
                + c[6] * z * x + c[7] * x * y * z)

    def grad(p):
        x, y, z = p[..., 0], p[..., 1], p[..., 2]
        return np.stack([c[1] + c[4] * y + c[6] * z + c[7] * y * z,
                         c[2] + c[4] * x + c[5] * z + c[7] * x * z,
                         c[3] + c[5] * y + c[6] * x + c[7] * x * y], -1)

    return val, grad


def _dense_blocks(lo, hi):
    r = [np.arange(lo[a], hi[a] + 1) for a in range(3)]
    return np.stack(np.meshgrid(*r, indexing="ij"), -1).reshape(-1, 3).astype(np.int32)


@pytest.mark.parametrize("C", [0, 2])
def test_multilinear_exact_power_of_two_voxel(oracle_lib, C):
    """h = 1/16 and origin 0: query points with few mantissa bits map to
    voxel space without rounding, so f and grad f must be exact (1e-12)."""
    rng = np.random.default_rng(21)
    h = 1.0 / 16
    origin = np.zeros(3, np.float32)
    blocks = _dense_blocks((-2, -2, -2), (1, 1, 1))
    val, grad = _multilinear(rng)
    pos = voxel_positions(blocks, h, origin)
    vox = np.empty((blocks.shape[0], 512, 1 + C))
    vox[..., 0] = val(pos)
    for ch in range(C):
        vox[..., 1 + ch] = (ch + 2.0) * val(pos) - ch
    # points strictly inside [-15, 14] voxels so all 8 corners exist; includes
    # cells spanning block boundaries (coordinate 7 -> 8, -1 -> 0, ...)
    m = 4000
    pv = rng.integers(-15 * 64, 14 * 64, size=(m, 3)) / 64.0  # voxel units, exact
    pv[:50] = rng.integers(-1, 2, size=(50, 3)) * 8 - 0.5  # cells whose corners lie in 8 blocks
    p = (pv * h).astype(np.float32)
    assert np.array_equal(p.astype(np.float64) / h, pv)
    valid, f, g, feat = oracle_lib.query(blocks, vox, C, np.float32(h), origin, p)
    assert valid.all()
    pw = pv * h
    np.testing.assert_allclose(f, val(pw), rtol=0, atol=1e-12)
    np.testing.assert_allclose(g, grad(pw), rtol=1e-12, atol=1e-11)
    for ch in range(C):
        np.testing.assert_allclose(feat[:, ch], (ch + 2.0) * val(pw) - ch, atol=1e-11)


def test_multilinear_general_voxel_size(oracle_lib):
    """h = 2 cm, origin offset: exact up to the float32 rounding of the
    voxel-space position (relative 1e-6)."""
    rng = np.random.default_rng(22)
    h = np.float32(0.02)
    origin = np.array([0.3, -0.7, 0.11], np.float32)
    blocks = _dense_blocks((-2, -1, 0), (1, 1, 2))
    val, grad = _multilinear(rng)
    pos = voxel_positions(blocks, float(h), origin.astype(np.float64))
    vox = val(pos)[..., None]
    lo = origin + h * (8 * blocks.min(0) + 0.1)  # base voxel of every cell inside the box
    hi = origin + h * (8 * blocks.max(0) + 6.9)
    p = rng.uniform(lo, hi, size=(3000, 3)).astype(np.float32)
    valid, f, g, _ = oracle_lib.query(blocks, vox, 0, h, origin, p)
    assert valid.all()
    # the oracle evaluates at the float32 voxel-space position
    inv_h = np.float32(1.0) / h
    pv = ((p - origin) * inv_h).astype(np.float32).astype(np.float64)
    pw = origin.astype(np.float64) + pv * float(h)
    np.testing.assert_allclose(f, val(pw), rtol=0, atol=1e-9)
    np.testing.assert_allclose(g, grad(pw), rtol=1e-9, atol=1e-8)


def test_query_invalid_when_corner_block_missing(oracle_lib):
    h = np.float32(1.0 / 16)
    blocks = np.array([[0, 0, 0]], np.int32)
    vox = np.zeros((1, 512, 1))
    # cell base in [0,6]^3 is inside; base voxel 7 on any axis needs block 1
    p = np.array([[3.5, 3.5, 3.5], [7.5, 3.5, 3.5], [3.5, 7.5, 3.5], [3.5, 3.5, 7.5],
                  [-0.5, 3.5, 3.5], [6.99, 6.99, 6.99]], np.float32) * h
    valid, *_ = oracle_lib.query(blocks, vox, 0, h, np.zeros(3, np.float32), p)
    np.testing.assert_array_equal(valid, [True, False, False, False, False, True])


@pytest.mark.parametrize("beta", [0.02, 0.5, 3.0])
def test_density_is_laplace_cdf(oracle_lib, beta):
    f = np.concatenate([np.linspace(-20 * beta, 20 * beta, 2001), [0.0, -0.0]])
    sigma, dsigma = oracle_lib.density(f, beta)
    np.testing.assert_allclose(sigma, stats.laplace.cdf(-f, scale=beta) / beta,
                               rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(dsigma, -stats.laplace.pdf(-f, scale=beta) / beta, rtol=1e-13)
    assert sigma[-1] == sigma[-2] == pytest.approx(0.5 / beta)


def _brute_force_samples(blocks, h, origin, ray, prm):
    """Float32 lattice walk, one rounding per operation (numpy scalars)."""
    B = set(map(tuple, blocks.tolist()))
    f32 = np.float32
    inv_h = f32(1.0) / f32(h)
    ov = [(f32(ray[a]) - f32(origin[a])) * inv_h for a in range(3)]
    dv = [f32(ray[3 + a]) * inv_h for a in range(3)]
    step, t0, t1 = f32(prm["step"]), f32(prm["t_near"]), f32(prm["t_far"])
    ks, iis = [], []
    k = 0
    while len(ks) < prm["max_samples"]:
        t = t0 + f32(k) * step
        if not t <= t1:
            break
        xv = [ov[a] + t * dv[a] for a in range(3)]
        i = [int(np.floor(x)) for x in xv]
        ok = all((((i[0] + (c & 1)) // 8), ((i[1] + ((c >> 1) & 1)) // 8),
                  ((i[2] + ((c >> 2) & 1)) // 8)) in B for c in range(8))
        if ok:
            ks.append(k)
            iis.append(i)
        k += 1
    return np.array(ks, np.int64), np.array(iis, np.int64).reshape(-1, 3)


def test_ray_samples_match_brute_force(oracle_lib):
    from synth import workloads
    w = workloads.sphere_tiny()
    rng = np.random.default_rng(23)
    prm = dict(w["params"])
    for r in rng.choice(w["rays"].shape[0], 40, replace=False):
        s = oracle_lib.ray_samples(w["block_coords"], w["h"], w["origin"], w["rays"][r], prm)
        ks, iis = _brute_force_samples(w["block_coords"], w["h"], w["origin"], w["rays"][r], prm)
        np.testing.assert_array_equal(s["k"], ks)
        np.testing.assert_array_equal(s["i"], iis)


def test_ray_samples_cap_and_t_far_inclusive(oracle_lib):
    h = np.float32(1.0 / 16)
    blocks = _dense_blocks((0, 0, 0), (1, 0, 0))  # 16 x 8 x 8 voxels
    ray = np.array([0, 3.25 * h, 3.25 * h, 1, 0, 0], np.float32)  # along +x
    prm = {"step": float(h) / 2, "t_near": 0.0, "t_far": float(h) * 5, "beta": 0.1,
           "max_samples": 128}
    s = oracle_lib.ray_samples(blocks, h, np.zeros(3, np.float32), ray, prm)
    np.testing.assert_array_equal(s["k"], np.arange(11))  # t = 5h is kept
    prm["max_samples"] = 4
    s = oracle_lib.ray_samples(blocks, h, np.zeros(3, np.float32), ray, prm)
    np.testing.assert_array_equal(s["k"], np.arange(4))


def test_query_backward_is_the_adjoint_of_query(oracle_lib):
    """<g, J theta> = <J^T g, theta> for random upstream gradients, with the
    forward from or_query (f, grad f and features are linear in theta), and
    central differences of a loss on the query outputs."""
    rng = np.random.default_rng(51)
    h = np.float32(0.05)
    origin = np.array([0.1, -0.2, 0.05], np.float32)
    blocks = _dense_blocks((-1, -1, -1), (1, 0, 1))
    C = 2
    vox = rng.normal(size=(blocks.shape[0], 512, 1 + C))
    lo = origin + h * (8 * blocks.min(0) + 0.5)
    hi = origin + h * (8 * blocks.max(0) + 6.5)
    p = rng.uniform(lo, hi, size=(400, 3)).astype(np.float32)
    p[:5] = [1e3, 0, 0]  # invalid points contribute nothing
    gf, gg, gc = rng.normal(size=400), rng.normal(size=(400, 3)), rng.normal(size=(400, C))
    gv, _ = oracle_lib.query_backward(blocks, C, h, origin, p, gf, gg, gc)
    valid, f, g, feat = oracle_lib.query(blocks, vox, C, h, origin, p)
    lhs = (gf * f).sum() + (gg * g).sum() + (gc * feat).sum()
    assert float((gv * vox).sum()) == pytest.approx(float(lhs), rel=1e-10)
    assert valid[5:].all() and not valid[:5].any()
    # central differences on a few voxels
    loss = lambda vx: float(sum((w * o).sum() for w, o in zip(
        (gf, gg, gc), oracle_lib.query(blocks, vx, C, h, origin, p)[1:])))
    touched = np.argwhere(np.abs(gv) > 0)
    for b, v, c in touched[rng.choice(len(touched), 12, replace=False)]:
        hi_, lo_ = vox.copy(), vox.copy()
        hi_[b, v, c] += 1e-6
        lo_[b, v, c] -= 1e-6
        fd = (loss(hi_) - loss(lo_)) / 2e-6
        assert fd == pytest.approx(gv[b, v, c], rel=1e-5, abs=1e-8)
