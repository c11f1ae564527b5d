"""Pins of the oracle's forward render (Sec. 3.5.1, Eq. 12-15) and its adjoint.

Each check compares the oracle with something other than its own formula:
  * 1-sample special case: w = 1 - exp(-sigma delta), D = w t, N = w n;
  * the telescoped weight sum: W = 1 - exp(-sum_k sigma_k delta);
  * planar SDF (a linear field, so interpolation is exact): N = W n, and a
    constant colour c0 gives C = W c0;
  * depth on a plane converges at first order, as the step shrinks, to the
    continuous volume-rendering integral evaluated with scipy.integrate.quad;
  * a ray through the centre of the sphere: depth ~ hit distance + the
    continuum offset, normal = -d;
  * compositing two halves of a ray with (T1 T2, A1 + T1 A2) gives the whole;
  * empty and non-finite rays give exact zeros;
  * the adjoint equals float64 central differences of the forward;
  * the normal's tolerance scale is the size of the gradient's terms before
    its edge differences cancel (a cell whose edge differences cancel exactly:
    normal 0, scale w * 4 in closed form).
"""
import numpy as np
import pytest
from scipy import integrate

H = np.float32(1.0 / 16)


def _plane_setup(cos_theta=0.8, beta=2 * float(H), C=1, seed=31):
    """Dense block slab around a ray that hits the plane n.x = 0 at t_hit."""
    rng = np.random.default_rng(seed)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    perp = np.cross(n, rng.normal(size=3))
    perp /= np.linalg.norm(perp)
    sin_t = np.sqrt(1 - cos_theta ** 2)
    d = (-cos_theta * n + sin_t * perp).astype(np.float32)
    d = d / np.linalg.norm(d.astype(np.float64))
    t_hit = 1.0
    hit = np.array([0.013, -0.021, 0.007]) - np.dot([0.013, -0.021, 0.007], n) * n
    o = (hit - t_hit * d).astype(np.float32)
    # allocate every block the segment t in [-0.5, 2.5] passes near
    ts = np.linspace(-0.5, 2.5, 4000)
    pts = o[None].astype(np.float64) + ts[:, None] * d[None]
    core = np.unique(np.floor(pts / (8 * float(H))).astype(np.int64), axis=0)
    offs = np.stack(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1], indexing="ij"), -1).reshape(-1, 3)
    blocks = np.unique((core[:, None, :] + offs[None]).reshape(-1, 3), axis=0).astype(np.int32)
    from synth.scenes import voxel_positions
    pos = voxel_positions(blocks, float(H), np.zeros(3))
    vox = np.empty((blocks.shape[0], 512, 1 + C))
    vox[..., 0] = pos @ n
    for ch in range(C):
        vox[..., 1 + ch] = 0.25 + 0.5 * ch
    ray = np.concatenate([o, d]).astype(np.float32)
    # actual ray distance to the plane for the float32 ray
    t_hit_exact = -np.dot(o.astype(np.float64), n) / np.dot(d.astype(np.float64), n)
    return dict(blocks=blocks, vox=vox, n=n, ray=ray, t_hit=t_hit_exact, beta=beta, C=C,
                cos=-np.dot(d.astype(np.float64), n))


def _params(step, t_near, t_far, beta, max_samples):
    return {"step": float(np.float32(step)), "t_near": float(np.float32(t_near)),
            "t_far": float(np.float32(t_far)), "beta": float(np.float32(beta)),
            "max_samples": max_samples}


def _sample_sdf(oracle_lib, s, n):
    """Analytic plane SDF at the oracle's float32 sample positions."""
    xv = s["i"].astype(np.float64) + s["u"].astype(np.float64)
    return (xv * float(H)) @ n


def test_single_sample_closed_form(oracle_lib):
    P = _plane_setup()
    beta = np.float32(P["beta"])
    prm = _params(float(H) / 2, P["t_hit"] - 0.05, P["t_hit"] + 1.0, beta, 1)
    out = oracle_lib.render_forward(P["blocks"], P["vox"], 1, H, np.zeros(3, np.float32),
                                    P["ray"][None], prm)
    s = oracle_lib.ray_samples(P["blocks"], H, np.zeros(3, np.float32), P["ray"], prm)
    assert out["nsamples"][0] == 1 and len(s["k"]) == 1
    f0 = _sample_sdf(oracle_lib, s, P["n"])[0]
    sigma = 0.5 * np.exp(-f0 / float(beta)) / float(beta) if f0 >= 0 else \
        (1 - 0.5 * np.exp(f0 / float(beta))) / float(beta)
    w = 1 - np.exp(-sigma * prm["step"])
    assert out["wsum"][0] == pytest.approx(w, rel=1e-10)
    assert out["depth"][0] == pytest.approx(w * float(s["t"][0]), rel=1e-10)
    np.testing.assert_allclose(out["normal"][0], w * P["n"], rtol=1e-9, atol=1e-12)
    assert out["feat"][0, 0] == pytest.approx(0.25 * w, rel=1e-10)


@pytest.mark.parametrize("max_samples", [2, 7, 128, 1024])
def test_weight_sum_telescopes(oracle_lib, max_samples):
    P = _plane_setup(cos_theta=0.6, C=2)
    prm = _params(float(H) / 2, P["t_hit"] - 0.6, P["t_hit"] + 0.8, P["beta"], max_samples)
    out = oracle_lib.render_forward(P["blocks"], P["vox"], 2, H, np.zeros(3, np.float32),
                                    P["ray"][None], prm)
    s = oracle_lib.ray_samples(P["blocks"], H, np.zeros(3, np.float32), P["ray"], prm)
    f = _sample_sdf(oracle_lib, s, P["n"])
    sigma, _ = oracle_lib.density(f, prm["beta"])
    W = out["wsum"][0]
    assert W == pytest.approx(-np.expm1(-np.sum(sigma) * prm["step"]), rel=1e-12)
    assert 0 <= W <= 1
    # linear SDF: the gradient is n everywhere; constant colours
    np.testing.assert_allclose(out["normal"][0], W * P["n"], rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(out["feat"][0], W * np.array([0.25, 0.75]), rtol=1e-12)


def _continuum_depth(t_hit, cos, beta, t0, t1):
    """E[t] and W of the continuous render of a plane on [t0, t1]."""
    def G(s):  # integral of the unit Laplace CDF
        return 0.5 * np.exp(s) if s <= 0 else s + 0.5 * np.exp(-s)

    def sv(t):
        return cos * (t - t_hit) / beta

    def sigma(t):
        s = sv(t)
        return (0.5 * np.exp(s) if s <= 0 else 1 - 0.5 * np.exp(-s)) / beta

    def T(t):
        return np.exp(-(G(sv(t)) - G(sv(t0))) / cos)

    pts = [t_hit]
    D = integrate.quad(lambda t: t * sigma(t) * T(t), t0, t1, points=pts, limit=400,
                       epsabs=1e-14, epsrel=1e-13)[0]
    W = 1 - T(t1)
    return D / W, W


@pytest.mark.parametrize("cos_theta", [1.0, 0.7])
def test_depth_converges_to_continuum(oracle_lib, cos_theta):
    """The discrete weights of Eq. 15 on the lattice converge to the
    continuous integral at second order in the step (a transmittance that
    included the sample's own opacity, or depth taken at t_{k+1}, would leave
    a first-order error)."""
    P = _plane_setup(cos_theta=cos_theta)
    beta = P["beta"]
    t0, t1 = P["t_hit"] - 10 * beta / P["cos"], P["t_hit"] + 11 * beta / P["cos"]
    E, Wc = _continuum_depth(P["t_hit"], P["cos"], beta, np.float32(t0), np.float32(t1))
    errs = []
    for k in (4, 8, 16, 32):
        prm = _params(beta / k, t0, t1, beta, 1024)
        out = oracle_lib.render_forward(P["blocks"], P["vox"], 1, H, np.zeros(3, np.float32),
                                        P["ray"][None], prm)
        assert out["nsamples"][0] < 1024
        assert out["wsum"][0] == pytest.approx(Wc, abs=3e-5)  # lattice end vs t_far
        errs.append(out["depth"][0] / out["wsum"][0] - E)
    for a, b in zip(errs[:-1], errs[1:]):
        assert abs(b) < abs(a) / 3
    assert abs(errs[-1]) < 5e-5 * beta
    if cos_theta == 1.0:
        # head-on offset of the Laplace density past the surface: 0.3431 beta
        assert (E - P["t_hit"]) / beta == pytest.approx(0.3431, abs=2e-4)


def test_sphere_centre_ray(oracle_lib):
    from synth import workloads
    w = workloads.sphere_tiny()
    h, beta = float(w["h"]), w["params"]["beta"]
    eye = np.array([1.1, -0.7, 0.6])
    eye *= 1.5 / np.linalg.norm(eye)
    d = -eye / np.linalg.norm(eye)
    ray = np.concatenate([eye, d]).astype(np.float32)[None]
    out = oracle_lib.render_forward(w["block_coords"], w["vox"], 3, w["h"], w["origin"], ray,
                                    w["params"])
    assert out["wsum"][0] == pytest.approx(1.0, abs=1e-9)
    E, _ = _continuum_depth(1.0, 1.0, beta, 0.5, 1.5)
    dw = out["depth"][0] / out["wsum"][0]
    # discretisation (step = beta/2) and curvature shift the offset by a few percent of beta
    assert abs(dw - E) < 0.03 * beta
    nw = out["normal"][0] / out["wsum"][0]
    np.testing.assert_allclose(nw, -d, atol=2e-3)


def test_split_and_merge_is_associative(oracle_lib):
    from synth import workloads
    w = workloads.sphere_tiny()
    prm = dict(w["params"])
    rays = w["rays"][::17]
    full = oracle_lib.render_forward(w["block_coords"], w["vox"], 3, w["h"], w["origin"], rays, prm)
    kmid = 150
    t_mid = np.float32(prm["t_near"]) + np.float32(kmid) * np.float32(prm["step"])
    a = oracle_lib.render_forward(w["block_coords"], w["vox"], 3, w["h"], w["origin"], rays,
                                  dict(prm, t_far=float(np.nextafter(t_mid, np.float32(-1)))))
    b = oracle_lib.render_forward(w["block_coords"], w["vox"], 3, w["h"], w["origin"], rays,
                                  dict(prm, t_near=float(t_mid)))
    keep = (a["nsamples"] + b["nsamples"]) <= prm["max_samples"]  # cap not reached
    assert keep.mean() > 0.5
    T1 = 1 - a["wsum"]
    np.testing.assert_allclose((a["wsum"] + T1 * b["wsum"])[keep], full["wsum"][keep], atol=1e-6)
    np.testing.assert_allclose((a["feat"] + T1[:, None] * b["feat"])[keep], full["feat"][keep],
                               atol=1e-6)
    np.testing.assert_allclose((a["depth"] + T1 * b["depth"])[keep], full["depth"][keep],
                               atol=1e-6)
    np.testing.assert_array_equal((a["nsamples"] + b["nsamples"])[keep], full["nsamples"][keep])


def test_empty_and_nonfinite_rays_give_zeros(oracle_lib):
    from synth import workloads
    w = workloads.sphere_tiny()
    rays = np.array([[3, 3, 3, 1, 0, 0], [0, 0, 5, 0, 0, 1], [np.nan, 0, 0, 1, 0, 0],
                     [0, 0, -1.5, 0, np.inf, 1], [0, 0, -1.5, 0, 0, 1]], np.float32)
    out = oracle_lib.render_forward(w["block_coords"], w["vox"], 3, w["h"], w["origin"], rays,
                                    w["params"])
    for r in range(4):
        assert out["nsamples"][r] == 0
        assert out["wsum"][r] == 0 and out["depth"][r] == 0
        assert not out["feat"][r].any() and not out["normal"][r].any()
    assert out["nsamples"][4] > 0


def _loss(oracle_lib, w, vox, rays, prm, g):
    out = oracle_lib.render_forward(w["block_coords"], vox, 3, w["h"], w["origin"], rays, prm)
    return (np.sum(g["feat"] * out["feat"]) + np.sum(g["depth"] * out["depth"])
            + np.sum(g["normal"] * out["normal"]) + np.sum(g["wsum"] * out["wsum"]))


def test_backward_matches_central_differences(oracle_lib):
    from synth import workloads
    w = workloads.sphere_tiny()
    rng = np.random.default_rng(33)
    rays = w["rays"][rng.choice(w["rays"].shape[0], 24, replace=False)]
    prm = w["params"]
    R = rays.shape[0]
    g = {"feat": rng.normal(size=(R, 3)), "depth": rng.normal(size=R),
         "normal": rng.normal(size=(R, 3)), "wsum": rng.normal(size=R)}
    vox = w["vox"].astype(np.float64)
    grad, mag = oracle_lib.render_backward(w["block_coords"], vox, 3, w["h"], w["origin"], rays,
                                           prm, g["feat"], g["depth"], g["normal"], g["wsum"],
                                           with_mag=True)
    nz = np.argwhere(np.abs(grad) > 1e-3 * np.abs(grad).max())
    assert nz.shape[0] > 50
    pick = nz[rng.choice(nz.shape[0], 40, replace=False)]
    # make sure SDF entries (channel 0) are among the checked ones
    sdf_nz = nz[nz[:, 2] == 0]
    pick = np.concatenate([pick, sdf_nz[rng.choice(sdf_nz.shape[0], 20, replace=False)]])
    for b, v, ch in pick:
        eps = 1e-5 * float(w["h"]) if ch == 0 else 1e-5
        vp, vm = vox.copy(), vox.copy()
        vp[b, v, ch] += eps
        vm[b, v, ch] -= eps
        fd = (_loss(oracle_lib, w, vp, rays, prm, g) - _loss(oracle_lib, w, vm, rays, prm, g)) / (2 * eps)
        assert abs(fd - grad[b, v, ch]) <= 1e-6 * mag[b, v, ch] + 1e-9, (b, v, ch, fd, grad[b, v, ch])


def test_normal_scale_counts_terms_before_cancellation(oracle_lib):
    """One sample at the centre of a cell face (u = (1/2, 1/2, 0)) in a single
    block, h = 1: the cell's SDF corners are 1, 3 (x edge +2) and 3, 1 (x edge
    -2) on the z = 0 face and 2 on the z = 1 face, so every gradient component
    cancels to 0 while each sums four terms of size 1/2 (|theta_1| + |theta_0|)
    (or 1/4 of it along z): the tolerance scale of the normal is w (4, 4, 4)."""
    C = 1
    blocks = np.zeros((1, 3), np.int32)
    vox = np.full((1, 512, 1 + C), 2.0)
    vox[..., 1] = 0.5

    def at(x, y, z):
        return x + 8 * y + 64 * z

    vox[0, at(3, 2, 0), 0] = 1.0
    vox[0, at(4, 2, 0), 0] = 3.0
    vox[0, at(3, 3, 0), 0] = 3.0
    vox[0, at(4, 3, 0), 0] = 1.0
    ray = np.array([[3.5, 2.5, -5.0, 0.0, 0.0, 1.0]], np.float32)
    prm = _params(0.5, 0.0, 20.0, 1.0, 1)
    out = oracle_lib.render_forward(blocks, vox, C, np.float32(1.0), np.zeros(3, np.float32), ray,
                                    prm, with_mag=True)
    assert out["nsamples"][0] == 1
    f = 0.25 * (1.0 + 3.0 + 3.0 + 1.0)
    sigma = 0.5 * np.exp(-f)  # beta = 1, f >= 0
    w = -np.expm1(-sigma * 0.5)
    assert out["wsum"][0] == pytest.approx(w, rel=1e-12)
    np.testing.assert_allclose(out["normal"][0], 0.0, atol=1e-15)
    np.testing.assert_allclose(out["mag_normal"][0], 4.0 * w, rtol=1e-12)
    # never below the magnitude after cancellation, on an ordinary scene
    P = _plane_setup(cos_theta=0.7)
    prm = _params(float(H) / 2, P["t_hit"] - 0.6, P["t_hit"] + 0.8, P["beta"], 128)
    o = oracle_lib.render_forward(P["blocks"], P["vox"], 1, H, np.zeros(3, np.float32),
                                  P["ray"][None], prm, with_mag=True)
    assert np.all(o["mag_normal"] >= np.abs(o["normal"]) * (1 - 1e-12))
