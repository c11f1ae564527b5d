"""Permutohedral-lattice filter and mean-field CRF update (Sec. 3.5.3) on the
GPU against the oracle.

Bars: number of lattice vertices bit-exact (the simplex vertices are
float32 decisions on both sides); filter output within 1e-5 of the oracle's
filter of |values| (all weights are positive); mean-field marginals within
1e-5 after each of 3 updates."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


def _sg():
    import paper_2305_13220_amd as sg
    return sg


def _surface_features(n_sem=16, n=20000, seed=0):
    """CRF nodes on the room's surface: points of a depth frame, features
    (xyz / 20 cm, rgb / 0.3), unary from noisy one-hot labels."""
    from synth import cameras, workloads
    fr = workloads.room_depth_frames(n_frames=2, W=160, H=120, n_sem=n_sem)
    pix = np.concatenate([cameras.frame_pixels(i, 160, 120) for i in range(2)])
    d = fr["depth"].reshape(-1)
    ok = np.isfinite(d)
    rays = cameras.pixel_rays(fr["cams"], pix).astype(np.float64)
    R = fr["cams"][pix[:, 0], 4:].astype(np.float64).reshape(-1, 3, 4)[:, :, 2]
    t = d / np.einsum("ij,ij->i", rays[:, 3:], R)
    xyz = rays[:, :3] + t[:, None] * rays[:, 3:]
    feat = fr["feat"].reshape(-1, 3 + n_sem)
    rng = np.random.default_rng(seed)
    idx = rng.choice(np.flatnonzero(ok), min(n, ok.sum()), replace=False)
    pos = np.concatenate([xyz[idx] / 0.2, feat[idx, :3] / 0.3], 1).astype(np.float32)
    lab = feat[idx, 3:].copy()
    flip = rng.random(len(idx)) < 0.1  # wrong labels the pairwise term should correct
    lab[flip] = np.eye(n_sem)[rng.integers(0, n_sem, flip.sum())]
    unary = (-np.log(np.clip(lab * 0.7 + 0.3 / n_sem + rng.uniform(0, 0.2, (len(idx), n_sem)),
                             1e-6, None))).astype(np.float32)
    return pos, unary


@pytest.mark.parametrize("d", [1, 3, 6, 9, 17, 22])
def test_lattice_filter_matches_oracle(d):
    sg = _sg()
    rng = np.random.default_rng(d)
    pos = rng.normal(scale=4.0, size=(20000, d)).astype(np.float32)
    val = rng.normal(size=(20000, 5)).astype(np.float32)
    lat = sg.Lattice(to_dev(pos), max_values=8)
    out = lat.filter(to_dev(val)).cpu().numpy()
    want, nv = oracle.lattice_filter(pos, val)
    mag, _ = oracle.lattice_filter(pos, np.abs(val))
    assert lat.n_vertices == nv
    bad = np.abs(out - want) > 1e-5 * mag + 1e-30
    assert not bad.any(), f"{bad.sum()} values out of tolerance"


def test_crf_meanfield_on_surface_samples():
    sg = _sg()
    pos, unary = _surface_features()
    lat = sg.Lattice(to_dev(pos), max_values=16)
    _, nv = oracle.lattice_filter(pos, np.ones((len(pos), 1)))
    assert lat.n_vertices == nv
    for it in (0, 1, 3):
        Q = lat.meanfield(to_dev(unary), 5.0, it).cpu().numpy()
        want = oracle.crf_meanfield(pos, unary, 5.0, it)
        err = np.abs(Q - want).max()
        assert err <= 1e-5, f"iteration {it}: {err}"
    # the pairwise term changes the labels of some nodes
    q0 = oracle.crf_meanfield(pos, unary, 5.0, 0)
    assert (q0.argmax(1) != want.argmax(1)).mean() > 0.01


def test_crf_meanfield_compat_on_surface_samples():
    """Mean field with a label compatibility matrix mu against the oracle.
    The softmax arguments carry the message sum_k mu(l,k) F(k), so the bar
    scales with the largest row sum of |mu|: 2e-6 of it, which is the 1e-5
    bar of the Potts weight 5 above.  The textbook Potts matrix 5 (1 - I)
    reproduces the oracle's Potts marginals, and an asymmetric matrix (a
    label attracted to its own kind and pushed towards some others) its own."""
    sg = _sg()
    pos, unary = _surface_features()
    L = unary.shape[1]
    lat = sg.Lattice(to_dev(pos), max_values=16)
    rng = np.random.default_rng(31)
    potts = (5.0 * (1.0 - np.eye(L))).astype(np.float32)
    asym = (-5.0 * np.eye(L) + 0.3 * rng.random((L, L))).astype(np.float32)
    for mu, what in ((potts, "potts"), (asym, "asymmetric")):
        tol = 2e-6 * np.abs(mu).sum(1).max()
        for it in (1, 3):
            Q = lat.meanfield(to_dev(unary), 0.0, it, compat=to_dev(mu)).cpu().numpy()
            if what == "potts":
                want = oracle.crf_meanfield(pos, unary, 5.0, it)
            else:
                want = oracle.crf_meanfield_compat(pos, unary, mu.astype(np.float64), it)
            err = np.abs(Q - want).max()
            assert err <= tol, f"{what}, iteration {it}: {err} > {tol}"
    with pytest.raises(ValueError):
        lat.meanfield(to_dev(unary), 0.0, 1, compat=to_dev(potts[:4, :4].copy()))


def test_crf_meanfield_compat_backward_matches_oracle():
    """Gradients of <gQ, Q> after 2 compatibility mean-field updates on 20,000
    surface samples with respect to the unaries and to mu.  float32 sums of
    20,000 signed products on the GPU against float64: g_mu within 1e-3 of its
    largest entry, g_unary within 1e-4 of its largest entry; both twice in a
    row (the workspace is reused by the second call)."""
    sg = _sg()
    pos, unary = _surface_features()
    n, L = unary.shape
    lat = sg.Lattice(to_dev(pos), max_values=16)
    rng = np.random.default_rng(32)
    mu = (-5.0 * np.eye(L) + 0.3 * rng.random((L, L))).astype(np.float32)
    gQ = rng.normal(size=(n, L)).astype(np.float32)
    want_u, want_mu = oracle.crf_meanfield_compat_backward(pos, unary, mu.astype(np.float64), 2, gQ)
    for call in range(2):
        g_u, g_mu = lat.meanfield_backward(to_dev(unary), to_dev(mu), 2, to_dev(gQ))
        g_u, g_mu = g_u.cpu().numpy(), g_mu.cpu().numpy()
        e_mu = np.abs(g_mu - want_mu).max() / np.abs(want_mu).max()
        e_u = np.abs(g_u - want_u).max() / np.abs(want_u).max()
        print(f"call {call}: relative errors g_mu {e_mu:.2e}, g_unary {e_u:.2e}", flush=True)
        assert e_mu <= 1e-3, f"g_mu: {e_mu}"
        assert e_u <= 1e-4, f"g_unary: {e_u}"


@pytest.mark.parametrize("L,iters", [(16, 0), (1, 2), (5, 1)])
def test_crf_meanfield_compat_edge_cases(L, iters):
    """No update (the gradient of softmax(-unary) only, g_mu zero), a single
    label (marginals 1, gradients zero) and a label count that is not a power
    of two; 3,001 points (a ragged last workgroup)."""
    sg = _sg()
    rng = np.random.default_rng(50 + L)
    n = 3001
    pos = rng.normal(scale=1.5, size=(n, 3)).astype(np.float32)
    unary = rng.normal(size=(n, L)).astype(np.float32)
    mu = (-2.0 * np.eye(L) + 0.5 * rng.random((L, L))).astype(np.float32)
    gQ = rng.normal(size=(n, L)).astype(np.float32)
    lat = sg.Lattice(to_dev(pos), max_values=max(L, 1))
    Q = lat.meanfield(to_dev(unary), 0.0, iters, compat=to_dev(mu)).cpu().numpy()
    want_Q = oracle.crf_meanfield_compat(pos, unary, mu.astype(np.float64), iters)
    assert np.abs(Q - want_Q).max() <= 2e-6 * max(1.0, np.abs(mu).sum(1).max())
    g_u, g_mu = lat.meanfield_backward(to_dev(unary), to_dev(mu), iters, to_dev(gQ))
    g_u, g_mu = g_u.cpu().numpy(), g_mu.cpu().numpy()
    want_u, want_mu = oracle.crf_meanfield_compat_backward(pos, unary, mu.astype(np.float64),
                                                            iters, gQ)
    if L == 1:
        assert not g_u.any() and not g_mu.any()
        return
    if iters == 0:
        assert not g_mu.any()
    else:
        assert np.abs(g_mu - want_mu).max() <= 1e-3 * np.abs(want_mu).max()
    assert np.abs(g_u - want_u).max() <= 1e-4 * np.abs(want_u).max()


def test_crf_meanfield_compat_backward_rejects_overlap():
    """The gradient of the unaries may not overwrite the upstream gradient it
    still has to read: rejected on the host before any launch."""
    sg = _sg()
    from paper_2305_13220_amd import _lib
    rng = np.random.default_rng(60)
    n, L = 500, 4
    lat = sg.Lattice(to_dev(rng.normal(size=(n, 3)).astype(np.float32)), max_values=L)
    u = to_dev(rng.normal(size=(n, L)).astype(np.float32))
    mu = to_dev(np.eye(L, dtype=np.float32))
    gQ = to_dev(rng.normal(size=(n, L)).astype(np.float32))
    nb = _lib.lib().sg_crf_meanfield_compat_backward_ws_bytes(n, L, 1)
    ws = torch.empty(nb, dtype=torch.uint8, device=u.device)
    g_mu = torch.empty((L, L), dtype=torch.float32, device=u.device)
    rc = _lib.lib().sg_crf_meanfield_compat_backward(lat._h, _lib.ptr(u), L, _lib.ptr(mu), 1,
                                                     _lib.ptr(gQ), _lib.ptr(gQ), _lib.ptr(g_mu),
                                                     _lib.ptr(ws), nb, None)
    assert rc == -1 and b"overlap" in _lib.lib().sg_last_error()
    torch.cuda.synchronize()


def test_lattice_invalid_inputs():
    sg = _sg()
    pos = np.zeros((10, 3), np.float32)
    pos[3, 1] = np.nan
    with pytest.raises(sg.SgridError, match="finite"):
        sg.Lattice(to_dev(pos))
    with pytest.raises(sg.SgridError):
        sg.Lattice(to_dev(np.zeros((10, 25), np.float32)))
    lat = sg.Lattice(to_dev(np.zeros((10, 3), np.float32)), max_values=2)
    with pytest.raises(sg.SgridError):
        lat.filter(to_dev(np.zeros((10, 3), np.float32)))
    assert lat.n_vertices == 4


def test_crf_label_loss_matches_oracle():
    sg = _sg()
    rng = np.random.default_rng(21)
    n, L, Cf, col0 = 5000, 16, 19, 3
    feat = rng.normal(scale=2.0, size=(n, Cf)).astype(np.float32)
    Q = rng.dirichlet(np.ones(L) * 0.5, size=n).astype(np.float32) + 1e-6
    Q = (Q / Q.sum(1, keepdims=True)).astype(np.float32)
    loss, g = sg.crf_label_loss(to_dev(feat), to_dev(Q), col0, 0.3)
    want_l, want_g = oracle.crf_label_loss(feat[:, col0:col0 + L], Q, 0.3)
    loss, g = loss.cpu().numpy(), g.cpu().numpy()
    scale = 0.3 * (1.0 + np.abs(np.log(Q)).max(1) + np.abs(feat[:, col0:col0 + L]).max(1))
    assert (np.abs(loss - want_l) <= 1e-5 * scale).all()
    assert (np.abs(g[:, col0:col0 + L] - want_g) <= 1e-5 * scale[:, None]).all()
    assert not g[:, :col0].any() and not g[:, col0 + L:].any()


def test_crf_label_loss_into_voxels_chain():
    """Surface samples of the 2 cm room with 16 semantic channels: query the
    logits, mean field on (xyz, rgb) features, label loss, and its gradient
    through the query adjoint into the voxels; the GPU chain against the
    oracle's, within 1e-3 of the largest gradient (float32 queries shift the
    unaries slightly and the shift propagates through three updates)."""
    sg = _sg()
    from synth import scenes
    from gpu_helpers import make_grid
    room = scenes.room_scene(h=0.02, band_vox=3, seed=0, n_sem=16)
    pos, _ = _surface_features()
    xyz = (pos[:, :3] * 0.2).astype(np.float32)  # world points of the nodes
    g = make_grid(room)
    vox = to_dev(room["vox"])
    q = sg.query(g, vox, to_dev(xyz))
    valid = q["valid"].cpu().numpy().astype(bool)
    assert valid.mean() > 0.9
    keep = np.flatnonzero(valid)
    xyz, pos = xyz[keep], pos[keep]
    feat = sg.query(g, vox, to_dev(xyz))["feat"]
    logits = feat[:, 3:].contiguous()
    unary = -torch.log_softmax(logits, 1)
    lat = sg.Lattice(to_dev(pos), max_values=16)
    Q = lat.meanfield(unary.contiguous(), 5.0, 3)
    _, g_feat = sg.crf_label_loss(feat, Q, 3, 0.1)
    gv = sg.query_backward(g, room["vox"].shape, to_dev(xyz), g_feat=g_feat).cpu().numpy()
    # oracle chain
    _, _, _, ofeat = oracle.query(room["block_coords"], room["vox"], 19, room["h"], room["origin"], xyz)
    ol = ofeat[:, 3:]
    ou = -(ol - ol.max(1, keepdims=True) - np.log(np.exp(ol - ol.max(1, keepdims=True)).sum(1, keepdims=True)))
    oQ = oracle.crf_meanfield(pos, ou, 5.0, 3)
    _, og = oracle.crf_label_loss(ol, oQ, 0.1)
    ogf = np.concatenate([np.zeros((len(xyz), 3)), og], 1)
    want, _ = oracle.query_backward(room["block_coords"], 19, room["h"], room["origin"], xyz,
                                    g_feat=ogf)
    assert np.abs(want).max() > 0
    assert np.abs(gv - want).max() <= 1e-3 * np.abs(want).max()


def test_crf_property_loss_matches_oracle():
    """Colour loss of room surface samples: the lattice over (xyz, semantic
    one-hot) features, the filter of [rgb, 1], the loss against the oracle's
    on the same filter inputs (filter within the filter bar, loss and
    gradient within 1e-4 relative plus 1e-6)."""
    sg = _sg()
    from synth import workloads
    fr = workloads.room_depth_frames(n_frames=2, W=160, H=120, n_sem=16)
    pos, _ = _surface_features()
    rng = np.random.default_rng(2)
    rgb = np.clip(rng.normal(0.5, 0.2, size=(len(pos), 3)), 0, 1).astype(np.float32)
    feats = np.concatenate([pos[:, :3], rng.normal(size=(len(pos), 2)).astype(np.float32)], 1)
    vals = np.concatenate([rgb, np.ones((len(pos), 1), np.float32)], 1)
    lat = sg.Lattice(to_dev(feats), max_values=4)
    filt = lat.filter(to_dev(vals))
    feat = np.concatenate([np.zeros((len(pos), 1), np.float32), rgb], 1)  # [sdf, rgb]
    loss, g = sg.crf_property_loss(to_dev(feat), filt, 1, 0.4)
    ofilt, _ = oracle.lattice_filter(feats, vals)
    ol, og = oracle.crf_property_loss(rgb, ofilt, 0.4)
    np.testing.assert_allclose(loss.cpu().numpy(), ol, rtol=1e-4, atol=1e-6)
    np.testing.assert_allclose(g.cpu().numpy()[:, 1:], og, rtol=1e-4, atol=1e-6)
    assert not g.cpu().numpy()[:, 0].any()


@pytest.mark.parametrize("which", ["sphere", "room"])
def test_surface_points_match_oracle(which):
    """Hit flags equal except where a sign decision is within float32
    rounding of zero (at most 1 in 1,000 rays); points, where the decisions
    have a margin above 1e-5 h, within 1e-4 of the step plus 1e-5 of the
    coordinates."""
    sg = _sg()
    from synth import workloads
    from gpu_helpers import make_grid
    w = workloads.sphere_tiny() if which == "sphere" else workloads.room_2cm()
    rays_np = w["rays"] if which == "sphere" else w["rays"][:16384]
    g = make_grid(w)
    pts, hit = sg.surface_points(g, to_dev(w["vox"]), to_dev(rays_np), w["params"])
    pts, hit = pts.cpu().numpy(), hit.cpu().numpy().astype(bool)
    ohit, opts, margin = oracle.surface_points(w["block_coords"], w["vox"], 3, w["h"], w["origin"],
                                               rays_np, w["params"])
    assert ohit.mean() > 0.3
    differ = hit != ohit
    assert differ.sum() <= max(2, int(1e-3 * len(hit)))
    both = hit & ohit & (margin > 1e-5 * float(w["h"]))
    err = np.abs(pts[both] - opts[both]).max()
    assert err <= 1e-4 * float(w["params"]["step"]) + 1e-5 * np.abs(opts[both]).max()
    assert not pts[~hit].any()
