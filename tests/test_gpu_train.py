"""Differentiation at scale on the noisy 2 cm room (SDF noise 0.5 voxel, RGB
noise 0.1): the float32 GPU gradient of the squared-L2 rendering loss
against float64 central differences of the oracle's loss on 64 sampled
voxels, and a short optimisation that must reduce the loss and the SDF error
against the clean grid."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import make_grid, to_dev

pytestmark = pytest.mark.gpu

LD, LN = 0.1, 0.05


@pytest.fixture(scope="module")
def noisy():
    from synth import workloads
    return workloads.room_2cm_noisy(n_rays=262144)


def _loss_on(w, vox64, rays, ref, R_total):
    o = oracle.render_forward(w["block_coords"], vox64, 3, w["h"], w["origin"], rays, w["params"])
    dc = o["feat"] - ref["feat"]
    dd = o["depth"] - ref["depth"]
    dn = o["normal"] - ref["normal"]
    return (np.sum(dc * dc) + LD * np.sum(dd * dd) + LN * np.sum(dn * dn)) / R_total


def test_gradient_matches_central_differences(noisy):
    import paper_2305_13220_amd as sg
    w = noisy
    rng = np.random.default_rng(77)
    R = 4096
    rays = w["rays"][rng.choice(w["rays"].shape[0], R, replace=False)]
    clean = oracle.render_forward(w["block_coords"], w["clean_vox"], 3, w["h"], w["origin"], rays,
                                  w["params"])
    ref = {"feat": clean["feat"], "depth": clean["depth"], "normal": clean["normal"]}
    g = make_grid(w)
    vox = to_dev(w["vox"])
    refd = {k: to_dev(v.astype(np.float32)) for k, v in ref.items()}
    _, grad = sg.render_l2_step(g, vox, to_dev(rays), w["params"], refd, LD, LN)
    grad = grad.cpu().numpy().astype(np.float64)
    # which rays touch which voxels (oracle sample lists)
    touch = {}
    for r in range(R):
        s = oracle.ray_samples(w["block_coords"], w["h"], w["origin"], rays[r], w["params"])
        for vid in set((s["blk"] * 512 + s["loc"]).ravel().tolist()):
            touch.setdefault(vid, []).append(r)
    vids = np.array(sorted(touch))
    mags = np.abs(grad.reshape(-1, 4)[vids])
    picked = []
    for ch in (0, 1, 2, 3):
        cand = vids[mags[:, ch] > 1e-3 * mags[:, ch].max()]
        picked += [(int(v), ch) for v in rng.choice(cand, 16, replace=False)]
    vox64 = w["vox"].astype(np.float64)
    h = float(w["h"])
    for vid, ch in picked:
        rr = touch[vid]
        sub = rays[rr]
        subref = {k: v[rr] for k, v in ref.items()}
        b, l = divmod(vid, 512)
        eps = 1e-4 * h if ch == 0 else 1e-4
        vp, vm = vox64.copy(), vox64.copy()
        vp[b, l, ch] += eps
        vm[b, l, ch] -= eps
        fd = (_loss_on(w, vp, sub, subref, R) - _loss_on(w, vm, sub, subref, R)) / (2 * eps)
        got = grad[b, l, ch]
        assert abs(got - fd) <= 1e-3 * abs(fd), (vid, ch, got, fd)


def test_optimisation_reduces_loss_and_sdf_error(noisy):
    import paper_2305_13220_amd as sg
    from paper_2305_13220_amd.train import TrainConfig, Trainer, render_reference_images
    w = noisy
    g = make_grid(w)
    clean = to_dev(w["clean_vox"])
    vox = to_dev(w["vox"])
    cams = to_dev(w["cams"])
    ref = render_reference_images(g, clean, cams, w["W"], w["H"], w["params"])
    # voxels seen by the training rays: measure the SDF error there
    pix = torch.from_numpy(w["pix"][:65536]).to(clean.device)
    _, touched = sg.render_footprint(g, sg.rays_pinhole(cams, pix), w["params"], touched=True)
    seen = touched.view(-1, 512).bool()
    err0 = ((vox[..., 0] - clean[..., 0])[seen]).pow(2).mean().sqrt().item()
    tr = Trainer(g, vox, cams, w["W"], w["H"], w["params"], ref,
                 TrainConfig(rays_per_step=262144, lr=2e-3, seed=3))
    losses = [tr.step(with_loss=True).item() for _ in range(40)]
    err1 = ((vox[..., 0] - clean[..., 0])[seen]).pow(2).mean().sqrt().item()
    assert np.mean(losses[-5:]) < 0.7 * np.mean(losses[:5]), losses
    assert err1 < err0, (err0, err1)
