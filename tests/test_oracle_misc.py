"""Pins of the oracle's footprint counts, camera rays and training glue.

* Footprint: per-ray distinct voxels / blocks equal Python-set counts over
  the corners of the brute-force sample list.
* Rays: projecting o + s d back through the pinhole camera lands on the
  pixel centre (the projection of Eq. 3 inverts the oracle's unprojection).
* Adam and RMSProp steps equal torch.optim's; the loss gradient equals
  torch.autograd's gradient of the same squared-L2 loss.
"""
import numpy as np
import pytest
import torch


def test_footprint_matches_sets(oracle_lib):
    from synth import workloads
    w = workloads.sphere_tiny()
    rng = np.random.default_rng(41)
    rays = w["rays"][rng.choice(w["rays"].shape[0], 60, replace=False)]
    counts, touched = oracle_lib.footprint(w["block_coords"], w["h"], w["origin"], rays,
                                           w["params"], with_touched=True)
    all_vox = set()
    for r in range(rays.shape[0]):
        s = oracle_lib.ray_samples(w["block_coords"], w["h"], w["origin"], rays[r], w["params"])
        # corner voxels by global integer coordinate, blocks by coordinate
        vox = {tuple(s["i"][q] + [a & 1, (a >> 1) & 1, (a >> 2) & 1])
               for q in range(len(s["k"])) for a in range(8)}
        blk = {tuple(np.floor_divide(v, 8)) for v in vox}
        assert counts[r, 0] == len(s["k"])
        assert counts[r, 1] == len(vox)
        assert counts[r, 2] == len(blk)
        bidx = {tuple(b): i for i, b in enumerate(w["block_coords"])}
        for v in vox:
            b = np.floor_divide(v, 8)
            l = np.asarray(v) - 8 * b
            all_vox.add(bidx[tuple(b)] * 512 + int(l[0] + 8 * l[1] + 64 * l[2]))
    assert int(touched.sum()) == len(all_vox)
    assert set(np.flatnonzero(touched)) == all_vox


def test_pinhole_rays_project_back(oracle_lib):
    from synth import cameras
    rng = np.random.default_rng(42)
    poses = [cameras.look_at(rng.uniform(-2, 2, 3), rng.uniform(-1, 1, 3)) for _ in range(4)]
    cams = cameras.make_cams(poses, 554.3, 541.0, 320.0, 240.0)
    pix = np.stack([rng.integers(0, 4, 500), rng.integers(0, 640, 500),
                    rng.integers(0, 480, 500)], -1).astype(np.int32)
    rays = oracle_lib.rays_pinhole(cams, pix)
    np.testing.assert_allclose(np.linalg.norm(rays[:, 3:], axis=1), 1.0, atol=1e-14)
    for r in range(pix.shape[0]):
        K = cams[pix[r, 0]].astype(np.float64)
        M = K[4:].reshape(3, 4)
        Rm, t = M[:, :3], M[:, 3]
        np.testing.assert_allclose(rays[r, :3], t, atol=0)
        pc = np.linalg.solve(Rm, rays[r, :3] + 2.5 * rays[r, 3:] - t)  # world -> camera
        u = K[0] * pc[0] / pc[2] + K[2]
        v = K[1] * pc[1] / pc[2] + K[3]
        assert pc[2] > 0
        assert u == pytest.approx(pix[r, 1] + 0.5, abs=1e-6)
        assert v == pytest.approx(pix[r, 2] + 0.5, abs=1e-6)
    bad = oracle_lib.rays_pinhole(cams, np.array([[4, 0, 0], [-1, 0, 0]], np.int32))
    assert np.isnan(bad).all()


@pytest.mark.parametrize("kind", [0, 1])
def test_optimiser_matches_torch(oracle_lib, kind):
    rng = np.random.default_rng(43)
    p0 = rng.normal(size=1000)
    p = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    opt = (torch.optim.Adam([p], lr=lr, betas=(b1, b2), eps=eps) if kind == 0 else
           torch.optim.RMSprop([p], lr=lr, alpha=b2, eps=eps))
    mine = p0.copy()
    m = np.zeros_like(p0) if kind == 0 else None
    v = np.zeros_like(p0)
    for t in range(1, 6):
        g = rng.normal(size=1000)
        p.grad = torch.tensor(g)
        opt.step()
        mine, m, v = oracle_lib.optim_step(kind, mine, g, m, v, lr, b1, b2, eps, t)
    np.testing.assert_allclose(mine, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_l2_loss_grad_matches_autograd(oracle_lib):
    rng = np.random.default_rng(44)
    R, C = 257, 3
    arrs = [rng.normal(size=s) for s in [(R, C), (R, C), (R,), (R,), (R, 3), (R, 3)]]
    loss, gc, gd, gn = oracle_lib.l2_loss_grad(*arrs, 0.1, 0.05)
    t = [torch.tensor(a, requires_grad=(i % 2 == 0)) for i, a in enumerate(arrs)]
    L = (torch.nn.functional.mse_loss(t[0], t[1], reduction="sum")
         + 0.1 * torch.nn.functional.mse_loss(t[2], t[3], reduction="sum")
         + 0.05 * torch.nn.functional.mse_loss(t[4], t[5], reduction="sum")) / R
    L.backward()
    assert loss == pytest.approx(L.item(), rel=1e-13)
    for mine, ref in ((gc, t[0]), (gd, t[2]), (gn, t[4])):
        np.testing.assert_allclose(mine, ref.grad.numpy(), rtol=1e-13)


def test_paper_hyperparameters_fixture():
    """The loss weights the losses use are the paper's (supplement)."""
    import json
    import os
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hyperparameters.json")))
    assert d["lambda_depth"]["value"] == 0.1 and d["lambda_normal"]["value"] == 0.05
    assert d["block_dim"]["value"] == 8
    assert d["rays_per_image"]["value"] * d["images_per_batch"]["value"] == 65536
