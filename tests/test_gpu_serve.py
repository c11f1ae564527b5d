"""Serving: packed multi-grid launches (continuous batching, HBM-budget
admission, graph replay) give every request exactly the result it gets alone
from the plain per-call path."""
import numpy as np
import pytest
import torch

from gpu_helpers import make_grid, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def resident():
    from synth import cameras, scenes, workloads
    sph = workloads.sphere_tiny()
    room = workloads.room_2cm(n_rays=1024)
    sph2 = scenes.sphere_scene(h=1.0 / 40, radius=0.6, band_vox=3, seed=9)
    grids, poses = [], []
    for w, prm, cams in (
            (sph, sph["params"], cameras.orbit_cams(seed=1, n=4, radius=1.5)),
            (room, room["params"], room["cams"][:6]),
            (sph2, {"step": float(np.float32(1 / 80)), "t_near": 0.2, "t_far": 3.0,
                    "beta": float(np.float32(1 / 40)), "max_samples": 96},
             cameras.orbit_cams(seed=2, n=4, radius=1.8))):
        grids.append((make_grid(w), to_dev(w["vox"]), prm))
        poses.append([c for c in cams])
    return grids, poses


def _requests(poses, n, seed, resolutions=((64, 48), (160, 120), (97, 61))):
    from paper_2305_13220_amd.serve import poisson_requests
    return poisson_requests(n, qps=1e9, n_grids=len(poses), cams_per_grid=poses,
                            resolutions=resolutions, seed=seed)


@pytest.mark.parametrize("use_graph,launch,order", [(False, "multi_grid", "fifo"),
                                                    (True, "multi_grid", "srpt"),
                                                    (False, "per_grid", "srpt"),
                                                    (True, "per_grid", "fifo")])
def test_packed_mix_equals_alone(resident, use_graph, launch, order):
    from paper_2305_13220_amd.serve import PackedServer, PlainServer
    grids, poses = resident
    mixed = _requests(poses, 24, seed=4)
    alone = _requests(poses, 24, seed=4)
    # small ticks: requests split across ticks and share them
    srv = PackedServer(grids, C=3, tick_rays=7000, max_slots=16, use_graph=use_graph,
                       launch=launch, order=order)
    srv.run(mixed, realtime=False)
    PlainServer(grids, C=3).run(alone, realtime=False)
    for a, b in zip(mixed, alone):
        assert a.done is not None
        for k in ("feat", "depth", "normal", "wsum", "nsamples"):
            assert torch.equal(a.out[k], b.out[k]), (a.rid, k)


def test_budget_limits_requests_in_flight(resident):
    from paper_2305_13220_amd.serve import PackedServer
    grids, poses = resident
    reqs = _requests(poses, 12, seed=5, resolutions=((160, 120),))
    per = reqs[0].out_bytes(3)
    srv = PackedServer(grids, C=3, hbm_budget_bytes=2 * per, tick_rays=5000, max_slots=8,
                       use_graph=True)
    admitted_at, seen = [], []
    orig = srv.tick

    def spy(work):
        live = {id(r) for r, _, _ in work}
        seen.append(len(live))
        return orig(work)

    srv.tick = spy
    srv.run(reqs, realtime=False)
    assert all(r.done is not None for r in reqs)
    assert max(seen) <= 2  # never more than two requests' outputs in flight


def _check_pixels_against_oracle(w, C, cam, pix_idx, width, out, what):
    """Pixels pix_idx of a frame rendered through a packed launch against the
    oracle: the rays are the library's pinhole rays of those pixels (the
    function the packed kernels evaluate in registers), themselves checked
    against the oracle's pinhole rays; then the oracle renders them."""
    import oracle
    import paper_2305_13220_amd as sg
    from gpu_helpers import check_forward
    pix_idx = np.unique(np.asarray(pix_idx, np.int64))
    pix = np.stack([np.zeros_like(pix_idx), pix_idx % width, pix_idx // width], 1).astype(np.int32)
    cams = np.asarray(cam, np.float32).reshape(1, 16)
    rays = sg.rays_pinhole(to_dev(cams), to_dev(pix)).cpu().numpy()
    np.testing.assert_allclose(rays, oracle.rays_pinhole(cams, pix), atol=2e-6, rtol=0)
    ref = oracle.render_forward(w["block_coords"], w["vox"], C, w["h"], w["origin"], rays,
                                w["params"], with_mag=True)
    sel = torch.from_numpy(pix_idx).to(out["depth"].device)
    got = {k: v[sel] for k, v in out.items()}
    check_forward(got, ref, what=what)


@pytest.mark.parametrize("launch", ["multi_grid", "per_grid"])
def test_packed_pixels_match_oracle(resident, launch):
    """Every request of a packed run (requests split over ticks and sharing
    them) at sampled pixels, including the first and last pixel of every
    slot, against the oracle: sample counts bit for bit, outputs within
    1e-5 of their magnitude sums."""
    from paper_2305_13220_amd.serve import PackedServer
    from synth import scenes, workloads
    grids, poses = resident
    srcs = [workloads.sphere_tiny(), workloads.room_2cm(n_rays=1024),
            scenes.sphere_scene(h=1.0 / 40, radius=0.6, band_vox=3, seed=9)]
    srcs = [dict(s, params=dict(prm)) for s, (_, _, prm) in zip(srcs, grids)]
    reqs = _requests(poses, 10, seed=7)
    srv = PackedServer(grids, C=3, tick_rays=6000, max_slots=16, launch=launch)
    ends = {r.rid: set() for r in reqs}
    orig = srv.tick

    def spy(work):
        for r, p0, cnt in work:
            ends[r.rid].update((p0, p0 + cnt - 1))
        return orig(work)

    srv.tick = spy
    srv.run(reqs, realtime=False)
    srv.close()
    rng = np.random.default_rng(11)
    for r in reqs:
        assert len(ends[r.rid]) >= 2
        idx = np.concatenate([rng.integers(0, r.pixels, 150), sorted(ends[r.rid])])
        _check_pixels_against_oracle(srcs[r.grid], 3, r.cam, idx, r.width, r.out,
                                     f"{launch} request {r.rid} grid {r.grid}")


def test_full_hd_request_over_three_ticks_matches_oracle(resident):
    """One 1920x1080 request on the room, split over three ticks of a packed
    multi-grid server, against the oracle at sampled pixels and the first and
    last pixel of each tick."""
    from paper_2305_13220_amd.serve import PackedServer, poisson_requests
    from synth import workloads
    grids, poses = resident
    room = workloads.room_2cm(n_rays=1024)
    req = poisson_requests(1, qps=1e9, n_grids=3, cams_per_grid=[poses[1]] * 3,
                           resolutions=((1920, 1080),), seed=3)[0]
    req.grid = 1
    srv = PackedServer(grids, C=3, tick_rays=800_000, max_slots=4)
    seen = []
    orig = srv.tick

    def spy(work):
        seen.extend((p0, cnt) for _, p0, cnt in work)
        return orig(work)

    srv.tick = spy
    srv.run([req], realtime=False)
    srv.close()
    assert len(seen) == 3 and sum(c for _, c in seen) == 1920 * 1080
    ends = [p for p0, c in seen for p in (p0, p0 + c - 1)]
    idx = np.concatenate([np.random.default_rng(5).integers(0, 1920 * 1080, 400), ends])
    _check_pixels_against_oracle(room, 3, req.cam, idx, 1920, req.out, "1920x1080 over 3 ticks")


def test_forward_slots_direct_matches_oracle(resident):
    """sg_render_forward_slots called through the C ABI on a table of three
    slots (two requests, one split in two) on the room grid, against the
    oracle at sampled pixels and the ends of each slot."""
    import ctypes
    from paper_2305_13220_amd._lib import check, lib, ptr, stream_ptr
    from paper_2305_13220_amd.grid import RenderParams
    from paper_2305_13220_amd.serve import SLOT_DTYPE, alloc_outputs
    from synth import workloads
    grids, poses = resident
    g, vox, prm = grids[1]
    room = workloads.room_2cm(n_rays=1024)
    cams = [np.array(poses[1][i], np.float32).copy() for i in (0, 3)]
    sizes = [(320, 240), (200, 150)]
    for c, (W, H) in zip(cams, sizes):
        f = (W / 2) / np.tan(np.deg2rad(30.0))
        c[:4] = (f, f, W / 2, H / 2)
    outs = [alloc_outputs(W * H, 3, g.device) for W, H in sizes]
    split = 30_001
    table = [(0, 0, split), (1, 0, sizes[1][0] * sizes[1][1]), (0, split, 320 * 240 - split)]
    slots = np.zeros(len(table), dtype=SLOT_DTYPE)
    base = 0
    for i, (q, p0, cnt) in enumerate(table):
        o = outs[q]
        slots[i] = (1, sizes[q][0], p0, cnt, base, cams[q], o["feat"].data_ptr(),
                    o["depth"].data_ptr(), o["normal"].data_ptr(), o["wsum"].data_ptr(),
                    o["nsamples"].data_ptr())
        base += cnt
    d_slots = torch.from_numpy(slots.view(np.uint8).copy()).to(g.device)
    d_n = torch.tensor([len(table)], dtype=torch.int32, device=g.device)
    pc = RenderParams.of(prm).c()
    check(lib().sg_render_forward_slots(g.handle, ptr(vox), 3, ctypes.byref(pc), ptr(d_slots),
                                        ptr(d_n), 8, base, stream_ptr(g.device)),
          "sg_render_forward_slots")
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    for q, (W, H) in enumerate(sizes):
        ends = [p for qq, p0, cnt in table if qq == q for p in (p0, p0 + cnt - 1)]
        idx = np.concatenate([rng.integers(0, W * H, 300), ends])
        _check_pixels_against_oracle(room, 3, cams[q], idx, W, outs[q], f"slots request {q}")


def test_extend_makes_descriptors_stale():
    """sg_grid_extend moves the grid's memory: a descriptor made before it is
    reported stale, one made after it is current, and a server holding the
    grid refuses the extend until it is closed."""
    import ctypes
    import paper_2305_13220_amd as sg
    from paper_2305_13220_amd._lib import RenderParamsC, lib
    from paper_2305_13220_amd.serve import PackedServer
    coords = to_dev(np.array([[0, 0, 0], [1, 0, 0]], np.int32))
    g = sg.Grid(coords, 0.02)
    vox = torch.zeros((2, 512, 4), device=coords.device)
    p = RenderParamsC(0.01, 0.0, 2.0, 0.02, 64)
    d0 = (ctypes.c_ubyte * 512)()
    assert lib().sg_packed_grid_desc(g.handle, ctypes.c_void_p(vox.data_ptr()), 3,
                                     ctypes.byref(p), d0) == 0
    assert lib().sg_packed_grid_check(g.handle, d0) == 0
    assert g.generation == 0
    srv = PackedServer([(g, vox, {"step": 0.01, "t_near": 0.0, "t_far": 2.0, "beta": 0.02,
                                  "max_samples": 64})], C=3)
    with pytest.raises(sg.SgridError, match="pinned"):
        g.extend(to_dev(np.array([[2, 0, 0]], np.int32)))
    srv.close()
    assert g.extend(to_dev(np.array([[2, 0, 0]], np.int32))) == 3
    assert g.generation == 1
    assert lib().sg_packed_grid_check(g.handle, d0) == -5
    assert "extend" in lib().sg_last_error().decode()
    d1 = (ctypes.c_ubyte * 512)()
    assert lib().sg_packed_grid_desc(g.handle, ctypes.c_void_p(vox.data_ptr()), 3,
                                     ctypes.byref(p), d1) == 0
    assert lib().sg_packed_grid_check(g.handle, d1) == 0
    g.destroy()
