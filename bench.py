"""Benchmark: forward + backward rays/s of the sparse-dense SDF renderer.

Headline workload (one GPU): differentiation at scale on the 6 x 6 x 3 m
synthetic room at 2 cm voxels (11,542 allocated 8^3 blocks, SDF + RGB) with
seeded noise on the voxels (0.5 voxel on SDF, 0.1 on RGB), batches of
2^18 random pixels from 30 seeded 640x480 poses, step 1 cm, t in [0, 12] m,
beta = 2 cm, at most 128 samples per ray, against renders of the clean grid.
One step = camera rays for the batch, gradient zeroing, and the fused
training kernel: block march, forward render (colour, depth, normal),
squared-L2 losses (colour + 0.1 depth + 0.05 normal), and the backward
scatter into the voxels.  Adam over every voxel parameter is timed on its
own; the same step built from separate calls (one march shared by forward
and backward, loss gradient, backward) is timed too.  Inputs are resident on
the GPU before timing starts.  Extra objects repeat the step on the
65,536-ray room batch (with the Eikonal term too) and on the 64x48 sphere.

Prints one JSON line.  `roofline` is for the dominant kernel (the fused
training kernel), timed with HIP events around each launch on the stream it
runs on; its algorithmic bytes are the forward plus backward bytes from
exact per-ray footprint counts (samples, distinct voxels, distinct blocks)
of the timed batch.  `cpu_baseline` times the CPU oracle on bounded samples
of the same workloads on the host, single-threaded and on all usable cores.

`serving` measures render serving over three resident grids (the room at
2 cm, the same room at 1 cm, a second room at 2 cm; C = 3): seeded Poisson
arrivals of full-frame requests (320x240, 640x480, 1296x968 or 1920x1080,
uniform), at 0.5x, 0.8x and 1.2x of the plain path's measured capacity,
served (i) by the plain path, one rays + forward call per request in
arrival order, and (ii) by packed multi-grid launches replayed from a HIP
graph with an 8 GiB budget for in-flight outputs, ticks of 2^20 pixels
filled shortest-remaining-request first (with aging).  The same is repeated
for a mix of small requests only (320x240 and 640x480), where per-call
launches weigh more.  Latency = GPU completion
time - arrival time; p50 / p99 over the requests of each point.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd rays/s, % HBM roofline; render p50/p99 ms vs plain per-call path"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(counts, C):
    """Per-launch algorithmic bytes from exact per-ray (S, U, K) counts.

    Per ray: 24 B of ray, 16 B per distinct block (hash entry), V = 4(1+C)
    bytes per distinct voxel read, the same per distinct voxel whose gradient
    is accumulated, O = 4(C+5) bytes of outputs, O-4 bytes of upstream
    gradients or reference values.  Forward: 24 + 16K + VU + O.  Separate
    backward (recomputes the forward): 24 + 16K + 2VU + O + (O-4).  Fused
    training step: 24 + 16K + 2VU + O (outputs written) + (O-4) (references).
    """
    import numpy as np
    c = counts.astype(np.int64)
    K = c[:, 2].sum()
    U = c[:, 1].sum()
    R = c.shape[0]
    V = 4 * (1 + C)
    O = 4 * (C + 1 + 3 + 1)
    fwd = R * 24 + 16 * K + V * U + R * O
    bwd = R * 24 + 16 * K + 2 * V * U + R * O + R * (O - 4)
    fused = R * 24 + 16 * K + 2 * V * U + R * O + R * (O - 4)
    return int(fwd), int(bwd), int(fused)


def source_hash():
    h = hashlib.sha256()
    for f in ("common.h", "render.hip"):
        h.update(open(os.path.join(ROOT, "paper_2305_13220_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, if current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d[workload][kernel]
        if e.get("source_hash") != source_hash():
            return None
        return e["bytes_per_launch"]
    except Exception:
        return None


def _cpu_info():
    import platform
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def _oracle_fwd_bwd(w, vox64, rays, threads, C=3):
    """Oracle forward, squared-L2 loss gradient and backward over `rays`, the
    rays split into `threads` contiguous shards rendered by a thread pool
    (ctypes releases the interpreter lock, so the shards run in parallel);
    the loss gradient is taken over the whole batch and the per-shard voxel
    gradients are summed.  The loss target is zero: the oracle takes no input
    from the GPU path, and the work does not depend on the target values."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import oracle
    R = rays.shape[0]
    cuts = np.linspace(0, R, threads + 1).astype(int)
    shards = [(cuts[i], cuts[i + 1]) for i in range(threads) if cuts[i + 1] > cuts[i]]
    args = (w["block_coords"], vox64, C, w["h"], w["origin"])
    with ThreadPoolExecutor(len(shards)) as ex:
        outs = list(ex.map(lambda ab: oracle.render_forward(*args, rays[ab[0]:ab[1]], w["params"]),
                           shards))
        feat = np.concatenate([o["feat"] for o in outs])
        depth = np.concatenate([o["depth"] for o in outs])
        normal = np.concatenate([o["normal"] for o in outs])
        _, gc, gd, gn = oracle.l2_loss_grad(feat, np.zeros_like(feat), depth, np.zeros_like(depth),
                                            normal, np.zeros_like(normal), 0.1, 0.05)
        grads = list(ex.map(lambda ab: oracle.render_backward(
            *args, rays[ab[0]:ab[1]], w["params"], gc[ab[0]:ab[1]], gd[ab[0]:ab[1]],
            gn[ab[0]:ab[1]], None), shards))
    total = grads[0]
    for g in grads[1:]:
        total += g
    return total


def _oracle_fwd(w, vox64, rays, threads, C):
    """Oracle forward over `rays` in `threads` shards (thread pool)."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import oracle
    R = rays.shape[0]
    cuts = np.linspace(0, R, threads + 1).astype(int)
    shards = [(cuts[i], cuts[i + 1]) for i in range(threads) if cuts[i + 1] > cuts[i]]
    with ThreadPoolExecutor(len(shards)) as ex:
        list(ex.map(lambda ab: oracle.render_forward(w["block_coords"], vox64, C, w["h"],
                                                     w["origin"], rays[ab[0]:ab[1]], w["params"]),
                    shards))


def _timed(fn, min_seconds, max_passes):
    done, dt = 0, 0.0
    while done < max_passes and (done == 0 or dt < min_seconds):
        t0 = time.perf_counter()
        fn()
        dt += time.perf_counter() - t0
        done += 1
    return done, dt


def cpu_baseline(w4, w2, w1, n_rays=65536, frames=True):
    """The oracle on the host cores, one thread and all usable cores, on
    bounded samples (rays/s of each leg):
      * the differentiation-at-scale batch (noisy 2 cm room): forward + loss
        gradient + backward on its first n_rays rays (the headline leg);
      * the 65,536-ray 2 cm room batch, the same work;
      * the 64x48 sphere frame, the same work, all 3,072 rays;
      * frame 0 of the 1 cm semantic room (C = 19), forward only, all
        1,254,528 rays with all cores, its first n_rays rays with one.
    Each leg repeats until it has run for a few seconds (at most 3 passes)."""
    import numpy as np
    info = _cpu_info()
    n_all = info["affinity"] or info["nproc"] or 1
    legs = {}

    def leg(name, w, rays, threads, fwd_only=False, C=3, min_s=3.0):
        vox64 = np.ascontiguousarray(w["vox"], np.float64)
        if fwd_only:
            fn = lambda: _oracle_fwd(w, vox64, rays, threads, C)
        else:
            fn = lambda: _oracle_fwd_bwd(w, vox64, rays, threads, C)
        done, dt = _timed(fn, min_s, 3)
        r = {"threads": threads, "rays": int(rays.shape[0]), "passes": done,
             "seconds": round(dt, 2), "rays_per_s": round(done * rays.shape[0] / dt, 1)}
        legs.setdefault(name, []).append(r)
        log(f"oracle {name} threads={threads}: {r['rays_per_s']:.0f} rays/s ({dt:.1f} s)")
        return r

    r4 = w4["rays"][:n_rays]
    one = leg("noisy_room_2cm_fwd_bwd", w4, r4, 1, min_s=6.0)
    full = leg("noisy_room_2cm_fwd_bwd", w4, r4, n_all, min_s=6.0)
    r2 = w2["rays"][:n_rays]
    leg("room_2cm_65536_fwd_bwd", w2, r2, 1)
    leg("room_2cm_65536_fwd_bwd", w2, r2, n_all)
    leg("sphere_64x48_fwd_bwd", w1, w1["rays"], 1, min_s=1.0)
    leg("sphere_64x48_fwd_bwd", w1, w1["rays"], n_all, min_s=1.0)
    if frames:
        from synth import cameras, workloads
        w3 = workloads.room_1cm_sem(n_cams=50)
        r3 = cameras.pixel_rays(w3["cams"], cameras.frame_pixels(0, w3["W"], w3["H"]))
        C3 = w3["vox"].shape[-1] - 1
        leg("room_1cm_sem_frame0_fwd", w3, r3[:n_rays], 1, fwd_only=True, C=C3, min_s=1.0)
        leg("room_1cm_sem_frame0_fwd", w3, r3, n_all, fwd_only=True, C=C3, min_s=1.0)
    return {"value": full["rays_per_s"], "unit": "rays/s", "cores": n_all, "kind": "oracle",
            "sample": f"forward + loss gradient + backward on the first {n_rays} rays of the "
                      f"2^18-ray noisy-room batch, {n_all} threads over ray shards "
                      f"({full['passes']} pass(es), {full['seconds']} s); single thread "
                      f"{one['rays_per_s']} rays/s",
            "value_1_thread": one["rays_per_s"], **info, "legs": legs}


RESOLUTIONS = ((320, 240), (640, 480), (1296, 968), (1920, 1080))
SMALL_RESOLUTIONS = ((320, 240), (640, 480))


def serve_bench(args, dev):
    import numpy as np  # noqa: F401
    import torch

    import paper_2305_13220_amd as sg
    from paper_2305_13220_amd.serve import (PackedServer, PlainServer, latency_stats,
                                            poisson_requests)
    from synth import scenes, workloads
    t0 = time.perf_counter()
    grids, poses, blocks = [], [], []
    for sc, prm, cams in workloads.serving_grids():
        g = sg.Grid(torch.from_numpy(sc["block_coords"]).to(dev), float(sc["h"]),
                    tuple(float(x) for x in sc["origin"]))
        grids.append((g, torch.from_numpy(sc["vox"]).to(dev), prm))
        poses.append(list(cams))
        blocks.append(g.n_blocks)
    log(f"serving setup {time.perf_counter() - t0:.1f}s: blocks {blocks}")
    plain = PlainServer(grids, 3, keep_outputs=False)
    packed = PackedServer(grids, 3, hbm_budget_bytes=int(args.serve_budget_gib * (1 << 30)),
                          keep_outputs=False)

    def scenario(name, res, sub):
        def reqs(n, qps, k):
            return poisson_requests(n, qps, len(grids), poses, res,
                                    seed=[0, scenes.SEED_ARRIVALS, sub, k])

        plain.run(reqs(16, 1e9, 1), realtime=False)  # warm-up: code, allocator, graphs
        packed.run(reqs(16, 1e9, 1), realtime=False)

        def capacity(server, n):
            r = reqs(n, 1e9, 2)
            server.run(r, realtime=False)
            span = max(q.done for q in r) - min(q.arrival for q in r)
            return n / span, latency_stats(r)["rays_per_s"]

        n_cal = max(16, args.serve_requests // 5)
        cap_plain, rays_plain = capacity(plain, n_cal)
        cap_packed, rays_packed = capacity(packed, n_cal)
        log(f"{name}: capacity plain {cap_plain:.1f} req/s, packed {cap_packed:.1f} req/s")
        points = []
        for k, load in enumerate((0.5, 0.8, 1.2)):
            qps = load * cap_plain
            a = reqs(args.serve_requests, qps, 10 + k)
            plain.run(a, realtime=True)
            b = reqs(args.serve_requests, qps, 10 + k)
            packed.run(b, realtime=True)
            pt = {"load": load, "qps": round(qps, 2),
                  "plain": {kk: round(v, 3) if isinstance(v, float) else v
                            for kk, v in latency_stats(a).items()},
                  "packed": {kk: round(v, 3) if isinstance(v, float) else v
                             for kk, v in latency_stats(b).items()}}
            log(f"{name} load {load}: plain p50/p99 {pt['plain']['p50_ms']}/"
                f"{pt['plain']['p99_ms']} ms, packed {pt['packed']['p50_ms']}/"
                f"{pt['packed']['p99_ms']} ms")
            points.append(pt)
        head = points[1]
        return {"resolutions": [f"{w}x{h}" for w, h in res],
                "requests_per_point": args.serve_requests,
                "capacity_req_per_s": {"plain": round(cap_plain, 2), "packed": round(cap_packed, 2)},
                "capacity_rays_per_s": {"plain": rays_plain, "packed": rays_packed},
                "p50_ms_at_0.8": {"plain": head["plain"]["p50_ms"],
                                  "packed": head["packed"]["p50_ms"]},
                "p99_ms_at_0.8": {"plain": head["plain"]["p99_ms"],
                                  "packed": head["packed"]["p99_ms"]},
                "points": points}

    out = {"grids": "room 2 cm, room 1 cm, second room 2 cm (C=3)", "blocks": blocks,
           "packed": {"tick_rays": packed.tick_rays, "order": packed.order,
                      "launch": packed.launch_mode, "hbm_budget_gib": args.serve_budget_gib}}
    out["full_mix"] = scenario("full mix", RESOLUTIONS, 0)
    out["small_mix"] = scenario("small mix", SMALL_RESOLUTIONS, 1)
    return out


def frames_bench(dev, n_frames=50):
    """Full-frame forward renders of the 1 cm room with 16 semantic logits
    (C = 19) at 1296x968 along a seeded 50-pose trajectory: camera rays and
    the forward render per frame, timed frame by frame with HIP events."""
    import numpy as np
    import torch
    import paper_2305_13220_amd as sg
    from synth import workloads
    t0 = time.perf_counter()
    w = workloads.room_1cm_sem(n_cams=n_frames)
    C = w["vox"].shape[-1] - 1
    W, H = w["W"], w["H"]
    grid = sg.Grid(torch.from_numpy(w["block_coords"]).to(dev), float(w["h"]),
                   tuple(float(x) for x in w["origin"]))
    vox = torch.from_numpy(w["vox"]).to(dev)
    cams = torch.from_numpy(w["cams"]).to(dev)
    params = sg.RenderParams.of(w["params"])
    R = W * H
    vv, uu = torch.meshgrid(torch.arange(H, device=dev, dtype=torch.int32),
                            torch.arange(W, device=dev, dtype=torch.int32), indexing="ij")
    pix = [torch.stack([torch.full_like(uu, i).reshape(-1), uu.reshape(-1), vv.reshape(-1)],
                       1).contiguous() for i in range(n_frames)]
    out = {"feat": torch.empty((R, C), device=dev), "depth": torch.empty(R, device=dev),
           "normal": torch.empty((R, 3), device=dev), "wsum": torch.empty(R, device=dev),
           "nsamples": torch.empty(R, dtype=torch.int32, device=dev)}
    rays = sg.rays_pinhole(cams, pix[0])
    fb, S = 0, 0
    for i in range(n_frames):
        rays = sg.rays_pinhole(cams, pix[i])
        c = sg.render_footprint(grid, rays, params).cpu().numpy()
        fb += algorithmic_bytes(c, C)[0]
        S += int(c[:, 0].astype(np.int64).sum())
    log(f"frames setup {time.perf_counter() - t0:.1f}s: {grid.n_blocks} blocks, C={C}")
    for _ in range(3):
        sg.render_forward(grid, vox, sg.rays_pinhole(cams, pix[0]), params, out=out)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(n_frames)]
    for i in range(n_frames):
        ev[i][0].record()
        rays = sg.rays_pinhole(cams, pix[i])
        ev[i][1].record()
        sg.render_forward(grid, vox, rays, params, out=out)
        ev[i][2].record()
    torch.cuda.synchronize()
    frame_ms = np.array([e[0].elapsed_time(e[2]) for e in ev])
    fwd_ms = np.array([e[1].elapsed_time(e[2]) for e in ev])
    total = float(frame_ms.sum())
    ach = fb / (fwd_ms.sum() * 1e-3) / 1e9
    res = {"workload": "room_1cm_sem_1296x968_50_frames",
           "scene": "room at h = 1 cm, 16 semantic logits + RGB (C = 19)",
           "blocks": grid.n_blocks, "frames": n_frames, "rays_per_frame": R,
           "frames_per_s": round(n_frames / (total * 1e-3), 2),
           "rays_per_s": n_frames * R / (total * 1e-3), "samples_per_s": S / (total * 1e-3),
           "ms_per_frame_p50": round(float(np.median(frame_ms)), 4),
           "ms_per_frame_p99": round(float(np.percentile(frame_ms, 99)), 4),
           "forward_kernel_ms_mean": round(float(fwd_ms.mean()), 4),
           "mean_samples_per_ray": S / (n_frames * R),
           "roofline_forward": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                                "kernel": "k_render_fwd<19, false>",
                                "algorithmic_bytes_per_frame": fb // n_frames}}
    del vox, grid, out, pix
    torch.cuda.empty_cache()
    return res


def fusion_bench(dev, n_frames=10, dilate=2, reps=5, n_sem=16):
    """Block allocation from depth maps, grid build and fusion of ten seeded
    640x480 depth + RGB + 16 semantic-logit frames of the 2 cm room (Sec.
    3.4): the set-up of the grid that the render then refines.  Dilation
    radius R = 2 blocks and truncation mu = 8 h R, the supplement's values."""
    import numpy as np
    import torch
    import paper_2305_13220_amd as sg
    from synth import workloads
    t0 = time.perf_counter()
    fr = workloads.room_depth_frames(n_frames=n_frames, W=640, H=480, n_sem=n_sem)
    cams, depth, feat = (torch.from_numpy(fr[k]).to(dev) for k in ("cams", "depth", "feat"))
    log(f"fusion setup {time.perf_counter() - t0:.1f}s")
    h = float(fr["h"])
    trunc = 8 * h * dilate
    blocks = sg.alloc_blocks(cams, depth, h, dilate=dilate)
    grid = sg.Grid(blocks, h)
    vox, wt = sg.fuse(grid, cams, depth, feat, trunc, n_sem=n_sem)
    torch.cuda.synchronize()
    t_alloc, t_build, t_fuse = [], [], []
    for _ in range(reps):
        a = time.perf_counter()
        blocks = sg.alloc_blocks(cams, depth, h, dilate=dilate)
        torch.cuda.synchronize()
        b = time.perf_counter()
        grid = sg.Grid(blocks, h)
        torch.cuda.synchronize()
        c = time.perf_counter()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        sg.fuse(grid, cams, depth, feat, trunc, n_sem=n_sem, vox=vox, weight=False)
        e[1].record()
        torch.cuda.synchronize()
        t_alloc.append(b - a)
        t_build.append(c - b)
        t_fuse.append(e[0].elapsed_time(e[1]) * 1e-3)
    t_fd = []
    for _ in range(reps):
        a = time.perf_counter()
        sg.Grid.from_depth(cams, depth, h, dilate=dilate)
        torch.cuda.synchronize()
        t_fd.append(time.perf_counter() - a)
    n_vox = grid.n_blocks * 512
    fuse_s = float(np.median(t_fuse))
    total = float(np.median(t_alloc)) + float(np.median(t_build)) + fuse_s
    # de-noising of the fused grid (radius 1, sigma 1 voxel)
    dn = torch.empty_like(vox)
    sg.denoise(grid, vox, 1, 1.0, out=dn)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e[0].record()
    for _ in range(reps):
        sg.denoise(grid, vox, 1, 1.0, out=dn)
    e[1].record()
    torch.cuda.synchronize()
    dn_ms = e[0].elapsed_time(e[1]) / reps
    dn_bytes = 2 * vox.numel() * 4  # each voxel read once and written once
    res = {"workload": "room_2cm_fusion_10x640x480", "frames": n_frames, "blocks": grid.n_blocks,
           "dilate": dilate, "trunc_m": round(trunc, 4),
           "denoise_ms": round(dn_ms, 4),
           "denoise_hbm_frac": round(dn_bytes / (dn_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "alloc_ms": round(float(np.median(t_alloc)) * 1e3, 3),
           "build_ms": round(float(np.median(t_build)) * 1e3, 3),
           "grid_from_depth_ms": round(float(np.median(t_fd)) * 1e3, 3),
           "fuse_ms": round(fuse_s * 1e3, 3),
           "fuse_voxel_frames_per_s": n_vox * n_frames / fuse_s,
           "frames_per_s_end_to_end": round(n_frames / total, 1),
           "associated_frac": round(float((wt > 0).float().mean().item()), 4),
           "kernel": "k_fuse<19>", "C": 3 + n_sem}
    del vox, wt, grid, cams, depth, feat, dn
    torch.cuda.empty_cache()
    return res


# Widths of the CRF's Gaussian kernels (features are divided by them): the
# supplement fixes sigma_color = 0.1 and sigma_sdf = 1.0 (taken here for the
# SDF-gradient, that is normal, features); the position and label-logit
# widths are readings (5 cm, 2.5 voxels of the 2 cm grid; 1.0).
CRF_SIGMA = {"pos": 0.05, "color": 0.1, "normal": 1.0, "label": 1.0}
# Loss weights of the supplement's hyper-parameters.
CRF_LAMBDA = {"color": 1e-3, "label": 0.1, "normal": 1.0}


def crf_bench(dev, n_rays=1 << 18, n_sem=16, iters=5, reps=5, w_potts=1.0):
    """The continuous CRF of Sec. 3.5.3 on the 2 cm room with 16 semantic
    logits per voxel (C = 19), as one training chain:

      nodes      zero crossings of the SDF along 2^18 rays from the room's 30
                 seeded poses (sg_surface_points), the rays that hit;
      features   sg_query at the nodes: position, RGB, grad f (the normal),
                 16 label logits;
      label      lattice over (position, RGB, normal) (d = 9), mean field of
                 5 updates from the logits (unary -logits, Potts
                 compatibility), KL label loss, lambda_label = 0.1;
      colour     lattice over (position, normal, logits) (d = 22), RGB
                 filtered and normalised, property loss, lambda_color = 1e-3;
      normal     lattice over (position, RGB, logits) (d = 22), the normal
                 filtered and normalised, property loss, lambda_normal = 1;
      adjoint    the three losses' gradients (logits, RGB, grad f) into the
                 voxels through sg_query_backward.

    Feature scaling and concatenation are torch glue; every step of the
    method is a library call.  The chain is timed on the host around
    synchronisations (the lattice builds synchronise); the filters, mean
    fields and the mean-field gradient (workspace allocated beforehand) are
    also timed with events."""
    import numpy as np
    import torch
    import paper_2305_13220_amd as sg
    from synth import workloads
    t0 = time.perf_counter()
    base = workloads.room_2cm(n_rays=n_rays)
    sem = workloads._room(0, 0.02, n_sem)
    C = 3 + n_sem
    grid = sg.Grid(torch.from_numpy(sem["block_coords"]).to(dev), float(sem["h"]),
                   tuple(float(x) for x in sem["origin"]))
    vox = torch.from_numpy(sem["vox"]).to(dev)
    rays = sg.rays_pinhole(torch.from_numpy(base["cams"]).to(dev),
                           torch.from_numpy(base["pix"]).to(dev))
    params = base["params"]
    log(f"crf setup {time.perf_counter() - t0:.1f}s: {grid.n_blocks} blocks, C={C}")
    sp, sc, sn, sl = (CRF_SIGMA[k] for k in ("pos", "color", "normal", "label"))
    mu = (w_potts * (1.0 - torch.eye(n_sem, device=dev))).contiguous()

    def chain(stats=None):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        pts, hit = sg.surface_points(grid, vox, rays, params)
        idx = torch.nonzero(hit, as_tuple=False).squeeze(1)
        nodes = pts.index_select(0, idx).contiguous()
        q = sg.query(grid, vox, nodes)
        rgb, logit, nrm = q["feat"][:, :3], q["feat"][:, 3:], q["grad"]
        f_lab = torch.cat([nodes / sp, rgb / sc, nrm / sn], 1).contiguous()
        f_col = torch.cat([nodes / sp, nrm / sn, logit / sl], 1).contiguous()
        f_nrm = torch.cat([nodes / sp, rgb / sc, logit / sl], 1).contiguous()
        ones = torch.ones((nodes.shape[0], 1), device=dev)
        lat_l = sg.Lattice(f_lab, max_values=n_sem)
        lat_c = sg.Lattice(f_col, max_values=4)
        lat_n = sg.Lattice(f_nrm, max_values=4)
        g_feat = torch.zeros_like(q["feat"])
        ev[0].record()
        Q = lat_l.meanfield((-logit).contiguous(), 0.0, iters, compat=mu)
        l_lab, _ = sg.crf_label_loss(q["feat"], Q, col0=3, weight=CRF_LAMBDA["label"], g_feat=g_feat)
        fc = lat_c.filter(torch.cat([rgb, ones], 1).contiguous())
        l_col, _ = sg.crf_property_loss(q["feat"], fc, col0=0, weight=CRF_LAMBDA["color"],
                                        g_feat=g_feat)
        fn = lat_n.filter(torch.cat([nrm, ones], 1).contiguous())
        l_nrm, g_nrm = sg.crf_property_loss(nrm.contiguous(), fn, col0=0,
                                            weight=CRF_LAMBDA["normal"])
        grad = sg.query_backward(grid, vox.shape, nodes, g_grad=g_nrm, g_feat=g_feat)
        ev[1].record()
        if stats is not None:
            torch.cuda.synchronize()
            stats.update(nodes=int(nodes.shape[0]), vertices={"label_d9": lat_l.n_vertices,
                                                               "color_d22": lat_c.n_vertices,
                                                               "normal_d22": lat_n.n_vertices},
                         loss={"label": float(l_lab.sum()), "color": float(l_col.sum()),
                               "normal": float(l_nrm.sum())},
                         after_builds_ms=ev[0].elapsed_time(ev[1]),
                         lat=(lat_l, lat_c, lat_n), Q=Q, logit=logit.contiguous(), rgb=rgb, nrm=nrm,
                         f_lab=f_lab, f_col=f_col, f_nrm=f_nrm)
        return grad

    chain()
    torch.cuda.synchronize()
    tc = []
    for _ in range(reps):
        a = time.perf_counter()
        chain()
        torch.cuda.synchronize()
        tc.append(time.perf_counter() - a)
    st = {}
    chain(st)
    lat_l, lat_c, lat_n = st.pop("lat")
    Q, logit = st.pop("Q"), st.pop("logit")
    n = st["nodes"]
    ones = torch.ones((n, 1), device=dev)
    v4 = torch.cat([st.pop("rgb"), ones], 1).contiguous()
    st.pop("nrm")
    # kernels on their own, with events
    ws = torch.empty(sg._lib.lib().sg_crf_meanfield_compat_backward_ws_bytes(n, n_sem, iters),
                     dtype=torch.uint8, device=dev)
    gQ = torch.from_numpy(np.random.default_rng(0).normal(size=(n, n_sem)).astype(np.float32)).to(dev)
    g_u = torch.empty((n, n_sem), device=dev)
    g_mu = torch.empty((n_sem, n_sem), device=dev)
    out16 = torch.empty((n, n_sem), device=dev)
    out4 = torch.empty((n, 4), device=dev)
    unary = (-logit).contiguous()
    L = sg._lib.lib()

    def mf_bwd():
        sg._lib.check(L.sg_crf_meanfield_compat_backward(
            lat_l._h, sg._lib.ptr(unary), n_sem, sg._lib.ptr(mu), iters, sg._lib.ptr(gQ),
            sg._lib.ptr(g_u), sg._lib.ptr(g_mu), sg._lib.ptr(ws), ws.numel(),
            sg._lib.stream_ptr(dev)), "sg_crf_meanfield_compat_backward")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        for _ in range(reps):
            fn()
        e[1].record()
        torch.cuda.synchronize()
        return e[0].elapsed_time(e[1]) / reps

    f16_ms = timed(lambda: lat_l.filter(Q, out=out16))
    f4_ms = timed(lambda: lat_c.filter(v4, out=out4))
    mf_ms = timed(lambda: lat_l.meanfield(unary, 0.0, iters, out=out16, compat=mu))
    mfb_ms = timed(mf_bwd)
    f_lab, f_col = st.pop("f_lab"), st.pop("f_col")
    st.pop("f_nrm")
    tb9, tb22 = [], []
    for _ in range(reps):
        a = time.perf_counter()
        sg.Lattice(f_lab, max_values=n_sem)
        tb9.append(time.perf_counter() - a)
        a = time.perf_counter()
        sg.Lattice(f_col, max_values=4)
        tb22.append(time.perf_counter() - a)

    def filt_bytes(lat, d, vd):
        # splat: (vid, weight) per point-vertex pair, the point's values,
        # one value row update per pair; blur: per vertex and direction its
        # list entry and two neighbour slots, three value rows read, one
        # written; slice: the pairs again, the values out
        nv = lat.n_vertices
        pairs = n * (d + 1)
        return (pairs * (8 + 4 * vd) + 4 * n * vd + (d + 1) * nv * (12 + 16 * vd)
                + pairs * (8 + 4 * vd) + 4 * n * vd)

    b16 = filt_bytes(lat_l, 9, n_sem)
    b4 = filt_bytes(lat_c, 22, 4)
    res = {"workload": "room_2cm_sem_surface_nodes_2^18_rays", "C": C, "rays": n_rays,
           "sigma": CRF_SIGMA, "lambda": CRF_LAMBDA, "potts_weight": w_potts,
           "chain_ms_p50": round(float(np.median(tc)) * 1e3, 3),
           "chain_after_lattice_builds_ms": round(st.pop("after_builds_ms"), 4),
           "build_d9_ms": round(float(np.median(tb9)) * 1e3, 3),
           "build_d22_ms": round(float(np.median(tb22)) * 1e3, 3),
           "filter_d9_16ch_ms": round(f16_ms, 4), "filter_d22_4ch_ms": round(f4_ms, 4),
           "meanfield_d9_ms": round(mf_ms, 4), "meanfield_iters": iters,
           "meanfield_backward_d9_ms": round(mfb_ms, 4),
           "filter_d9_16ch_hbm_frac": round(b16 / (f16_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "filter_d22_4ch_hbm_frac": round(b4 / (f4_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "filter_bytes_definition": "splat (vid, weight, values, row update per point-vertex "
                                      "pair), blur (list entry, two neighbour slots, three value "
                                      "rows read and one written per vertex and direction), slice",
           **st}
    del lat_l, lat_c, lat_n, ws, gQ, Q, grid, vox, rays, f_lab, f_col
    torch.cuda.empty_cache()
    return res


def query_bench(grid, vox, block_coords, dev, ks=(16, 32, 64, 128, 256, 512)):
    """SDF and gradient at the k^3 lattice points of the grid's bounding box
    (the point-query timing of Sec. 4), one sg_query call per k.  Bytes per
    point: 12 in, 4 + 4 + 12 out (valid, f, grad); the voxel reads are left
    out, so the bandwidth figure is a lower bound."""
    import torch
    import paper_2305_13220_amd as sg
    h = grid.voxel_size
    bmin, bmax = block_coords.min(0), block_coords.max(0)
    lo = [grid.origin[a] + 8 * h * float(bmin[a]) for a in range(3)]
    hi = [grid.origin[a] + 8 * h * float(bmax[a] + 1) for a in range(3)]
    rows = []
    for k in ks:
        ax = [torch.linspace(lo[a], hi[a], k, device=dev) for a in range(3)]
        zz, yy, xx = torch.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        pts = torch.stack([xx.reshape(-1), yy.reshape(-1), zz.reshape(-1)], 1).contiguous()
        del xx, yy, zz
        m = pts.shape[0]
        out = sg.query(grid, vox, pts, features=False)
        torch.cuda.synchronize()
        reps = max(3, min(200, int(2e8 // m)))
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        for _ in range(reps):
            sg.query(grid, vox, pts, features=False, out=out)
        e[1].record()
        torch.cuda.synchronize()
        ms = e[0].elapsed_time(e[1]) / reps
        gbs = 32 * m / (ms * 1e-3) / 1e9
        row = {"k": k, "points": m, "ms": round(ms, 4),
               "points_per_s": round(m / (ms * 1e-3), 1),
               "valid_frac": round(out["valid"].float().mean().item(), 4),
               "GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        if k == 128:
            # Eikonal regulariser on the same points: loss per point and the
            # scatter of its gradient into the SDF voxels
            gv = torch.zeros_like(vox)
            sg.eikonal(grid, vox, pts, 0.1, grad_vox=gv)
            torch.cuda.synchronize()
            e[0].record()
            for _ in range(reps):
                sg.eikonal(grid, vox, pts, 0.1, grad_vox=gv)
            e[1].record()
            torch.cuda.synchronize()
            row["eikonal_ms"] = round(e[0].elapsed_time(e[1]) / reps, 4)
            del gv
        rows.append(row)
        del pts, out
    torch.cuda.empty_cache()
    return {"what": "SDF + gradient at k^3 lattice points of the grid's bounding box "
                    "(room 2 cm, C=3 voxels), one call", "kernel": "k_query<3>",
            "bytes_per_point": 32, "sizes": rows}


def fused_bench(dev, w, target_vox, steps, warmup, lambda_d=0.1, lambda_n=0.05, adam=False,
                separate=False, eikonal=False, cold=False):
    """The training step on one batch: camera rays for the batch's (pose,
    pixel) pairs, gradient zeroing, and the fused kernel (block march,
    forward render, squared-L2 losses against the target renders, backward
    scatter into the voxels).  The step is timed over `steps` steps after
    `warmup`, with HIP events on the stream every kernel runs on (torch's
    current stream), and the fused kernel on its own with events around
    each launch.  Algorithmic bytes come from exact per-ray footprint counts
    of the timed batch.  Optionally also: Adam over every voxel parameter
    (timed alone), the same step from separate calls (march, forward, loss
    gradient, backward), the step with the Eikonal term on the ray samples,
    and the fused kernel with cold caches."""
    import numpy as np
    import torch
    import paper_2305_13220_amd as sg
    C = w["vox"].shape[-1] - 1
    grid = sg.Grid(torch.from_numpy(w["block_coords"]).to(dev), float(w["h"]),
                   tuple(float(x) for x in w["origin"]))
    vox = torch.from_numpy(w["vox"]).to(dev)
    tvox = torch.from_numpy(target_vox).to(dev)
    cams = torch.from_numpy(w["cams"]).to(dev)
    pix = torch.from_numpy(w["pix"]).to(dev)
    params = sg.RenderParams.of(w["params"])
    R = pix.shape[0]
    rays = sg.rays_pinhole(cams, pix)
    target = {k: v.clone() for k, v in sg.render_forward(grid, tvox, rays, params).items()}
    del tvox
    grad = torch.zeros_like(vox)
    out = {"feat": torch.empty((R, C), device=dev), "depth": torch.empty(R, device=dev),
           "normal": torch.empty((R, 3), device=dev), "wsum": torch.empty(R, device=dev),
           "nsamples": torch.empty(R, dtype=torch.int32, device=dev)}
    torch.cuda.synchronize()

    def events(k):
        return [torch.cuda.Event(enable_timing=True) for _ in range(k)]

    fused_ev = []

    def step_fused(timed, lam_e=0.0):
        rr = sg.rays_pinhole(cams, pix)
        grad.zero_()
        e = events(2) if timed else None
        if timed:
            e[0].record()
        sg.render_l2_step(grid, vox, rr, params, target, lambda_d, lambda_n, grad_vox=grad,
                          out=out, lambda_e=lam_e)
        if timed:
            e[1].record()
            fused_ev.append(e)

    def run(step):
        for _ in range(warmup):
            step(False)
        torch.cuda.synchronize()
        start, end = events(2)
        start.record()
        for _ in range(steps):
            step(True)
        end.record()
        torch.cuda.synchronize()
        return start.elapsed_time(end) / steps

    ms = run(step_fused)
    fused_each = np.array([a.elapsed_time(b) for a, b in fused_ev])
    fused_ms = float(fused_each.mean())
    counts, touched = sg.render_footprint(grid, rays, params, touched=True)
    counts = counts.cpu().numpy()
    fb, bb, fused_b = algorithmic_bytes(counts, C)
    u_all = int(touched.sum().item())
    k_all = int(touched.view(-1, 512).any(dim=1).sum().item())
    comp_b = 2 * 4 * (1 + C) * u_all + 16 * k_all + R * (24 + 4 * (C + 5) + 4 * (C + 4))
    del touched
    S = int(counts[:, 0].astype(np.int64).sum())
    fb_bb = fb + bb
    res = {"rays_per_step": R, "ms_per_step": round(ms, 4), "rays_per_s": R / (ms * 1e-3),
           "samples_per_s": S / (ms * 1e-3), "mean_samples_per_ray": S / R,
           "mean_voxels_per_ray": float(counts[:, 1].astype(np.int64).sum()) / R,
           "mean_blocks_per_ray": float(counts[:, 2].astype(np.int64).sum()) / R,
           "fused_kernel_ms": round(fused_ms, 4),
           "fused_kernel_ms_p50": round(float(np.median(fused_each)), 4),
           "fused_kernel_ms_p90": round(float(np.percentile(fused_each, 90)), 4),
           "bytes_fwd_plus_bwd": fb_bb, "bytes_fused": fused_b, "bytes_fwd": fb,
           "bytes_compulsory": comp_b,
           "hbm_frac_fwd_plus_bwd": round(fb_bb / (fused_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "hbm_frac_fused_bytes": round(fused_b / (fused_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "hbm_frac_compulsory": round(comp_b / (fused_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if eikonal:
        res["ms_per_step_with_eikonal"] = round(run(lambda t: step_fused(t, 0.1)), 4)
    if separate:
        lists = torch.empty(sg.list_bytes(R, params), dtype=torch.uint8, device=dev)
        gout = {"feat": torch.empty((R, C), device=dev), "depth": torch.empty(R, device=dev),
                "normal": torch.empty((R, 3), device=dev)}
        sep_ev = []

        def step_separate(timed):
            rr = sg.rays_pinhole(cams, pix)
            e = events(5) if timed else None
            if timed:
                e[0].record()
            sg.march(grid, rr, params, out=lists)
            if timed:
                e[1].record()
            sg.render_forward(grid, vox, rr, params, out=out, lists=lists)
            if timed:
                e[2].record()
            sg.l2_loss_grad(out, target, lambda_d, lambda_n, out=gout)
            grad.zero_()
            if timed:
                e[3].record()
            sg.render_backward(grid, vox, rr, params, gout["feat"], gout["depth"],
                               gout["normal"], None, grad_vox=grad, lists=lists)
            if timed:
                e[4].record()
                sep_ev.append(e)

        ms_sep = run(step_separate)
        fwd_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in sep_ev]))
        bwd_ms = float(np.mean([e[3].elapsed_time(e[4]) for e in sep_ev]))
        res["separate_calls"] = {
            "ms_per_step": round(ms_sep, 4), "rays_per_s": R / (ms_sep * 1e-3),
            "march_ms": round(float(np.mean([e[0].elapsed_time(e[1]) for e in sep_ev])), 4),
            "forward_ms": round(fwd_ms, 4), "backward_ms": round(bwd_ms, 4),
            "forward_hbm_frac": round(fb / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "backward_hbm_frac": round(bb / (bwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        del lists, gout
    if cold:
        # cold caches: 1 GiB written between steps evicts L2 and the Infinity Cache
        flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        ev = []
        for _ in range(10):
            rr = sg.rays_pinhole(cams, pix)
            grad.zero_()
            flush.fill_(1.0)
            e = events(2)
            e[0].record()
            sg.render_l2_step(grid, vox, rr, params, target, lambda_d, lambda_n, grad_vox=grad,
                              out=out)
            e[1].record()
            ev.append(e)
        torch.cuda.synchronize()
        res["fused_kernel_ms_cold"] = round(float(np.median([a.elapsed_time(b) for a, b in ev])), 4)
        del flush
    if adam:
        m = torch.zeros_like(vox)
        v = torch.zeros_like(vox)
        for t in range(1, 4):
            sg.optim_step(0, vox, grad, m, v, 1e-3, 0.9, 0.999, 1e-8, t)
        torch.cuda.synchronize()
        e = events(2)
        e[0].record()
        for t in range(steps):
            sg.optim_step(0, vox, grad, m, v, 1e-3, 0.9, 0.999, 1e-8, 4 + t)
        e[1].record()
        torch.cuda.synchronize()
        adam_ms = e[0].elapsed_time(e[1]) / steps
        res["adam_ms"] = round(adam_ms, 4)
        res["adam_hbm_frac"] = round(7 * vox.numel() * 4 / (adam_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        res["ms_per_step_with_adam"] = round(ms + adam_ms, 4)
        res["params"] = int(vox.numel())
        del m, v
    res["_grid"] = (grid, vox)
    del grad, out, target
    return res


def copy_ceiling(dev):
    """Empirical HBM ceiling: device copy of 1 GiB (reads 1 GiB, writes 1 GiB)."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e[0].record()
    for _ in range(5):
        dst.copy_(src)
    e[1].record()
    torch.cuda.synchronize()
    gbs = 5 * 2 * (1 << 30) / (e[0].elapsed_time(e[1]) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--rays", type=int, default=1 << 18,
                    help="rays per step of the headline (noisy-room) workload")
    ap.add_argument("--cpu-rays", type=int, default=65536)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-query", action="store_true", help="skip the k^3 point-query timing")
    ap.add_argument("--no-crf", action="store_true", help="skip the CRF message-passing timing")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 65,536-ray room and the sphere training steps")
    ap.add_argument("--no-fusion", action="store_true",
                    help="skip the allocation + fusion timing")
    ap.add_argument("--no-frames", action="store_true",
                    help="skip the 1 cm semantic full-frame render timing")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests per arrival-rate point of the serving measurement")
    ap.add_argument("--serve-budget-gib", type=float, default=8.0)
    ap.add_argument("--calib-mib", type=int, default=0,
                    help="run one elementwise kernel over a tensor of this size first "
                         "(reads and writes it once: a reference for memory counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(rays are independent; a multi-GPU step would shard the batch and all-reduce the "
              "voxel gradients). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from synth import workloads

    dev = torch.device("cuda:0")
    if args.calib_mib > 0:
        a = torch.ones(args.calib_mib << 18, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b
    t_setup = time.perf_counter()
    w4 = workloads.room_2cm_noisy(n_rays=args.rays)
    log(f"setup {time.perf_counter() - t_setup:.1f}s: {w4['block_coords'].shape[0]} blocks, "
        f"{args.rays} rays")
    head = fused_bench(dev, w4, w4["clean_vox"], args.steps, args.warmup, adam=True,
                       separate=True, cold=True)
    grid4, vox4 = head.pop("_grid")
    log(f"headline: {head['ms_per_step']:.4f} ms/step, fused kernel {head['fused_kernel_ms']:.4f} "
        f"ms, frac {head['hbm_frac_fwd_plus_bwd']}")
    kname = "k_render_bwd<3, true, false>"
    fused_ms = head["fused_kernel_ms"]
    achieved = head["bytes_fwd_plus_bwd"] / (fused_ms * 1e-3) / 1e9
    copy_gbs = copy_ceiling(dev)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(kname, "noisy_room_2cm_262144"), "kernel": kname,
            "bytes_per_launch": head["bytes_fwd_plus_bwd"],
            "bytes_definition": "sum over rays of B_f + B_b (forward and backward algorithmic "
                                "bytes from exact per-ray footprint counts)",
            "launch_ms": fused_ms, "launch_ms_p50": head["fused_kernel_ms_p50"],
            "launch_ms_p90": head["fused_kernel_ms_p90"],
            "launch_ms_cold": head.get("fused_kernel_ms_cold"),
            "frac_fused_bytes": head["hbm_frac_fused_bytes"],
            "fused_bytes_per_launch": head["bytes_fused"],
            "compulsory_bytes_per_launch": head["bytes_compulsory"],
            "compulsory_frac": head["hbm_frac_compulsory"],
            "copy_ceiling_GBps": round(copy_gbs, 1)}
    R = head["rays_per_step"]
    res = {
        "metric": METRIC, "value": head["rays_per_s"], "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"noisy_room_2cm_{R}", "scene": "6x6x3 m room, 20 primitives, "
                   "h=2 cm, SDF noise 0.5 voxel, RGB noise 0.1; target = clean renders",
                   "blocks": grid4.n_blocks, "rays_per_step": R, "step_m": 0.01, "t_far_m": 12.0,
                   "beta_m": 0.02, "max_samples": 128, "C": 3,
                   "loss": "L2 colour + 0.1 depth + 0.05 normal",
                   "step": "camera rays + gradient zeroing + fused march/forward/loss/backward "
                           "(Adam timed separately)"},
        "samples_per_s": head["samples_per_s"],
        "roofline": roof,
        "headline": head,
    }
    if not args.no_query:
        res["query"] = query_bench(grid4, vox4, w4["block_coords"], dev)
    del grid4, vox4
    torch.cuda.empty_cache()
    if not args.no_extra:
        w2 = workloads.room_2cm(n_rays=65536)
        c2 = fused_bench(dev, w2, workloads.room_2cm_target()["vox"], args.steps, args.warmup,
                         eikonal=True, separate=True)
        c2.pop("_grid")
        c2["workload"] = "room_2cm_65536"
        res["room_2cm_65536"] = c2
        w1 = workloads.sphere_tiny()
        c1 = fused_bench(dev, w1, w1["target_vox"], args.steps, args.warmup, lambda_d=0.0,
                         lambda_n=0.0)
        c1.pop("_grid")
        c1["workload"] = "sphere_64x48"
        c1["loss"] = "L2 colour only"
        res["sphere_64x48"] = c1
        torch.cuda.empty_cache()
    if not args.no_frames:
        res["frames"] = frames_bench(dev)
    if not args.no_fusion:
        res["fusion"] = fusion_bench(dev)
    if not args.no_crf:
        res["crf"] = crf_bench(dev)
    if not args.no_serve:
        res["serving"] = serve_bench(args, dev)
    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        oracle._load()
        res["cpu_baseline"] = cpu_baseline(w4, workloads.room_2cm(n_rays=65536),
                                           workloads.sphere_tiny(), min(args.cpu_rays, R),
                                           frames=not args.no_frames)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
