"""Benchmark: forward + backward rays/s of the sparse-dense SDF renderer.

Workload (one GPU): the 6 x 6 x 3 m synthetic room at 2 cm voxels
(11,542 allocated 8^3 blocks, SDF + RGB), batches of 65,536 random pixels
from 30 seeded 640x480 poses, step 1 cm, t in [0, 12] m, beta = 2 cm, at
most 128 samples per ray.  One step = camera rays for the batch, forward
render (colour, depth, normal), squared-L2 loss gradient against renders
of the same room with a second texture, gradient zeroing, backward render.
Inputs are resident on the GPU before timing starts.

Prints one JSON line.  `roofline` is for the dominant kernel, timed with
HIP events on its own stream over the timed steps; its algorithmic bytes
come from exact per-ray footprint counts (samples, distinct voxels,
distinct blocks).  `cpu_baseline` times the CPU oracle on a bounded
sample of the same batch on the host.
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
    """Per-launch algorithmic bytes of forward and backward from (S, U, K)."""
    import numpy as np
    c = counts.astype(np.int64)
    K = c[:, 2].sum()
    U = c[:, 1].sum()
    R = c.shape[0]
    V = 4 * (1 + C)
    O = 4 * (C + 1 + 3 + 1)
    fwd = R * 24 + 16 * K + V * U + R * O
    bwd = R * 24 + 16 * K + 2 * V * U + R * O + R * (O - 4)
    return int(fwd), int(bwd)


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


def cpu_baseline(w, n_rays):
    """Oracle forward + loss gradient + backward on the first n_rays rays.

    The loss target is zero (the oracle takes no input from the GPU path;
    the work done does not depend on the target values)."""
    import numpy as np
    import oracle
    rays = w["rays"][:n_rays]
    target = {"feat": np.zeros((n_rays, 3)), "depth": np.zeros(n_rays), "normal": np.zeros((n_rays, 3))}
    t0 = time.perf_counter()
    out = oracle.render_forward(w["block_coords"], w["vox"], 3, w["h"], w["origin"], rays, w["params"])
    L, gc, gd, gn = oracle.l2_loss_grad(out["feat"], target["feat"], out["depth"],
                                        target["depth"], out["normal"], target["normal"], 0.1, 0.05)
    oracle.render_backward(w["block_coords"], w["vox"], 3, w["h"], w["origin"], rays, w["params"],
                           gc, gd, gn, None)
    dt = time.perf_counter() - t0
    return {"value": n_rays / dt, "unit": "rays/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_rays} rays of the 65,536-ray batch, forward + loss gradient + "
                      f"backward, single thread ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--rays", type=int, default=65536)
    ap.add_argument("--cpu-rays", type=int, default=32768)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib-mib", type=int, default=0,
                    help="run one elementwise kernel over a tensor of this size first "
                         "(reads and writes it once: a reference for memory counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(rays are independent; a multi-GPU step would shard the batch and all-reduce the "
              "voxel gradients). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2305_13220_amd as sg
    from synth import workloads

    dev = torch.device("cuda:0")
    t_setup = time.perf_counter()
    w = workloads.room_2cm(n_rays=args.rays)
    tgt_scene = workloads.room_2cm_target()
    C = 3
    grid = sg.Grid(torch.from_numpy(w["block_coords"]).to(dev), float(w["h"]),
                   tuple(float(x) for x in w["origin"]))
    vox = torch.from_numpy(w["vox"]).to(dev)
    tvox = torch.from_numpy(tgt_scene["vox"]).to(dev)
    cams = torch.from_numpy(w["cams"]).to(dev)
    pix = torch.from_numpy(w["pix"]).to(dev)
    params = sg.RenderParams.of(w["params"])
    R = args.rays
    rays = sg.rays_pinhole(cams, pix)
    target = sg.render_forward(grid, tvox, rays, params)
    target = {k: v.clone() for k, v in target.items()}
    grad = torch.zeros_like(vox)
    out = {"feat": torch.empty((R, C), device=dev), "depth": torch.empty(R, device=dev),
           "normal": torch.empty((R, 3), device=dev), "wsum": torch.empty(R, device=dev),
           "nsamples": torch.empty(R, dtype=torch.int32, device=dev)}
    gout = {"feat": torch.empty((R, C), device=dev), "depth": torch.empty(R, device=dev),
            "normal": torch.empty((R, 3), device=dev)}
    if args.calib_mib > 0:
        a = torch.ones(args.calib_mib << 18, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.neg(a, out=b)
        del a, b
    torch.cuda.synchronize()
    log(f"setup {time.perf_counter() - t_setup:.1f}s: {grid.n_blocks} blocks, {R} rays")

    ev = []

    def step(timed):
        rr = sg.rays_pinhole(cams, pix)
        if timed:
            e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            e[0].record()
        sg.render_forward(grid, vox, rr, params, out=out)
        if timed:
            e[1].record()
        sg.l2_loss_grad(out, target, 0.1, 0.05, out=gout)
        grad.zero_()
        if timed:
            e[2].record()
        sg.render_backward(grid, vox, rr, params, gout["feat"], gout["depth"], gout["normal"],
                           None, grad_vox=grad)
        if timed:
            e[3].record()
            ev.append(e)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        step(True)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / args.steps
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    bwd_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in ev]))

    counts = sg.render_footprint(grid, rays, params).cpu().numpy()
    fb, bb = algorithmic_bytes(counts, C)
    S = int(counts[:, 0].sum())
    dominant = "backward" if bwd_ms >= fwd_ms else "forward"
    k_ms, k_bytes = (bwd_ms, bb) if dominant == "backward" else (fwd_ms, fb)
    achieved = k_bytes / (k_ms * 1e-3) / 1e9
    kname = "k_render_bwd<3>" if dominant == "backward" else "k_render_fwd<3>"
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(kname, "room_2cm_65536"), "kernel": kname,
            "algorithmic_bytes_per_launch": k_bytes, "launch_ms": round(k_ms, 4)}
    res = {
        "metric": METRIC, "value": R / (ms * 1e-3), "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "room_2cm_65536", "scene": "6x6x3 m room, 20 primitives, h=2 cm",
                   "blocks": grid.n_blocks, "rays_per_step": R, "step_m": 0.01, "t_far_m": 12.0,
                   "beta_m": 0.02, "max_samples": 128, "C": C},
        "samples_per_s": S / (ms * 1e-3),
        "mean_samples_per_ray": S / R,
        "fwd_ms": round(fwd_ms, 4), "bwd_ms": round(bwd_ms, 4),
        "fwd_bwd_hbm_roofline_pct": round(100 * (fb + bb) / ((fwd_ms + bwd_ms) * 1e-3) / 1e9
                                          / HBM_PEAK_GBS, 2),
        "roofline": roof,
    }
    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        res["cpu_baseline"] = cpu_baseline(w, min(args.cpu_rays, R))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
