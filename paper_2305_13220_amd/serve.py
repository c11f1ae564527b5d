"""Render serving on one GPU: resident grids, HBM-budget admission, continuous
batching into packed multi-grid launches replayed from a HIP graph.

A request asks for a full frame (width x height, pinhole camera) of one of
the resident grids.  Arriving requests are admitted in order while the
output buffers of the requests in flight fit a device-memory budget.  Every
tick packs up to `tick_rays` pixels from the unfinished requests (a large
request spans several ticks; several requests share a tick; by default the
request with the fewest remaining pixels goes first, with its waiting time
counted against its size), into a slot table that is copied to the device and rendered
by one `sg_render_forward_packed` launch.  Two table buffers and two
captured graphs alternate, so the host fills one table while the GPU renders
the other.  A request completes with the tick that renders its last pixels.

`PlainServer` is the baseline: each request, in arrival order, gets its own
`sg_rays_pinhole` + `sg_render_forward` calls.  Both report per-request
latency (completion - arrival) from GPU events; completion times are GPU
timestamps relative to a reference event recorded with a known host time.
Results are identical per pixel in both paths (same per-ray code).
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from ._lib import check, lib, ptr, stream_ptr
from .grid import Grid, RenderParams, rays_pinhole, render_forward


class SlotC(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32), ("width", ctypes.c_int32),
                ("pixel_begin", ctypes.c_int64), ("count", ctypes.c_int64),
                ("ray_base", ctypes.c_int64), ("cam", ctypes.c_float * 16),
                ("feat", ctypes.c_void_p), ("depth", ctypes.c_void_p),
                ("normal", ctypes.c_void_p), ("wsum", ctypes.c_void_p),
                ("nsamples", ctypes.c_void_p)]


SLOT_DTYPE = np.dtype({
    "names": ["grid", "width", "pixel_begin", "count", "ray_base", "cam", "feat", "depth",
              "normal", "wsum", "nsamples"],
    "formats": ["<i4", "<i4", "<i8", "<i8", "<i8", ("<f4", (16,)), "<u8", "<u8", "<u8", "<u8",
                "<u8"],
    "offsets": [SlotC.grid.offset, SlotC.width.offset, SlotC.pixel_begin.offset,
                SlotC.count.offset, SlotC.ray_base.offset, SlotC.cam.offset, SlotC.feat.offset,
                SlotC.depth.offset, SlotC.normal.offset, SlotC.wsum.offset,
                SlotC.nsamples.offset],
    "itemsize": ctypes.sizeof(SlotC)})

PACKED_GRID_BYTES = 512




@dataclass
class Request:
    rid: int
    grid: int
    cam: np.ndarray        # float32 [16]
    width: int
    height: int
    arrival: float         # seconds, relative to the start of the run
    out: dict = field(default=None, repr=False)
    out_ptrs: tuple = field(default=None, repr=False)  # device addresses of the outputs
    done: float = None     # completion time, seconds relative to the start of the run

    @property
    def pixels(self):
        return self.width * self.height

    def out_bytes(self, C):
        return self.pixels * 4 * (C + 6)


def alloc_outputs(n, C, device):
    """The five per-pixel outputs of a request as views of one allocation."""
    buf = torch.empty(n * (C + 6), dtype=torch.float32, device=device)
    o = {}
    at = 0
    for k, w in (("feat", C), ("depth", 1), ("normal", 3), ("wsum", 1), ("nsamples", 1)):
        v = buf[at:at + n * w]
        o[k] = v.view(n, w) if k in ("feat", "normal") else v
        at += n * w
    o["nsamples"] = o["nsamples"].view(torch.int32)
    return o


class _Clock:
    """GPU completion times relative to a host-timed reference event."""

    def __init__(self):
        torch.cuda.synchronize()
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record()
        torch.cuda.synchronize()
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def event_time(self, ev):
        return self.ref.elapsed_time(ev) * 1e-3


class PackedServer:
    """Continuous batching of render requests into packed, graph-replayed launches."""

    def __init__(self, grids, C=3, hbm_budget_bytes=8 << 30, tick_rays=1 << 20, max_slots=256,
                 use_graph=True, keep_outputs=True, order="srpt", aging_px_per_s=2e8,
                 one_grid_per_tick=False, launch="multi_grid", small_tick_rays=None, n_tables=2,
                 max_inflight=None):
        """grids: list of (Grid, vox tensor, RenderParams or dict).  With
        keep_outputs False a request's outputs are released when it completes.

        order "fifo" packs ticks in admission order; "srpt" packs the
        admitted request with the fewest remaining pixels first, where every
        second of waiting counts as aging_px_per_s fewer pixels (so a large
        request is not starved).  With one_grid_per_tick a tick holds only
        requests on the grid of its first request, so a launch works on one
        grid's voxels (better cache reuse than mixing grids).

        With small_tick_rays set, a tick whose first request has at most that
        many pixels left is limited to that many pixels (and launched with a
        grid of that size), so small requests are not held up behind a full
        tick.

        n_tables slot tables are used in turn: up to n_tables ticks can be
        queued on the GPU while the host fills the next table.  max_inflight
        (default n_tables) bounds the ticks queued on the GPU: with 1 the
        next tick is packed only when the previous one has finished, so a
        request arriving meanwhile joins it (lower latency, at the cost of
        the GPU idling while the host packs).

        launch "per_grid" (implies one grid per tick) renders a tick with
        sg_render_forward_slots on that grid (one captured graph per grid and
        table); "multi_grid" with sg_render_forward_packed over the
        descriptor table of all grids (one graph per table)."""
        if order not in ("fifo", "srpt"):
            raise ValueError("order must be 'fifo' or 'srpt'")
        if launch not in ("per_grid", "multi_grid"):
            raise ValueError("launch must be 'per_grid' or 'multi_grid'")
        self.launch_mode = launch
        one_grid_per_tick = one_grid_per_tick or launch == "per_grid"
        self.order = order
        self.aging = float(aging_px_per_s)
        self.one_grid = bool(one_grid_per_tick)
        L = lib()
        self.C = C
        self.dev = grids[0][0].device
        self.budget = int(hbm_budget_bytes)
        self.tick_rays = int(tick_rays)
        self.small_tick = self.tick_rays if small_tick_rays is None else min(int(small_tick_rays),
                                                                             self.tick_rays)
        self.max_slots = int(max_slots)
        descs = (ctypes.c_ubyte * (PACKED_GRID_BYTES * len(grids)))()
        cap = 1
        for i, (g, vox, prm) in enumerate(grids):
            prm = RenderParams.of(prm)
            if vox.shape[-1] - 1 != C:
                raise ValueError("every resident grid must have C feature channels")
            cap = max(cap, prm.max_samples)
            pc = prm.c()
            check(L.sg_packed_grid_desc(g.handle, ptr(vox), C, ctypes.byref(pc),
                                        ctypes.byref(descs, PACKED_GRID_BYTES * i)),
                  "sg_packed_grid_desc")
        self.keep = grids  # grids and voxels must outlive the launches
        # the grids' memory must not move while descriptors or captured
        # launches refer to it: extend is refused until close()
        for g, _, _ in grids:
            g.pin()
        self._closed = False
        self._descs = descs
        self.grid_args = [(g, vox, RenderParams.of(prm).c()) for g, vox, prm in grids]
        self.n_grids = len(grids)
        self.q_cap = cap
        self.d_grids = torch.frombuffer(bytearray(descs), dtype=torch.uint8).to(self.dev)
        n = self.max_slots
        self.n_tables = max(2, int(n_tables))
        nt = self.n_tables
        # one table = [slot count (int32), padding to 256 B | slots]: filled in
        # place in pinned memory and sent with one copy
        hdr = self._hdr = 256
        size = hdr + n * SLOT_DTYPE.itemsize
        self.h_tab = [torch.zeros(size, dtype=torch.uint8).pin_memory() for _ in range(nt)]
        self._h_count = [t.numpy()[:4].view(np.int32) for t in self.h_tab]
        self._h_slots = [t.numpy()[hdr:].view(SLOT_DTYPE) for t in self.h_tab]
        self.d_tab = [torch.zeros(size, dtype=torch.uint8, device=self.dev) for _ in range(nt)]
        self.d_count = [ctypes.c_void_p(t.data_ptr()) for t in self.d_tab]
        self.d_slots = [ctypes.c_void_p(t.data_ptr() + hdr) for t in self.d_tab]
        self.graphs = {}  # (table, grid or -1, rays) -> captured graph
        self.use_graph = use_graph
        self.busy = [None] * nt  # end event of the tick that last used each table
        self.max_inflight = nt if max_inflight is None else max(1, int(max_inflight))
        self.next_b = 0
        self.keep_outputs = keep_outputs
        if use_graph:
            # capture every (table, grid, launch size) now, on empty tables,
            # so that no capture lands inside a run
            for b in range(nt):
                for gi in (range(self.n_grids) if self.launch_mode == "per_grid" else (0,)):
                    for rays in self._launch_sizes():
                        self._render(b, gi, rays)
            torch.cuda.synchronize()

    def _launch_sizes(self):
        rays, out = 1 << 16, []
        while rays < self.tick_rays:
            out.append(rays)
            rays <<= 1
        return out + [self.tick_rays]

    def close(self):
        """Release the grids (extend is allowed again) and the captured graphs."""
        if not self._closed:
            self.graphs.clear()
            for g, _, _ in self.keep:
                g.unpin()
            self._closed = True

    def check_grids(self):
        """Raise if any resident grid's memory moved since the descriptors
        were made (sg_packed_grid_check)."""
        for i, (g, _, _) in enumerate(self.keep):
            check(lib().sg_packed_grid_check(
                g.handle, ctypes.byref(self._descs, PACKED_GRID_BYTES * i)), "sg_packed_grid_check")

    def _launch(self, b, gi, rays):
        if self.launch_mode == "per_grid":
            g, vox, pc = self.grid_args[gi]
            check(lib().sg_render_forward_slots(g.handle, ptr(vox), self.C, ctypes.byref(pc),
                                                self.d_slots[b], self.d_count[b],
                                                self.max_slots, rays, stream_ptr(self.dev)),
                  "sg_render_forward_slots")
            return
        check(lib().sg_render_forward_packed(ptr(self.d_grids), self.n_grids, self.d_slots[b],
                                             self.d_count[b], self.max_slots, self.C,
                                             self.q_cap, rays, stream_ptr(self.dev)),
              "sg_render_forward_packed")

    def _render(self, b, gi, rays):
        if not self.use_graph:
            self._launch(b, gi, rays)
            return
        key = (b, gi if self.launch_mode == "per_grid" else -1, rays)
        if key not in self.graphs:
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            s = torch.cuda.Stream(self.dev)
            s.wait_stream(torch.cuda.current_stream(self.dev))
            with torch.cuda.stream(s):
                self._launch(b, gi, rays)  # warm-up outside capture
            torch.cuda.current_stream(self.dev).wait_stream(s)
            torch.cuda.synchronize()
            with torch.cuda.graph(g):
                self._launch(b, gi, rays)
            self.graphs[key] = g
            torch.cuda.synchronize()
        self.graphs[key].replay()

    def tick(self, work):
        """Render one tick: work = list of (request, pixel_begin, count).  Returns its end event."""
        b = self.next_b
        self.next_b = (b + 1) % self.n_tables
        if self.busy[b] is not None:
            self.busy[b].synchronize()  # the table is free once its tick has finished
        slots = self._h_slots[b]
        base = 0
        for i, (req, p0, cnt) in enumerate(work):
            slots[i] = (req.grid, req.width, p0, cnt, base, req.cam) + req.out_ptrs
            base += cnt
        self._h_count[b][0] = len(work)
        nbytes = self._hdr + len(work) * SLOT_DTYPE.itemsize
        self.d_tab[b][:nbytes].copy_(self.h_tab[b][:nbytes], non_blocking=True)
        total = base
        # launch grid: the smallest of the launch sizes that holds the tick, so
        # a tick of one small request does not launch a full tick's waves
        rays = next(r for r in self._launch_sizes() if r >= total or r == self.tick_rays)
        self._render(b, work[0][0].grid, rays)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record()
        self.busy[b] = ev
        return ev

    def run(self, requests, realtime=True):
        """Serve requests (sorted by arrival); fills req.done; returns the requests."""
        if self._closed:
            raise RuntimeError("server is closed")
        self.check_grids()
        clock = _Clock()
        pending = list(requests)
        admitted = []  # requests with pixels left to schedule: [req, next_pixel]
        in_flight_bytes = 0
        inflight = []  # (end event, [requests completed by it], bytes released)
        i = 0
        while i < len(pending) or admitted or inflight:
            now = clock.now() if realtime else float("inf")
            # admission by device-memory budget, in arrival order
            while i < len(pending) and pending[i].arrival <= now:
                req = pending[i]
                need = req.out_bytes(self.C)
                if admitted or inflight:
                    if in_flight_bytes + need > self.budget:
                        break
                in_flight_bytes += need  # reserved now, allocated when first packed
                admitted.append([req, 0])
                i += 1
            # retire finished ticks
            keep = []
            for ev, finished, freed in inflight:
                if ev.query():
                    t = clock.event_time(ev)
                    for r in finished:
                        r.done = t
                        if not self.keep_outputs:
                            r.out = None
                    in_flight_bytes -= freed
                else:
                    keep.append((ev, finished, freed))
            inflight = keep
            if not admitted or len(inflight) >= self.max_inflight:
                if inflight:
                    time.sleep(0.00002)
                elif i < len(pending):
                    wait = pending[i].arrival - clock.now()
                    if wait > 0:
                        time.sleep(min(wait, 0.002))
                continue
            # pack one tick
            if self.order == "srpt" and len(admitted) > 1:
                t_now = clock.now()
                admitted.sort(key=lambda e: (e[0].pixels - e[1]) - self.aging * (t_now - e[0].arrival))
            first_left = admitted[0][0].pixels - admitted[0][1]
            budget = self.small_tick if first_left <= self.small_tick else self.tick_rays
            work, finished, freed = [], [], 0
            g0 = admitted[0][0].grid
            k = 0
            while k < len(admitted) and budget > 0 and len(work) < self.max_slots:
                req, nxt = admitted[k]
                if self.one_grid and req.grid != g0:
                    k += 1
                    continue
                cnt = min(budget, req.pixels - nxt)
                if req.out is None:
                    req.out = alloc_outputs(req.pixels, self.C, self.dev)
                    o = req.out
                    req.out_ptrs = (o["feat"].data_ptr(), o["depth"].data_ptr(),
                                    o["normal"].data_ptr(), o["wsum"].data_ptr(),
                                    o["nsamples"].data_ptr())
                work.append((req, nxt, cnt))
                budget -= cnt
                if nxt + cnt == req.pixels:
                    admitted.pop(k)
                    finished.append(req)
                    freed += req.out_bytes(self.C)
                else:
                    admitted[k][1] = nxt + cnt
                    k += 1
            ev = self.tick(work)
            inflight.append((ev, finished, freed))
        torch.cuda.synchronize()
        return requests


class PlainServer:
    """Baseline: one sg_rays_pinhole + sg_render_forward per request, in arrival order."""

    def __init__(self, grids, C=3, keep_outputs=True):
        self.grids = grids
        self.C = C
        self.dev = grids[0][0].device
        self.keep_outputs = keep_outputs
        self._pix = {}  # (W, H) -> int32 [W*H, 3] pixel table (camera 0), made once

    def render(self, req, cam_row=None):
        g, vox, prm = self.grids[req.grid]
        W, H = req.width, req.height
        pix = self._pix.get((W, H))
        if pix is None:
            v, u = torch.meshgrid(torch.arange(H, device=self.dev),
                                  torch.arange(W, device=self.dev), indexing="ij")
            pix = torch.stack([torch.zeros_like(u).reshape(-1), u.reshape(-1), v.reshape(-1)],
                              -1).to(torch.int32)
            self._pix[(W, H)] = pix
        if cam_row is None:
            cam = torch.from_numpy(np.asarray(req.cam, np.float32).reshape(1, 16)).to(self.dev)
        else:  # a row of pinned memory: the copy does not wait for the GPU queue
            cam_row.copy_(torch.from_numpy(np.asarray(req.cam, np.float32).reshape(1, 16)))
            cam = cam_row.to(self.dev, non_blocking=True)
        rays = rays_pinhole(cam, pix)
        req.out = render_forward(g, vox, rays, prm)

    def run(self, requests, realtime=True):
        """Serve requests in arrival order; fills req.done.  With keep_outputs
        False the outputs are released after launch (stream order makes the
        memory safe to reuse), as a server that hands results on would."""
        cams = torch.empty((len(requests), 16), dtype=torch.float32).pin_memory()
        clock = _Clock()
        pend = []
        for i, req in enumerate(requests):
            if realtime:
                while clock.now() < req.arrival:
                    time.sleep(min(0.002, max(0.0, req.arrival - clock.now())))
            self.render(req, cams[i:i + 1])
            ev = torch.cuda.Event(enable_timing=True)
            ev.record()
            if not self.keep_outputs:
                req.out = None
            pend.append((req, ev))
        torch.cuda.synchronize()
        for req, ev in pend:
            req.done = clock.event_time(ev)
        return requests


def poisson_requests(n, qps, n_grids, cams_per_grid, resolutions, seed=0, fov_deg=60.0):
    """Seeded requests: Poisson arrivals at rate qps, uniform grid, resolution
    and camera (pose from cams_per_grid[grid], intrinsics from the resolution)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / qps, size=n))
    reqs = []
    for i in range(n):
        gi = int(rng.integers(0, n_grids))
        W, H = resolutions[int(rng.integers(0, len(resolutions)))]
        poses = cams_per_grid[gi]
        cam = np.array(poses[int(rng.integers(0, len(poses)))], np.float32).copy()
        f = (W / 2) / np.tan(np.deg2rad(fov_deg) / 2)
        cam[:4] = (f, f, W / 2, H / 2)
        reqs.append(Request(i, gi, cam, W, H, float(t[i])))
    return reqs


def latency_stats(requests):
    lat = np.array([r.done - r.arrival for r in requests]) * 1e3
    span = max(r.done for r in requests) - min(r.arrival for r in requests)
    px = sum(r.pixels for r in requests)
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "rays_per_s": px / span, "requests": len(requests)}
