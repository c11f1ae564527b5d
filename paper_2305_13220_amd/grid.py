"""Python face of the sparse-dense grid and its render calls.

Thin wrappers over the C ABI in include/sgrid.h (see _lib.py): they check
arguments, allocate output tensors with torch and launch the library's HIP
kernels on the current stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import SgridError, check, lib, ptr, stream_ptr, want

SUPPORTED_C = (0, 1, 2, 3, 4, 8, 16, 19, 32)


@dataclass(frozen=True)
class RenderParams:
    """Lattice spacing, t range (t_far inclusive), Laplace scale, sample cap."""
    step: float
    t_near: float
    t_far: float
    beta: float
    max_samples: int = 128

    def c(self):
        return _lib.RenderParamsC(self.step, self.t_near, self.t_far, self.beta, self.max_samples)

    @staticmethod
    def of(p):
        if isinstance(p, RenderParams):
            return p
        return RenderParams(p["step"], p["t_near"], p["t_far"], p["beta"], p["max_samples"])


class Grid:
    """Hash of allocated 8^3 blocks (collision-free, first-occurrence indices)."""

    def __init__(self, block_coords: torch.Tensor, voxel_size: float, origin=(0.0, 0.0, 0.0),
                 return_index: bool = False, dense_map_max_cells: int = -1, _handle=None):
        """dense_map_max_cells: 0 = hash only; < 0 = library default."""
        if _handle is not None:  # a grid the library already built (see from_depth)
            self.device = block_coords
            self._h = _handle
            self.index_of_input = None
        else:
            want(block_coords, "block_coords", torch.int32, (None, 3))
            self.device = block_coords.device
            n = block_coords.shape[0]
            org = (ctypes.c_float * 3)(*[float(x) for x in origin])
            handle = ctypes.c_void_p()
            idx = torch.empty(n, dtype=torch.int32, device=self.device) if return_index else None
            opts = _lib.BuildOptionsC(int(dense_map_max_cells))
            with torch.cuda.device(self.device):
                check(lib().sg_grid_build_ex(ptr(block_coords), n, ctypes.c_float(voxel_size), org,
                                             stream_ptr(self.device), ctypes.byref(handle), ptr(idx),
                                             ctypes.byref(opts)), "sg_grid_build_ex")
            self._h = handle
            self.index_of_input = idx
        nb = ctypes.c_int64()
        check(lib().sg_grid_num_blocks(self._h, ctypes.byref(nb)), "sg_grid_num_blocks")
        self.n_blocks = nb.value
        vs = ctypes.c_float()
        o = (ctypes.c_float * 3)()
        check(lib().sg_grid_geometry(self._h, ctypes.byref(vs), o), "sg_grid_geometry")
        self.voxel_size = vs.value
        self.origin = tuple(o)

    @classmethod
    def from_depth(cls, cams: torch.Tensor, depth: torch.Tensor, voxel_size: float,
                   origin=(0.0, 0.0, 0.0), dilate: int = 2, depth_max: float = float("inf"),
                   dense_map_max_cells: int = -1):
        """The grid of the blocks allocated for depth maps [F,H,W] seen by
        cams [F,16] (Sec. 3.4.1), built in one library call."""
        want(cams, "cams", torch.float32, (None, 16))
        want(depth, "depth", torch.float32, (cams.shape[0], None, None), cams.device)
        F, H, W = depth.shape
        org = (ctypes.c_float * 3)(*[float(x) for x in origin])
        handle = ctypes.c_void_p()
        opts = _lib.BuildOptionsC(int(dense_map_max_cells))
        with torch.cuda.device(cams.device):
            check(lib().sg_grid_from_depth(ptr(cams), F, ptr(depth), W, H,
                                           ctypes.c_float(voxel_size), org, dilate,
                                           ctypes.c_float(depth_max), stream_ptr(cams.device),
                                           ctypes.byref(handle), ctypes.byref(opts)),
                  "sg_grid_from_depth")
        return cls(cams.device, voxel_size, origin, _handle=handle)

    def pin(self):
        """Register a user of the grid's index memory (a render server's
        descriptors or captured launches): extend is refused until unpin."""
        self._pins = getattr(self, "_pins", 0) + 1

    def unpin(self):
        self._pins = max(0, getattr(self, "_pins", 0) - 1)

    @property
    def generation(self):
        """0 when built, one more per extend (which moves the grid's memory)."""
        gen = ctypes.c_uint64()
        check(lib().sg_grid_generation(self.handle, ctypes.byref(gen)), "sg_grid_generation")
        return gen.value

    def extend(self, new_coords: torch.Tensor, dense_map_max_cells: int = -1):
        """Add blocks: existing blocks keep their indices, new ones follow in
        order of first occurrence.  Returns the new number of blocks.  The
        grid's memory moves, so this is refused while a server holds the grid
        (descriptors and captured launches would point at freed memory)."""
        if getattr(self, "_pins", 0) > 0:
            raise SgridError("extend refused: the grid is pinned by a render server (its packed "
                             "descriptors and captured launches would refer to freed memory); "
                             "close the server first")
        want(new_coords, "new_coords", torch.int32, (None, 3), self.device)
        opts = _lib.BuildOptionsC(int(dense_map_max_cells))
        with torch.cuda.device(self.device):
            torch.cuda.synchronize(self.device)
            check(lib().sg_grid_extend(self.handle, ptr(new_coords), new_coords.shape[0],
                                       stream_ptr(self.device), ctypes.byref(opts)),
                  "sg_grid_extend")
        nb = ctypes.c_int64()
        check(lib().sg_grid_num_blocks(self._h, ctypes.byref(nb)), "sg_grid_num_blocks")
        self.n_blocks = nb.value
        return self.n_blocks

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise SgridError("grid has been destroyed")
        return self._h

    def block_coords(self):
        out = torch.empty((self.n_blocks, 3), dtype=torch.int32, device=self.device)
        check(lib().sg_grid_block_coords(self.handle, ptr(out), stream_ptr(self.device)),
              "sg_grid_block_coords")
        return out

    def dense_map(self):
        """(map int32 [dz,dy,dx] or None, bmin (x,y,z)) of the dense block map."""
        dims = (ctypes.c_int32 * 3)()
        bmin = (ctypes.c_int32 * 3)()
        check(lib().sg_grid_dense_map(self.handle, dims, bmin), "sg_grid_dense_map")
        if dims[0] == 0:
            return None, tuple(bmin)
        out = torch.empty((dims[2], dims[1], dims[0]), dtype=torch.int32, device=self.device)
        check(lib().sg_grid_copy_dense_map(self.handle, ptr(out), stream_ptr(self.device)),
              "sg_grid_copy_dense_map")
        return out, tuple(bmin)

    def neighbors(self):
        out = torch.empty((self.n_blocks, 8), dtype=torch.int32, device=self.device)
        check(lib().sg_grid_neighbors(self.handle, ptr(out), stream_ptr(self.device)),
              "sg_grid_neighbors")
        return out

    def lookup(self, coords: torch.Tensor):
        want(coords, "coords", torch.int32, (None, 3), self.device)
        out = torch.empty(coords.shape[0], dtype=torch.int32, device=self.device)
        check(lib().sg_grid_lookup(self.handle, ptr(coords), coords.shape[0], ptr(out),
                                   stream_ptr(self.device)), "sg_grid_lookup")
        return out

    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self.device)
            check(lib().sg_grid_destroy(self._h), "sg_grid_destroy")
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _check_vox(grid, vox, C):
    if C not in SUPPORTED_C:
        raise ValueError(f"C={C} unsupported; supported: {SUPPORTED_C}")
    want(vox, "vox", torch.float32, (grid.n_blocks, 512, 1 + C), grid.device)


# Sample lists.  A single call marches in its own kernel (lists=None, the
# default: cheapest when one kernel consumes the samples).  When several
# calls consume the same rays (a forward and its backward), march() once and
# pass the buffer; lists="auto" does that for one call, up to this size.
LISTS_AUTO_MAX = 4 << 30


def list_bytes(n_rays: int, params) -> int:
    """Bytes of the sample lists of n_rays rays (sg_render_list_bytes)."""
    prm = RenderParams.of(params).c()
    return int(lib().sg_render_list_bytes(int(n_rays), ctypes.byref(prm)))


def march(grid: Grid, rays: torch.Tensor, params, out: torch.Tensor = None) -> torch.Tensor:
    """Run the block march alone: the kept samples of every ray, as a uint8
    buffer that render_forward / render_backward / render_l2_step accept as
    `lists` for the same grid, rays and params."""
    params = RenderParams.of(params)
    want(rays, "rays", torch.float32, (None, 6), grid.device)
    R = rays.shape[0]
    nb = list_bytes(R, params)
    if out is None:
        out = torch.empty(max(nb, 8), dtype=torch.uint8, device=grid.device)
    want(out, "lists", torch.uint8, (None,), grid.device)
    prm = params.c()
    check(lib().sg_render_march(grid.handle, ptr(rays), R, ctypes.byref(prm), ptr(out), out.numel(),
                                stream_ptr(grid.device)), "sg_render_march")
    return out


def _lists(lists, grid, rays, params):
    """(pointer, bytes, buffer) for a render call.  "auto" marches into a new
    buffer when it is at most LISTS_AUTO_MAX bytes; None lets the shading
    kernel march; a uint8 tensor from march() is used as given."""
    if lists is None:
        return None, 0, None
    if isinstance(lists, str):
        if lists != "auto":
            raise ValueError("lists must be 'auto', None or a buffer from march()")
        nb = list_bytes(rays.shape[0], params)
        if nb == 0 or nb > LISTS_AUTO_MAX:
            return None, 0, None
        lists = march(grid, rays, params)
    want(lists, "lists", torch.uint8, (None,), grid.device)
    return ptr(lists), lists.numel(), lists


def render_forward(grid: Grid, vox: torch.Tensor, rays: torch.Tensor, params, out=None,
                   lists=None):
    """Colour/feature, depth, normal, weight sum and sample count per ray."""
    params = RenderParams.of(params)
    C = vox.shape[-1] - 1
    _check_vox(grid, vox, C)
    want(rays, "rays", torch.float32, (None, 6), grid.device)
    R = rays.shape[0]
    dev = grid.device
    if out is None:
        out = {"feat": torch.empty((R, C), dtype=torch.float32, device=dev),
               "depth": torch.empty(R, dtype=torch.float32, device=dev),
               "normal": torch.empty((R, 3), dtype=torch.float32, device=dev),
               "wsum": torch.empty(R, dtype=torch.float32, device=dev),
               "nsamples": torch.empty(R, dtype=torch.int32, device=dev)}
    prm = params.c()
    wp, wb, _keep = _lists(lists, grid, rays, params)
    check(lib().sg_render_forward(grid.handle, ptr(vox), C, ptr(rays), R, ctypes.byref(prm),
                                  ptr(out["feat"]) if C else None, ptr(out["depth"]),
                                  ptr(out["normal"]), ptr(out["wsum"]), ptr(out.get("nsamples")),
                                  wp, wb, stream_ptr(dev)), "sg_render_forward")
    return out


def render_backward(grid: Grid, vox: torch.Tensor, rays: torch.Tensor, params, g_feat, g_depth,
                    g_normal, g_wsum=None, grad_vox=None, lists=None):
    """Accumulate dL/dvox for upstream gradients of the render outputs."""
    params = RenderParams.of(params)
    C = vox.shape[-1] - 1
    _check_vox(grid, vox, C)
    want(rays, "rays", torch.float32, (None, 6), grid.device)
    R = rays.shape[0]
    if C:
        want(g_feat, "g_feat", torch.float32, (R, C), grid.device)
    want(g_depth, "g_depth", torch.float32, (R,), grid.device)
    want(g_normal, "g_normal", torch.float32, (R, 3), grid.device)
    if g_wsum is not None:
        want(g_wsum, "g_wsum", torch.float32, (R,), grid.device)
    if grad_vox is None:
        grad_vox = torch.zeros_like(vox)
    else:
        want(grad_vox, "grad_vox", torch.float32, tuple(vox.shape), grid.device)
    prm = params.c()
    wp, wb, _keep = _lists(lists, grid, rays, params)
    check(lib().sg_render_backward(grid.handle, ptr(vox), C, ptr(rays), R, ctypes.byref(prm),
                                   ptr(g_feat) if C else None, ptr(g_depth), ptr(g_normal),
                                   ptr(g_wsum), ptr(grad_vox), wp, wb, stream_ptr(grid.device)),
          "sg_render_backward")
    return grad_vox


def render_l2_step(grid: Grid, vox: torch.Tensor, rays: torch.Tensor, params, ref, lambda_d=0.1,
                   lambda_n=0.05, grad_vox=None, out=None, with_loss=False, lists=None,
                   lambda_e=0.0):
    """Fused forward + squared-L2 loss (+ lambda_e times the Eikonal term on
    the ray samples) + gradient (accumulated into grad_vox).

    ref: dict of reference "feat" [R,C], "depth" [R], "normal" [R,3].
    Returns (outputs dict, grad_vox[, loss_per_ray]).
    """
    params = RenderParams.of(params)
    C = vox.shape[-1] - 1
    _check_vox(grid, vox, C)
    want(rays, "rays", torch.float32, (None, 6), grid.device)
    R = rays.shape[0]
    dev = grid.device
    if C:
        want(ref["feat"], "ref.feat", torch.float32, (R, C), dev)
    want(ref["depth"], "ref.depth", torch.float32, (R,), dev)
    want(ref["normal"], "ref.normal", torch.float32, (R, 3), dev)
    if out is None:
        out = {"feat": torch.empty((R, C), dtype=torch.float32, device=dev),
               "depth": torch.empty(R, dtype=torch.float32, device=dev),
               "normal": torch.empty((R, 3), dtype=torch.float32, device=dev),
               "wsum": torch.empty(R, dtype=torch.float32, device=dev),
               "nsamples": torch.empty(R, dtype=torch.int32, device=dev)}
    if grad_vox is None:
        grad_vox = torch.zeros_like(vox)
    else:
        want(grad_vox, "grad_vox", torch.float32, tuple(vox.shape), dev)
    loss = torch.empty(R, dtype=torch.float32, device=dev) if with_loss else None
    prm = params.c()
    wp, wb, _keep = _lists(lists, grid, rays, params)
    check(lib().sg_render_l2_step(grid.handle, ptr(vox), C, ptr(rays), R, ctypes.byref(prm),
                                  ptr(ref["feat"]) if C else None, ptr(ref["depth"]),
                                  ptr(ref["normal"]), ctypes.c_float(lambda_d),
                                  ctypes.c_float(lambda_n), ctypes.c_float(lambda_e),
                                  ptr(out["feat"]) if C else None,
                                  ptr(out["depth"]), ptr(out["normal"]), ptr(out["wsum"]),
                                  ptr(out.get("nsamples")), ptr(loss), ptr(grad_vox), wp, wb,
                                  stream_ptr(dev)), "sg_render_l2_step")
    return (out, grad_vox, loss) if with_loss else (out, grad_vox)


def query(grid: Grid, vox: torch.Tensor, points: torch.Tensor, features: bool = True, out=None):
    """f, grad f and (if features) the C features at world points [m,3]
    (Eq. 17-18), with a validity flag (all 8 corner blocks allocated).
    Returns a dict; out may hold preallocated tensors of the same keys."""
    C = vox.shape[-1] - 1
    _check_vox(grid, vox, C)
    want(points, "points", torch.float32, (None, 3), grid.device)
    m = points.shape[0]
    dev = grid.device
    shapes = {"valid": ((m,), torch.int32), "f": ((m,), torch.float32),
              "grad": ((m, 3), torch.float32)}
    if features:
        shapes["feat"] = ((m, C), torch.float32)
    res = {}
    for k, (shape, dt) in shapes.items():
        t = None if out is None else out.get(k)
        if t is None:
            t = torch.empty(shape, dtype=dt, device=dev)
        else:
            want(t, k, dt, shape, dev)
        res[k] = t
    feat = res.get("feat")
    check(lib().sg_query(grid.handle, ptr(vox), C, ptr(points), m, ptr(res["valid"]),
                         ptr(res["f"]), ptr(res["grad"]), ptr(feat) if C and feat is not None
                         else None, stream_ptr(dev)), "sg_query")
    return res


def surface_points(grid: Grid, vox: torch.Tensor, rays: torch.Tensor, params):
    """First entering zero crossing of the SDF along each ray (the CRF's
    surface nodes, Sec. 3.5.3).  Returns (points [R,3], hit [R] int32)."""
    params = RenderParams.of(params)
    C = vox.shape[-1] - 1
    _check_vox(grid, vox, C)
    want(rays, "rays", torch.float32, (None, 6), grid.device)
    R = rays.shape[0]
    pts = torch.empty((R, 3), dtype=torch.float32, device=grid.device)
    hit = torch.empty(R, dtype=torch.int32, device=grid.device)
    prm = params.c()
    check(lib().sg_surface_points(grid.handle, ptr(vox), C, ptr(rays), R, ctypes.byref(prm),
                                  ptr(pts), ptr(hit), stream_ptr(grid.device)), "sg_surface_points")
    return pts, hit


def query_backward(grid: Grid, vox_shape, points: torch.Tensor, g_f=None, g_grad=None, g_feat=None,
                   grad_vox=None):
    """Accumulate the adjoint of ``query`` into grad_vox (zeros of vox_shape
    if None) for upstream gradients of f [m], grad f [m,3], features [m,C]."""
    C = vox_shape[-1] - 1
    want(points, "points", torch.float32, (None, 3), grid.device)
    m = points.shape[0]
    if grad_vox is None:
        grad_vox = torch.zeros(tuple(vox_shape), dtype=torch.float32, device=grid.device)
    _check_vox(grid, grad_vox, C)
    for t, name, shape in ((g_f, "g_f", (m,)), (g_grad, "g_grad", (m, 3)), (g_feat, "g_feat", (m, C))):
        if t is not None:
            want(t, name, torch.float32, shape, grid.device)
    check(lib().sg_query_backward(grid.handle, C, ptr(points), m, ptr(g_f), ptr(g_grad),
                                  ptr(g_feat), ptr(grad_vox), stream_ptr(grid.device)),
          "sg_query_backward")
    return grad_vox


def uniform_points(grid: Grid, n: int, seed: int = 0):
    """n points uniform over the allocated blocks [n,3] (Sec. 3.5.2's uniform
    in-grid samples; counter-based SplitMix64 draws, reproducible)."""
    out = torch.empty((n, 3), dtype=torch.float32, device=grid.device)
    check(lib().sg_uniform_points(grid.handle, n, ctypes.c_uint64(seed & ((1 << 64) - 1)), ptr(out),
                                  stream_ptr(grid.device)), "sg_uniform_points")
    return out


def eikonal(grid: Grid, vox: torch.Tensor, points: torch.Tensor, weight: float = 1.0,
            grad_vox=None, loss: bool = True):
    """Eikonal loss weight * (|grad f| - 1)^2 per point (Eq. 16) and its
    gradient accumulated into grad_vox (SDF channel).  Returns
    (loss [m] or None, grad_vox or None)."""
    C = vox.shape[-1] - 1
    _check_vox(grid, vox, C)
    want(points, "points", torch.float32, (None, 3), grid.device)
    if grad_vox is not None:
        want(grad_vox, "grad_vox", torch.float32, tuple(vox.shape), grid.device)
    m = points.shape[0]
    out = torch.empty(m, dtype=torch.float32, device=grid.device) if loss else None
    check(lib().sg_eikonal(grid.handle, ptr(vox), C, ptr(points), m, ctypes.c_float(weight),
                           ptr(out), ptr(grad_vox), stream_ptr(grid.device)), "sg_eikonal")
    return out, grad_vox


def alloc_blocks(cams: torch.Tensor, depth: torch.Tensor, voxel_size: float, origin=(0.0, 0.0, 0.0),
                 dilate: int = 2, depth_max: float = float("inf")):
    """Block coordinates [n,3] int32 allocated for depth maps [F,H,W] seen by
    cams [F,16] (Sec. 3.4.1), in order of first occurrence."""
    want(cams, "cams", torch.float32, (None, 16))
    want(depth, "depth", torch.float32, (cams.shape[0], None, None), cams.device)
    F, H, W = depth.shape
    org = (ctypes.c_float * 3)(*[float(x) for x in origin])
    n = ctypes.c_int64(0)
    dev = cams.device
    with torch.cuda.device(dev):
        rc = lib().sg_alloc_blocks(ptr(cams), F, ptr(depth), W, H, ctypes.c_float(voxel_size), org,
                                   dilate, ctypes.c_float(depth_max), None, 0, ctypes.byref(n),
                                   stream_ptr(dev))
        if rc != 0 and n.value == 0:
            check(rc, "sg_alloc_blocks")
        out = torch.empty((n.value, 3), dtype=torch.int32, device=dev)
        if n.value:
            check(lib().sg_alloc_blocks(ptr(cams), F, ptr(depth), W, H, ctypes.c_float(voxel_size),
                                        org, dilate, ctypes.c_float(depth_max), ptr(out), n.value,
                                        ctypes.byref(n), stream_ptr(dev)), "sg_alloc_blocks")
    return out


def fuse(grid: Grid, cams: torch.Tensor, depth: torch.Tensor, feat: torch.Tensor, trunc: float,
         n_sem: int = 0, vox=None, weight: bool = True):
    """Fused voxels [n,512,1+C] (and association counts [n,512]) of depth
    [F,H,W] and features [F,H,W,C] seen by cams [F,16] (Sec. 3.4.2).  The
    supplement's defaults are dilate R = 2 at allocation and trunc = 8 h R."""
    want(cams, "cams", torch.float32, (None, 16), grid.device)
    F = cams.shape[0]
    want(depth, "depth", torch.float32, (F, None, None), grid.device)
    H, W = depth.shape[1], depth.shape[2]
    want(feat, "feat", torch.float32, (F, H, W, None), grid.device)
    C = feat.shape[-1]
    if vox is None:
        vox = torch.empty((grid.n_blocks, 512, 1 + C), dtype=torch.float32, device=grid.device)
    else:
        want(vox, "vox", torch.float32, (grid.n_blocks, 512, 1 + C), grid.device)
    wt = torch.empty((grid.n_blocks, 512), dtype=torch.float32, device=grid.device) if weight else None
    check(lib().sg_fuse(grid.handle, ptr(cams), F, ptr(depth), ptr(feat) if C else None, C, W, H,
                        ctypes.c_float(trunc), n_sem, ptr(vox), ptr(wt), stream_ptr(grid.device)),
          "sg_fuse")
    return vox, wt


def denoise(grid: Grid, vox: torch.Tensor, radius: int = 1, sigma: float = 1.0, out=None):
    """Gaussian blur of every channel over allocated voxels (Sec. 3.4.3)."""
    C = vox.shape[-1] - 1
    _check_vox(grid, vox, C)
    if out is None:
        out = torch.empty_like(vox)
    else:
        want(out, "out", torch.float32, tuple(vox.shape), grid.device)
    check(lib().sg_denoise(grid.handle, ptr(vox), C, radius, ctypes.c_float(sigma), ptr(out),
                           stream_ptr(grid.device)), "sg_denoise")
    return out


def crf_label_loss(feat: torch.Tensor, Q: torch.Tensor, col0: int = 0, weight: float = 1.0,
                   g_feat=None):
    """KL(softmax(feat[:, col0:col0+L]) || Q) per node times weight (Sec.
    3.5.3), and its gradient written into g_feat[:, col0:col0+L] (a zero
    array shaped like feat if None).  Returns (loss [n], g_feat)."""
    want(feat, "feat", torch.float32, (None, None))
    n, Cf = feat.shape
    want(Q, "Q", torch.float32, (n, None), feat.device)
    L = Q.shape[1]
    if col0 < 0 or col0 + L > Cf:
        raise ValueError("the label columns lie outside feat")
    if g_feat is None:
        g_feat = torch.zeros_like(feat)
    else:
        want(g_feat, "g_feat", torch.float32, (n, Cf), feat.device)
    loss = torch.empty(n, dtype=torch.float32, device=feat.device)
    base = ctypes.c_void_p(feat.data_ptr() + 4 * col0) if n else None
    gbase = ctypes.c_void_p(g_feat.data_ptr() + 4 * col0) if n else None
    check(lib().sg_crf_label_loss(base, Cf, ptr(Q), n, L, ctypes.c_float(weight), ptr(loss), gbase,
                                  Cf, stream_ptr(feat.device)), "sg_crf_label_loss")
    return loss, g_feat


def crf_property_loss(feat: torch.Tensor, filtered: torch.Tensor, col0: int, weight: float = 1.0,
                      g_feat=None):
    """|x - F(x)/F(1)|^2 per node times weight for the property
    x = feat[:, col0:col0+P] (Sec. 3.5.3), filtered = lattice filter of
    [x, 1] [n, P+1]; the gradient goes into g_feat[:, col0:col0+P].
    Returns (loss [n], g_feat)."""
    want(feat, "feat", torch.float32, (None, None))
    n, Cf = feat.shape
    want(filtered, "filtered", torch.float32, (n, None), feat.device)
    P = filtered.shape[1] - 1
    if P < 1 or col0 < 0 or col0 + P > Cf:
        raise ValueError("the property columns lie outside feat")
    if g_feat is None:
        g_feat = torch.zeros_like(feat)
    else:
        want(g_feat, "g_feat", torch.float32, (n, Cf), feat.device)
    loss = torch.empty(n, dtype=torch.float32, device=feat.device)
    base = ctypes.c_void_p(feat.data_ptr() + 4 * col0) if n else None
    gbase = ctypes.c_void_p(g_feat.data_ptr() + 4 * col0) if n else None
    check(lib().sg_crf_property_loss(base, Cf, ptr(filtered), n, P, ctypes.c_float(weight),
                                     ptr(loss), gbase, Cf, stream_ptr(feat.device)),
          "sg_crf_property_loss")
    return loss, g_feat


class Lattice:
    """Permutohedral lattice of scaled feature positions [n,d] (Sec. 3.5.3)."""

    def __init__(self, pos: torch.Tensor, max_values: int = 32):
        want(pos, "pos", torch.float32, (None, None))
        self.device = pos.device
        self.n, self.d = pos.shape
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().sg_lattice_build(ptr(pos), self.n, self.d, max_values,
                                         stream_ptr(self.device), ctypes.byref(handle)),
                  "sg_lattice_build")
        self._h = handle
        nv = ctypes.c_int64()
        check(lib().sg_lattice_num_vertices(self._h, ctypes.byref(nv)), "sg_lattice_num_vertices")
        self.n_vertices = nv.value

    def filter(self, val: torch.Tensor, out=None):
        """Unnormalised lattice Gaussian filter of values [n,vd]."""
        want(val, "val", torch.float32, (self.n, None), self.device)
        if out is None:
            out = torch.empty_like(val)
        check(lib().sg_lattice_filter(self._h, ptr(val), val.shape[1], ptr(out),
                                      stream_ptr(self.device)), "sg_lattice_filter")
        return out

    def meanfield(self, unary: torch.Tensor, w_p: float, iters: int, out=None, compat=None):
        """Label marginals [n,L] after `iters` mean-field updates: a Potts
        compatibility of weight w_p, or, if compat [L,L] is given, the label
        compatibility matrix compat (row l: mu(l, .); w_p is then unused)."""
        want(unary, "unary", torch.float32, (self.n, None), self.device)
        L = unary.shape[1]
        if out is None:
            out = torch.empty_like(unary)
        if compat is not None:
            want(compat, "compat", torch.float32, (L, L), self.device)
            check(lib().sg_crf_meanfield_compat(self._h, ptr(unary), L, ptr(compat), iters,
                                                ptr(out), stream_ptr(self.device)),
                  "sg_crf_meanfield_compat")
            return out
        check(lib().sg_crf_meanfield(self._h, ptr(unary), L, ctypes.c_float(w_p),
                                     iters, ptr(out), stream_ptr(self.device)), "sg_crf_meanfield")
        return out

    def meanfield_backward(self, unary: torch.Tensor, compat: torch.Tensor, iters: int,
                           g_Q: torch.Tensor):
        """Gradients (g_unary [n,L], g_compat [L,L]) of a scalar whose
        gradient at meanfield(unary, compat=compat, iters)'s output is g_Q."""
        want(unary, "unary", torch.float32, (self.n, None), self.device)
        L = unary.shape[1]
        want(compat, "compat", torch.float32, (L, L), self.device)
        want(g_Q, "g_Q", torch.float32, (self.n, L), self.device)
        nb = lib().sg_crf_meanfield_compat_backward_ws_bytes(self.n, L, iters)
        if nb == 0:
            raise ValueError("invalid sizes for the mean-field backward")
        ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        g_u = torch.empty_like(unary)
        g_mu = torch.empty_like(compat)
        check(lib().sg_crf_meanfield_compat_backward(self._h, ptr(unary), L, ptr(compat), iters,
                                                     ptr(g_Q), ptr(g_u), ptr(g_mu), ptr(ws), nb,
                                                     stream_ptr(self.device)),
              "sg_crf_meanfield_compat_backward")
        return g_u, g_mu

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                torch.cuda.synchronize(self.device)
                lib().sg_lattice_destroy(h)
            except Exception:
                pass
            self._h = None


def render_footprint(grid: Grid, rays: torch.Tensor, params, touched: bool = False):
    """Per-ray (samples, distinct voxels, distinct blocks) and the touched map."""
    params = RenderParams.of(params)
    want(rays, "rays", torch.float32, (None, 6), grid.device)
    R = rays.shape[0]
    counts = torch.empty((R, 3), dtype=torch.int32, device=grid.device)
    tmap = torch.zeros(grid.n_blocks * 512, dtype=torch.uint8, device=grid.device) if touched else None
    prm = params.c()
    check(lib().sg_render_footprint(grid.handle, ptr(rays), R, ctypes.byref(prm), ptr(counts),
                                    ptr(tmap), stream_ptr(grid.device)), "sg_render_footprint")
    return (counts, tmap) if touched else counts


def rays_pinhole(cams: torch.Tensor, pix: torch.Tensor):
    """Unit rays [R,6] through pixel centres of pinhole cameras [n,16]."""
    want(cams, "cams", torch.float32, (None, 16))
    want(pix, "pix", torch.int32, (None, 3), cams.device)
    out = torch.empty((pix.shape[0], 6), dtype=torch.float32, device=cams.device)
    check(lib().sg_rays_pinhole(ptr(cams), cams.shape[0], ptr(pix), pix.shape[0], ptr(out),
                                stream_ptr(cams.device)), "sg_rays_pinhole")
    return out


def l2_loss_grad(pred, ref, lambda_d=0.1, lambda_n=0.05, with_loss=False, out=None):
    """Gradient (and optionally value) of the squared-L2 rendering loss."""
    R = pred["depth"].shape[0]
    C = pred["feat"].shape[1]
    dev = pred["depth"].device
    for k, shp in (("feat", (R, C)), ("depth", (R,)), ("normal", (R, 3))):
        want(pred[k], "pred." + k, torch.float32, shp, dev)
        want(ref[k], "ref." + k, torch.float32, shp, dev)
    if out is None:
        out = {"feat": torch.empty((R, C), dtype=torch.float32, device=dev),
               "depth": torch.empty(R, dtype=torch.float32, device=dev),
               "normal": torch.empty((R, 3), dtype=torch.float32, device=dev)}
    loss = torch.empty(1, dtype=torch.float32, device=dev) if with_loss else None
    check(lib().sg_l2_loss_grad(ptr(pred["feat"]) if C else None, ptr(ref["feat"]) if C else None,
                                ptr(pred["depth"]), ptr(ref["depth"]), ptr(pred["normal"]),
                                ptr(ref["normal"]), R, C, ctypes.c_float(lambda_d),
                                ctypes.c_float(lambda_n), ptr(out["feat"]) if C else None,
                                ptr(out["depth"]), ptr(out["normal"]), ptr(loss), stream_ptr(dev)),
          "sg_l2_loss_grad")
    return (out, loss) if with_loss else out


def optim_step(kind: int, param, grad, m, v, lr, b1, b2, eps, t):
    """In-place Adam (kind 0) or RMSProp (kind 1) step on float32 tensors."""
    want(param, "param", torch.float32)
    n = param.numel()
    for name, x in (("grad", grad), ("v", v)):
        want(x, name, torch.float32, None, param.device)
        if x.numel() != n:
            raise ValueError(f"{name} has {x.numel()} elements, expected {n}")
    if kind == 0:
        want(m, "m", torch.float32, None, param.device)
        if m.numel() != n:
            raise ValueError("m has the wrong size")
    check(lib().sg_optim_step(kind, ptr(param), ptr(grad), ptr(m) if kind == 0 else None, ptr(v), n,
                              ctypes.c_float(lr), ctypes.c_float(b1), ctypes.c_float(b2),
                              ctypes.c_float(eps), t, stream_ptr(param.device)), "sg_optim_step")


class SdfRender(torch.autograd.Function):
    """Differentiable render: vox -> (feat, depth, normal, wsum).

    The backward recomputes the per-sample values from the grid (only the
    sample lists of the march, which do not depend on vox, are kept from the
    forward) and accumulates into a freshly zeroed gradient tensor.
    """

    @staticmethod
    def forward(ctx, vox, grid, rays, params):
        _, _, lists = _lists("auto", grid, rays, params)
        out = render_forward(grid, vox.detach(), rays, params, lists=lists)
        ctx.grid, ctx.params, ctx.lists = grid, params, lists
        ctx.save_for_backward(vox, rays)
        ctx.mark_non_differentiable(out["nsamples"])
        return out["feat"], out["depth"], out["normal"], out["wsum"], out["nsamples"]

    @staticmethod
    def backward(ctx, g_feat, g_depth, g_normal, g_wsum, _g_ns):
        vox, rays = ctx.saved_tensors
        R = rays.shape[0]
        C = vox.shape[-1] - 1
        z = lambda *s: torch.zeros(s, dtype=torch.float32, device=vox.device)
        g_feat = z(R, C) if g_feat is None else g_feat.contiguous()
        g_depth = z(R) if g_depth is None else g_depth.contiguous()
        g_normal = z(R, 3) if g_normal is None else g_normal.contiguous()
        g_wsum = None if g_wsum is None else g_wsum.contiguous()
        grad = render_backward(ctx.grid, vox.detach(), rays, ctx.params, g_feat, g_depth,
                               g_normal, g_wsum, lists=ctx.lists)
        ctx.lists = None
        return grad, None, None, None


def render(grid: Grid, vox: torch.Tensor, rays: torch.Tensor, params):
    """Differentiable render; returns (feat, depth, normal, wsum, nsamples)."""
    return SdfRender.apply(vox, grid, rays, RenderParams.of(params))
