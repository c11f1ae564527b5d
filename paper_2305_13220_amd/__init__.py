"""Sparse-dense SDF grid renderer for AMD gfx950 (Dong et al., CVPR 2023).

Global-sparse / local-dense voxel grid: allocated 8^3 blocks found through a
collision-free spatial hash, per-voxel SDF + features, differentiable volume
rendering (ray march, trilinear interpolation with closed-form gradient,
Laplace-CDF density, alpha compositing) and its backward pass, all as HIP
kernels behind the C ABI in include/sgrid.h.  This package is the thin
Python binding plus the training / serving loops around it.
"""
from ._lib import SgridError, lib  # noqa: F401
from .grid import (  # noqa: F401
    Grid, Lattice, RenderParams, SdfRender, crf_label_loss, crf_property_loss, l2_loss_grad, optim_step, rays_pinhole, render,
    alloc_blocks, denoise, eikonal, fuse, list_bytes, march, query, query_backward, render_backward, surface_points, uniform_points, render_footprint, render_forward, render_l2_step,
)

__all__ = ["Grid", "Lattice", "RenderParams", "SdfRender", "SgridError", "l2_loss_grad", "optim_step",
           "rays_pinhole", "render", "render_backward", "render_footprint", "render_forward",
           "render_l2_step", "list_bytes", "march", "query", "query_backward", "surface_points", "uniform_points", "eikonal", "alloc_blocks", "fuse", "denoise", "crf_label_loss", "crf_property_loss", "lib"]
