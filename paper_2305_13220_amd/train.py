"""Grid refinement by volume rendering (Sec. 3.5.1, 3.5.4) on one GPU.

A training step: draw a batch of (camera, pixel) pairs, make their rays
(`sg_rays_pinhole`), run the fused forward + squared-L2 colour/depth/normal
losses + backward (`sg_render_l2_step`) into a zeroed gradient, and update
the voxel parameters with Adam or RMSProp (`sg_optim_step`).  Reference
colour, depth and normal per pixel are given as images (one per camera).

Random pixel draws come from torch's generator on the device; they are the
input of the step, not part of its arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from .grid import Grid, RenderParams, optim_step, rays_pinhole, render_forward, render_l2_step


@dataclass
class TrainConfig:
    rays_per_step: int = 262144
    lr: float = 1e-3
    optimizer: str = "adam"  # "adam" or "rmsprop" (the paper's, Sec. 3.5.4)
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    lambda_d: float = 0.1
    lambda_n: float = 0.05
    seed: int = 0


def render_reference_images(grid: Grid, vox: torch.Tensor, cams: torch.Tensor, W: int, H: int,
                            params, chunk: int = 1 << 20):
    """Full-frame renders of every camera: dict feat [n,H*W,C], depth, normal."""
    n = cams.shape[0]
    C = vox.shape[-1] - 1
    dev = vox.device
    feat = torch.empty((n, H * W, C), dtype=torch.float32, device=dev)
    depth = torch.empty((n, H * W), dtype=torch.float32, device=dev)
    normal = torch.empty((n, H * W, 3), dtype=torch.float32, device=dev)
    v, u = torch.meshgrid(torch.arange(H, device=dev), torch.arange(W, device=dev), indexing="ij")
    uv = torch.stack([u.reshape(-1), v.reshape(-1)], -1).to(torch.int32)
    for c in range(n):
        for s in range(0, H * W, chunk):
            e = min(H * W, s + chunk)
            pix = torch.cat([torch.full((e - s, 1), c, dtype=torch.int32, device=dev), uv[s:e]], 1)
            out = render_forward(grid, vox, rays_pinhole(cams, pix.contiguous()), params)
            feat[c, s:e] = out["feat"]
            depth[c, s:e] = out["depth"]
            normal[c, s:e] = out["normal"]
    return {"feat": feat, "depth": depth, "normal": normal}


class Trainer:
    """Optimises vox (float32 [n,512,1+C], updated in place) against reference images."""

    def __init__(self, grid: Grid, vox: torch.Tensor, cams: torch.Tensor, W: int, H: int, params,
                 ref_images, cfg: TrainConfig = TrainConfig()):
        self.grid, self.vox, self.cams, self.W, self.H = grid, vox, cams, W, H
        self.params = RenderParams.of(params)
        self.ref = ref_images
        self.cfg = cfg
        dev = vox.device
        self.grad = torch.zeros_like(vox)
        self.m = torch.zeros_like(vox) if cfg.optimizer == "adam" else None
        self.v = torch.zeros_like(vox)
        self.t = 0
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(cfg.seed)
        R = cfg.rays_per_step
        C = vox.shape[-1] - 1
        self.out = {"feat": torch.empty((R, C), device=dev), "depth": torch.empty(R, device=dev),
                    "normal": torch.empty((R, 3), device=dev), "wsum": torch.empty(R, device=dev),
                    "nsamples": torch.empty(R, dtype=torch.int32, device=dev)}
        self.loss_ray = None

    def sample(self):
        R, dev = self.cfg.rays_per_step, self.vox.device
        cam = torch.randint(0, self.cams.shape[0], (R,), generator=self.gen, device=dev)
        px = torch.randint(0, self.W * self.H, (R,), generator=self.gen, device=dev)
        pix = torch.stack([cam, px % self.W, px // self.W], -1).to(torch.int32).contiguous()
        ref = {k: v[cam, px].contiguous() for k, v in self.ref.items()}
        return pix, ref

    def step(self, with_loss: bool = False):
        pix, ref = self.sample()
        rays = rays_pinhole(self.cams, pix)
        self.grad.zero_()
        res = render_l2_step(self.grid, self.vox, rays, self.params, ref, self.cfg.lambda_d,
                             self.cfg.lambda_n, grad_vox=self.grad, out=self.out,
                             with_loss=with_loss)
        self.t += 1
        kind = 0 if self.cfg.optimizer == "adam" else 1
        optim_step(kind, self.vox, self.grad, self.m, self.v, self.cfg.lr, self.cfg.beta1,
                   self.cfg.beta2, self.cfg.eps, self.t)
        return res[2].sum() if with_loss else None
