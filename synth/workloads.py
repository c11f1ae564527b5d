"""Named, seeded workloads: grid + parameters + rays + march settings.

  sphere_tiny   sphere r=0.5 m, h=1/64 m, band 4 voxels, one 64x48 camera
                (fx=fy=60) on a 1.5 m orbit, step h/2, t in [0,3], beta=h,
                128 samples max; second colour field as the photometric target.
  room_2cm      6x6x3 m room, 20 seeded primitives, h=2 cm, band 3 voxels;
                batches of random pixels from 30 seeded 640x480 poses
                (60 deg HFOV); step 1 cm, t in [0,12], beta=h, 128 max.
  room_1cm_sem  same room at h=1 cm with 16 one-hot semantic channels
                (C=19); 50 poses along a loop, 1296x968 (fx=fy=1122.4);
                step 0.5 cm, beta=h, 128 max.
  room_2cm_noisy  room_2cm with Gaussian noise (0.5 voxel on SDF, 0.1 on
                RGB) as the starting point and the clean grid as target.
  serving_grids three resident grids for render serving: the room at 2 cm,
                the same room at 1 cm (SDF + RGB), a second seeded room at
                2 cm; 30 seeded poses each.
"""
from __future__ import annotations

import numpy as np

from . import cameras, scenes

_CACHE: dict = {}


def params(step, t_near, t_far, beta, max_samples=128):
    return {"step": float(np.float32(step)), "t_near": float(t_near), "t_far": float(t_far),
            "beta": float(np.float32(beta)), "max_samples": int(max_samples)}


def sphere_tiny(seed=0):
    key = ("sphere_tiny", seed)
    if key not in _CACHE:
        sc = scenes.sphere_scene(h=1.0 / 64, radius=0.5, band_vox=4, seed=seed)
        cams = cameras.orbit_cams(seed=seed, n=1, radius=1.5, W=64, H=48, f=60.0)
        pix = cameras.frame_pixels(0, 64, 48)
        rays = cameras.pixel_rays(cams, pix)
        h = float(sc["h"])
        target = scenes.sphere_colour_field(sc["vox"], sc["block_coords"], h, sc["origin"],
                                            seed=seed + 1)
        _CACHE[key] = dict(sc, cams=cams, pix=pix, rays=rays, W=64, H=48,
                           params=params(h / 2, 0.0, 3.0, h, 128), target_vox=target)
    return _CACHE[key]


def room_2cm(seed=0, n_rays=65536, n_cams=30):
    key = ("room_2cm", seed, n_rays, n_cams)
    if key not in _CACHE:
        base = _room(seed, 0.02, 0)
        cams = cameras.room_cams(base["meta"]["objects"], seed=seed, n=n_cams, W=640, H=480)
        pix = cameras.random_pixels(n_cams, 640, 480, n_rays, seed=seed)
        rays = cameras.pixel_rays(cams, pix)
        _CACHE[key] = dict(base, cams=cams, pix=pix, rays=rays, W=640, H=480,
                           params=params(0.01, 0.0, 12.0, 0.02, 128))
    return _CACHE[key]


def room_2cm_target(seed=0):
    """Same geometry as room_2cm with a second texture seed (training target)."""
    key = ("room_2cm_target", seed)
    if key not in _CACHE:
        _CACHE[key] = scenes.room_scene(h=0.02, band_vox=3, seed=seed, texture_seed=seed + 100)
    return _CACHE[key]


def room_1cm_sem(seed=0, n_cams=50):
    key = ("room_1cm_sem", seed, n_cams)
    if key not in _CACHE:
        base = _room(seed, 0.01, 16)
        cams = cameras.trajectory_cams(seed=seed, n=n_cams, W=1296, H=968, f=1122.4)
        _CACHE[key] = dict(base, cams=cams, W=1296, H=968,
                           params=params(0.005, 0.0, 12.0, 0.01, 128))
    return _CACHE[key]


def room_2cm_noisy(seed=0, n_rays=262144):
    key = ("room_2cm_noisy", seed, n_rays)
    if key not in _CACHE:
        w = room_2cm(seed, n_rays=n_rays)
        noisy = scenes.perturb(w["vox"], w["h"], seed=seed)
        _CACHE[key] = dict(w, clean_vox=w["vox"], vox=noisy)
    return _CACHE[key]


def _room(seed, h, n_sem):
    key = ("room", seed, h, n_sem)
    if key not in _CACHE:
        _CACHE[key] = scenes.room_scene(h=h, band_vox=3, seed=seed, n_sem=n_sem)
    return _CACHE[key]


def serving_grids(seed=0):
    """[(scene dict, params, cams [30,16])] for the three resident grids."""
    key = ("serving", seed)
    if key not in _CACHE:
        out = []
        for sd, h in ((seed, 0.02), (seed, 0.01), (seed + 1, 0.02)):
            sc = _room(sd, h, 0)
            cams = cameras.room_cams(sc["meta"]["objects"], seed=sd, n=30, W=640, H=480)
            out.append((sc, params(h / 2, 0.0, 12.0, h, 128), cams))
        _CACHE[key] = out
    return _CACHE[key]


def room_depth_frames(seed=0, n_frames=10, W=640, H=480, n_sem=0):
    """Depth and RGB(+semantic) images of the 2 cm room from seeded poses
    (the input of block allocation and fusion)."""
    key = ("room_frames", seed, n_frames, W, H, n_sem)
    if key not in _CACHE:
        base = _room(seed, 0.02, 0)
        cams = cameras.room_cams(base["meta"]["objects"], seed=seed + 7, n=n_frames, W=W, H=H)
        depth, feat = scenes.room_frames(base["meta"], cams, W, H, n_sem=n_sem)
        _CACHE[key] = {"cams": cams, "depth": depth, "feat": feat, "W": W, "H": H,
                       "h": np.float32(0.02), "origin": np.zeros(3, np.float32), "room": base}
    return _CACHE[key]
