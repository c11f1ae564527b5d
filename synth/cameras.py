"""Seeded pinhole cameras, poses and ray batches (input generation only).

Cameras are float32 rows [fx, fy, cx, cy, R(3x4 camera-to-world, row-major)]
with OpenCV axes (x right, y down, z forward).  Rays are float32 [R,6]
(origin, unit direction) through pixel centres.
"""
from __future__ import annotations

import numpy as np

from .scenes import SEED_POSES, SEED_RAYS, ROOM_HI, ROOM_LO, room_sdf


def look_at(eye, target, up=(0.0, 0.0, 1.0)):
    """3x4 camera-to-world [R | t] looking from eye to target (OpenCV axes)."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    x = np.cross(z, np.asarray(up, np.float64))
    if np.linalg.norm(x) < 1e-8:
        x = np.cross(z, np.array([1.0, 0.0, 0.0]))
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    M = np.zeros((3, 4))
    M[:, 0], M[:, 1], M[:, 2], M[:, 3] = x, y, z, eye
    return M


def make_cams(poses, fx, fy, cx, cy):
    cams = np.zeros((len(poses), 16), np.float32)
    for i, M in enumerate(poses):
        cams[i, :4] = (fx, fy, cx, cy)
        cams[i, 4:] = np.asarray(M, np.float32).ravel()
    return cams


def orbit_cams(seed=0, n=1, radius=1.5, W=64, H=48, f=60.0):
    """Cameras on a sphere of `radius` around the origin looking at it."""
    rng = np.random.default_rng([seed, SEED_POSES])
    poses = []
    for _ in range(n):
        az = rng.uniform(0, 2 * np.pi)
        el = np.deg2rad(rng.uniform(-30, 30))
        eye = radius * np.array([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)])
        poses.append(look_at(eye, np.zeros(3)))
    return make_cams(poses, f, f, W / 2, H / 2)


def room_cams(objs, seed=0, n=30, W=640, H=480, hfov_deg=60.0):
    """Seeded poses inside the room: eye in [0.8,5.2]^2 x [1,2] with SDF >= 0.3 m."""
    rng = np.random.default_rng([seed, SEED_POSES])
    f = (W / 2) / np.tan(np.deg2rad(hfov_deg) / 2)
    poses = []
    while len(poses) < n:
        eye = rng.uniform([0.8, 0.8, 1.0], [5.2, 5.2, 2.0])
        if room_sdf(eye[None], objs)[0] < 0.3:
            continue
        tgt = rng.uniform(ROOM_LO + 0.3, ROOM_HI - 0.3)
        if np.linalg.norm(tgt - eye) < 0.5:
            continue
        poses.append(look_at(eye, tgt))
    return make_cams(poses, f, f, W / 2, H / 2)


def trajectory_cams(seed=0, n=50, W=1296, H=968, f=1122.4):
    """Poses along a smooth closed Catmull-Rom loop through 6 seeded waypoints."""
    rng = np.random.default_rng([seed, SEED_POSES, 3])
    centre = (ROOM_LO + ROOM_HI) / 2
    ang = np.sort(rng.uniform(0, 2 * np.pi, 6))
    rad = rng.uniform(1.2, 2.2, 6)
    way = np.stack([centre[0] + rad * np.cos(ang), centre[1] + rad * np.sin(ang),
                    rng.uniform(1.2, 1.8, 6)], axis=-1)
    poses = []
    for j in range(n):
        s = 6.0 * j / n
        i = int(np.floor(s))
        u = s - i
        p0, p1, p2, p3 = (way[(i + d) % 6] for d in (-1, 0, 1, 2))
        eye = 0.5 * ((2 * p1) + (-p0 + p2) * u + (2 * p0 - 5 * p1 + 4 * p2 - p3) * u * u
                     + (-p0 + 3 * p1 - 3 * p2 + p3) * u ** 3)
        tgt = centre + rng.uniform(-0.5, 0.5, 3) * np.array([1, 1, 0.3])
        poses.append(look_at(eye, tgt))
    return make_cams(poses, f, f, W / 2, H / 2)


def random_pixels(n_cams, W, H, n_rays, seed=0):
    """[R,3] int32 (camera, u, v), uniform and seeded."""
    rng = np.random.default_rng([seed, SEED_RAYS])
    pix = np.empty((n_rays, 3), np.int32)
    pix[:, 0] = rng.integers(0, n_cams, n_rays)
    pix[:, 1] = rng.integers(0, W, n_rays)
    pix[:, 2] = rng.integers(0, H, n_rays)
    return pix


def frame_pixels(cam, W, H):
    """All pixels of one frame, row-major: [W*H,3] int32."""
    v, u = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    pix = np.empty((W * H, 3), np.int32)
    pix[:, 0] = cam
    pix[:, 1] = u.ravel()
    pix[:, 2] = v.ravel()
    return pix


def pixel_rays(cams, pix):
    """float32 [R,6] rays through pixel centres (computed in float64, rounded once)."""
    cams = np.asarray(cams, np.float64).reshape(-1, 16)
    pix = np.asarray(pix)
    K = cams[pix[:, 0]]
    M = K[:, 4:].reshape(-1, 3, 4)
    x = (pix[:, 1] + 0.5 - K[:, 2]) / K[:, 0]
    y = (pix[:, 2] + 0.5 - K[:, 3]) / K[:, 1]
    dc = np.stack([x, y, np.ones_like(x)], axis=-1)
    d = np.einsum("rij,rj->ri", M[:, :, :3], dc)
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return np.concatenate([M[:, :, 3], d], axis=-1).astype(np.float32)
