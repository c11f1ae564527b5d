"""Seeded synthetic scenes stored as sparse 8^3-block SDF grids.

Input generation only: analytic signed-distance shapes sampled at voxel
positions, blocks kept inside a band around the surface, colour / label
fields.  Nothing here renders; the renderer and the oracle both consume the
arrays these functions return.

Grid layout shared by every consumer: voxel with global integer index i
sits at ``origin + i * h``; block ``b = floor(i / 8)``; local index
``lx + 8*ly + 64*lz``; parameters ``vox[n_blocks, 512, 1 + C]`` float32 with
channel 0 the SDF.

Stand-ins: the paper evaluates on ScanNet and 7-Scenes rooms with 1.5 cm
voxels and 8^3 blocks.  These generators produce rooms of the same kind of
shape (a box room with furniture-sized primitives) at 2 cm and 1 cm, and a
sphere for the tiny case.
"""
from __future__ import annotations

import numpy as np

SEED_SCENE = 1
SEED_POSES = 2
SEED_RAYS = 3
SEED_NOISE = 4
SEED_ARRIVALS = 5

_L = np.arange(512)
LOCAL_XYZ = np.stack([_L % 8, (_L // 8) % 8, _L // 64], axis=-1)  # [512,3]


def voxel_positions(block_coords, h, origin):
    """World positions [n,512,3] (float64) of every voxel of the given blocks."""
    bc = np.asarray(block_coords, np.int64).reshape(-1, 3)
    gi = bc[:, None, :] * 8 + LOCAL_XYZ[None, :, :]
    return np.asarray(origin, np.float64)[None, None, :] + h * gi.astype(np.float64)


# --- exact SDFs of primitives (p given as a tuple of per-axis arrays) --------

def _split(p):
    p = np.asarray(p, np.float64)
    return p[..., 0], p[..., 1], p[..., 2]


def sd_sphere(p, c, r):
    x, y, z = _split(p) if not isinstance(p, tuple) else p
    return np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) - r


def sd_box(p, c, half):
    x, y, z = _split(p) if not isinstance(p, tuple) else p
    qx = np.abs(x - c[0]) - half[0]
    qy = np.abs(y - c[1]) - half[1]
    qz = np.abs(z - c[2]) - half[2]
    outside = np.sqrt(np.maximum(qx, 0.0) ** 2 + np.maximum(qy, 0.0) ** 2
                      + np.maximum(qz, 0.0) ** 2)
    inside = np.minimum(np.maximum(np.maximum(qx, qy), qz), 0.0)
    return outside + inside


def sd_cylinder_z(p, c, r, half_h):
    x, y, z = _split(p) if not isinstance(p, tuple) else p
    dxy = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2) - r
    dz = np.abs(z - c[2]) - half_h
    return (np.minimum(np.maximum(dxy, dz), 0.0)
            + np.sqrt(np.maximum(dxy, 0.0) ** 2 + np.maximum(dz, 0.0) ** 2))


def _allocate(sdf_fn, lo, hi, h, origin, band, chunk=4096):
    """Blocks (within the block-box [lo, hi]) holding a voxel with |SDF| <= band.

    Uses that exact SDFs (and their min) are 1-Lipschitz to prune by the
    block centre before evaluating every voxel.  Returns block coords in
    lexicographic (z, y, x) scan order.
    """
    zz, yy, xx = np.meshgrid(np.arange(lo[2], hi[2] + 1), np.arange(lo[1], hi[1] + 1),
                             np.arange(lo[0], hi[0] + 1), indexing="ij")
    cand = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=-1).astype(np.int64)
    centres = np.asarray(origin)[None] + h * (cand * 8 + 3.5)
    reach = band + 3.5 * np.sqrt(3.0) * h + 1e-9
    keep = np.abs(sdf_fn(centres)) <= reach
    cand = cand[keep]
    out = []
    for s in range(0, cand.shape[0], chunk):
        bc = cand[s:s + chunk]
        d = sdf_fn(voxel_positions(bc, h, origin))
        out.append(bc[np.any(np.abs(d) <= band, axis=1)])
    return np.concatenate(out, axis=0).astype(np.int32) if out else np.zeros((0, 3), np.int32)


# --- C1: sphere ---------------------------------------------------------------

def sphere_scene(h=1.0 / 64, radius=0.5, band_vox=4, seed=0, C=3):
    """Sphere |x| - radius centred at the origin in the [-1,1]^3 cube.

    Colour channel c(x) = 1/2 + 1/2 sin(2 pi f_c . x + phi_c) with seeded
    frequency vectors (0.5-2 cycles/m) and phases.
    """
    rng = np.random.default_rng([seed, SEED_SCENE])
    origin = np.zeros(3)
    nb = int(np.ceil(1.0 / (8 * h)))
    fn = lambda p: sd_sphere(p, np.zeros(3), radius)
    bc = _allocate(fn, (-nb, -nb, -nb), (nb - 1, nb - 1, nb - 1), h, origin, band_vox * h)
    pos = voxel_positions(bc, h, origin)
    freq = rng.uniform(0.5, 2.0, size=C)[:, None] * _unit(rng.normal(size=(C, 3)))
    phase = rng.uniform(0, 2 * np.pi, size=C)
    vox = np.empty((bc.shape[0], 512, 1 + C), np.float32)
    vox[..., 0] = fn(pos)
    for c in range(C):
        vox[..., 1 + c] = 0.5 + 0.5 * np.sin(2 * np.pi * pos @ freq[c] + phase[c])
    return {"name": "sphere", "block_coords": bc, "vox": vox, "h": np.float32(h),
            "origin": origin.astype(np.float32), "C": C, "radius": radius}


def sphere_colour_field(vox, block_coords, h, origin, seed, C=3):
    """A second seeded colour field on the same sphere grid (training target)."""
    rng = np.random.default_rng([seed, SEED_SCENE, 7])
    pos = voxel_positions(block_coords, h, origin)
    freq = rng.uniform(0.5, 2.0, size=C)[:, None] * _unit(rng.normal(size=(C, 3)))
    phase = rng.uniform(0, 2 * np.pi, size=C)
    out = vox.copy()
    for c in range(C):
        out[..., 1 + c] = 0.5 + 0.5 * np.sin(2 * np.pi * pos @ freq[c] + phase[c])
    return out


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


# --- C2 / C3: synthetic room ----------------------------------------------------

ROOM_LO = np.array([0.0, 0.0, 0.0])
ROOM_HI = np.array([6.0, 6.0, 3.0])


def room_objects(seed=0, n_objects=20):
    """Seeded furniture: boxes, spheres and vertical cylinders resting on the floor."""
    rng = np.random.default_rng([seed, SEED_SCENE])
    objs = []
    for _ in range(n_objects):
        kind = int(rng.integers(0, 3))
        size = rng.uniform(0.2, 1.2)
        if kind == 0:  # box
            half = rng.uniform(0.1, 0.6, size=3)
            half[2] = size / 2
            xy = rng.uniform(ROOM_LO[:2] + half[:2] + 0.05, ROOM_HI[:2] - half[:2] - 0.05)
            objs.append(("box", np.array([xy[0], xy[1], half[2]]), half))
        elif kind == 1:  # sphere
            r = size / 2
            xy = rng.uniform(ROOM_LO[:2] + r + 0.05, ROOM_HI[:2] - r - 0.05)
            objs.append(("sphere", np.array([xy[0], xy[1], r]), r))
        else:  # cylinder
            r = rng.uniform(0.1, 0.6)
            hh = size / 2
            xy = rng.uniform(ROOM_LO[:2] + r + 0.05, ROOM_HI[:2] - r - 0.05)
            objs.append(("cyl", np.array([xy[0], xy[1], hh]), (r, hh)))
    base = rng.uniform(0.1, 0.9, size=(n_objects + 3, 3))
    tex_f = rng.uniform(1.0, 4.0, size=(n_objects + 3, 3))[..., None] * _unit(
        rng.normal(size=(n_objects + 3, 3, 3)))
    tex_p = rng.uniform(0, 2 * np.pi, size=(n_objects + 3, 3))
    labels = np.concatenate([[0, 1, 2], rng.integers(3, 16, size=n_objects)])
    return {"objects": objs, "base": base, "tex_f": tex_f, "tex_p": tex_p, "labels": labels}


def _room_min(p, objs):
    """(SDF, nearest part id) of the room at points p [...,3].

    Parts: 0 floor, 1 walls, 2 ceiling (free space positive inside the
    room; outside it all three take the exact box distance), then objects.
    """
    x, y, z = _split(p)
    room = -sd_box((x, y, z), (ROOM_LO + ROOM_HI) / 2, (ROOM_HI - ROOM_LO) / 2)
    outside = room < 0
    walls = np.minimum(np.minimum(x - ROOM_LO[0], ROOM_HI[0] - x),
                       np.minimum(y - ROOM_LO[1], ROOM_HI[1] - y))
    best = np.where(outside, room, z - ROOM_LO[2])
    arg = np.zeros(best.shape, np.int64)
    for pid, d in ((1, np.where(outside, room, walls)),
                   (2, np.where(outside, room, ROOM_HI[2] - z))):
        better = d < best
        best = np.where(better, d, best)
        arg[better] = pid
    for j, (kind, c, prm) in enumerate(objs):
        if kind == "box":
            d = sd_box((x, y, z), c, prm)
        elif kind == "sphere":
            d = sd_sphere((x, y, z), c, prm)
        else:
            d = sd_cylinder_z((x, y, z), c, prm[0], prm[1])
        better = d < best
        best = np.where(better, d, best)
        arg[better] = 3 + j
    return best, arg


def room_sdf(p, objs):
    return _room_min(p, objs)[0]


def part_features(pos, near, meta, n_sem=0):
    """RGB (+ n_sem one-hot semantic logits) of room part `near` at points pos."""
    out = np.empty(pos.shape[:-1] + (3 + n_sem,), np.float32)
    for ch in range(3):
        f = meta["tex_f"][near, ch]
        ph = 2 * np.pi * (pos[..., 0] * f[..., 0] + pos[..., 1] * f[..., 1]
                          + pos[..., 2] * f[..., 2]) + meta["tex_p"][near, ch]
        out[..., ch] = np.clip(meta["base"][near, ch] + 0.2 * np.sin(ph), 0.0, 1.0)
    if n_sem:
        out[..., 3:] = (meta["labels"][near][..., None] == np.arange(n_sem)).astype(np.float32)
    return out


def room_frames(meta, cams, W, H, n_sem=0, max_depth=20.0):
    """Depth and feature images of the analytic room seen by cams [F,16]:
    depth [F,H,W] float32 (z in the camera frame of the first surface,
    found by sphere tracing the exact SDF in float64; NaN where nothing is
    hit) and features [F,H,W,3+n_sem] (RGB, one-hot semantics) of the part
    hit."""
    from .cameras import frame_pixels, pixel_rays
    objs = meta["objects"]
    F = cams.shape[0]
    depth = np.full((F, H, W), np.nan, np.float32)
    feat = np.zeros((F, H, W, 3 + n_sem), np.float32)
    for i in range(F):
        r = pixel_rays(cams, frame_pixels(i, W, H)).astype(np.float64)
        o, d = r[:, :3], r[:, 3:]
        t = np.zeros(len(r))
        act = np.ones(len(r), bool)
        hit = np.zeros(len(r), bool)
        for _ in range(400):
            idx = np.flatnonzero(act)
            if idx.size == 0:
                break
            sd = room_sdf(o[idx] + t[idx, None] * d[idx], objs)
            t[idx] += sd
            done = sd < 1e-6
            hit[idx[done]] = True
            act[idx[done | (t[idx] > max_depth)]] = False
        R = cams[i, 4:].astype(np.float64).reshape(3, 4)[:, :3]
        z = t * (d @ R[:, 2])
        pts = o + t[:, None] * d
        _, near = _room_min(pts, objs)
        depth[i].reshape(-1)[hit] = z[hit].astype(np.float32)
        feat[i].reshape(-1, 3 + n_sem)[hit] = part_features(pts[hit], near[hit], meta, n_sem)
    return depth, feat


def room_scene(h=0.02, band_vox=3, seed=0, n_objects=20, n_sem=0, texture_seed=None):
    """6 x 6 x 3 m box room with seeded furniture, exact union SDF.

    Features: RGB of the nearest part (seeded base colour + 0.2-amplitude
    sinusoid texture, clamped to [0,1]), then optionally n_sem one-hot
    semantic logits of that part's label.  texture_seed re-draws only the
    texture (same geometry) for training targets.
    """
    meta = room_objects(seed, n_objects)
    objs = meta["objects"]
    origin = np.zeros(3)
    band = band_vox * h
    bs = 8 * h
    lo = np.floor((ROOM_LO - band - bs) / bs).astype(int)
    hi = np.ceil((ROOM_HI + band + bs) / bs).astype(int)
    zz, yy, xx = np.meshgrid(np.arange(lo[2], hi[2] + 1), np.arange(lo[1], hi[1] + 1),
                             np.arange(lo[0], hi[0] + 1), indexing="ij")
    cand = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=-1).astype(np.int64)
    centres = origin[None] + h * (cand * 8 + 3.5)
    cand = cand[np.abs(room_sdf(centres, objs)) <= band + 3.5 * np.sqrt(3.0) * h + 1e-9]
    if texture_seed is not None:
        alt = room_objects(texture_seed, n_objects)
        meta = dict(meta, base=alt["base"], tex_f=alt["tex_f"], tex_p=alt["tex_p"])
    C = 3 + n_sem
    blocks, chunks = [], []
    for s in range(0, cand.shape[0], 2048):
        bc = cand[s:s + 2048]
        pos = voxel_positions(bc, h, origin)
        sdf, near = _room_min(pos, objs)
        keep = np.any(np.abs(sdf) <= band, axis=1)
        bc, pos, sdf, near = bc[keep], pos[keep], sdf[keep], near[keep]
        v = np.empty((bc.shape[0], 512, 1 + C), np.float32)
        v[..., 0] = sdf
        v[..., 1:] = part_features(pos, near, meta, n_sem)
        blocks.append(bc.astype(np.int32))
        chunks.append(v)
    bc = np.concatenate(blocks, axis=0)
    vox = np.concatenate(chunks, axis=0)
    return {"name": f"room_h{h}", "block_coords": bc, "vox": vox, "h": np.float32(h),
            "origin": origin.astype(np.float32), "C": C, "meta": meta}


def perturb(vox, h, seed, sdf_sigma_vox=0.5, feat_sigma=0.1):
    """Seeded Gaussian noise on SDF (in voxels) and features, no clamp."""
    rng = np.random.default_rng([seed, SEED_NOISE])
    out = vox.copy()
    out[..., 0] += rng.normal(0.0, sdf_sigma_vox * float(h), size=vox.shape[:2]).astype(np.float32)
    out[..., 1:] += rng.normal(0.0, feat_sigma, size=vox[..., 1:].shape).astype(np.float32)
    return out
