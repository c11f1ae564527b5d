"""Permutohedral-lattice filter and mean-field CRF update (Sec. 3.5.3) on the
GPU against the oracle.

Bars: number of lattice vertices bit-exact (the simplex vertices are
float32 decisions on both sides); filter output within 1e-5 of the oracle's
filter of |values| (all weights are positive); mean-field marginals within
1e-5 after each of 3 updates."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


def _sg():
    import paper_2305_13220_amd as sg
    return sg


def _surface_features(n_sem=16, n=20000, seed=0):
    """CRF nodes on the room's surface: points of a depth frame, features
    (xyz / 20 cm, rgb / 0.3), unary from noisy one-hot labels."""
    from synth import cameras, workloads
    fr = workloads.room_depth_frames(n_frames=2, W=160, H=120, n_sem=n_sem)
    pix = np.concatenate([cameras.frame_pixels(i, 160, 120) for i in range(2)])
    d = fr["depth"].reshape(-1)
    ok = np.isfinite(d)
    rays = cameras.pixel_rays(fr["cams"], pix).astype(np.float64)
    R = fr["cams"][pix[:, 0], 4:].astype(np.float64).reshape(-1, 3, 4)[:, :, 2]
    t = d / np.einsum("ij,ij->i", rays[:, 3:], R)
    xyz = rays[:, :3] + t[:, None] * rays[:, 3:]
    feat = fr["feat"].reshape(-1, 3 + n_sem)
    rng = np.random.default_rng(seed)
    idx = rng.choice(np.flatnonzero(ok), min(n, ok.sum()), replace=False)
    pos = np.concatenate([xyz[idx] / 0.2, feat[idx, :3] / 0.3], 1).astype(np.float32)
    lab = feat[idx, 3:].copy()
    flip = rng.random(len(idx)) < 0.1  # wrong labels the pairwise term should correct
    lab[flip] = np.eye(n_sem)[rng.integers(0, n_sem, flip.sum())]
    unary = (-np.log(np.clip(lab * 0.7 + 0.3 / n_sem + rng.uniform(0, 0.2, (len(idx), n_sem)),
                             1e-6, None))).astype(np.float32)
    return pos, unary


@pytest.mark.parametrize("d", [1, 3, 6])
def test_lattice_filter_matches_oracle(d):
    sg = _sg()
    rng = np.random.default_rng(d)
    pos = rng.normal(scale=4.0, size=(20000, d)).astype(np.float32)
    val = rng.normal(size=(20000, 5)).astype(np.float32)
    lat = sg.Lattice(to_dev(pos), max_values=8)
    out = lat.filter(to_dev(val)).cpu().numpy()
    want, nv = oracle.lattice_filter(pos, val)
    mag, _ = oracle.lattice_filter(pos, np.abs(val))
    assert lat.n_vertices == nv
    bad = np.abs(out - want) > 1e-5 * mag + 1e-30
    assert not bad.any(), f"{bad.sum()} values out of tolerance"


def test_crf_meanfield_on_surface_samples():
    sg = _sg()
    pos, unary = _surface_features()
    lat = sg.Lattice(to_dev(pos), max_values=16)
    _, nv = oracle.lattice_filter(pos, np.ones((len(pos), 1)))
    assert lat.n_vertices == nv
    for it in (0, 1, 3):
        Q = lat.meanfield(to_dev(unary), 5.0, it).cpu().numpy()
        want = oracle.crf_meanfield(pos, unary, 5.0, it)
        err = np.abs(Q - want).max()
        assert err <= 1e-5, f"iteration {it}: {err}"
    # the pairwise term changes the labels of some nodes
    q0 = oracle.crf_meanfield(pos, unary, 5.0, 0)
    assert (q0.argmax(1) != want.argmax(1)).mean() > 0.01


def test_lattice_invalid_inputs():
    sg = _sg()
    pos = np.zeros((10, 3), np.float32)
    pos[3, 1] = np.nan
    with pytest.raises(sg.SgridError, match="finite"):
        sg.Lattice(to_dev(pos))
    with pytest.raises(sg.SgridError):
        sg.Lattice(to_dev(np.zeros((10, 17), np.float32)))
    lat = sg.Lattice(to_dev(np.zeros((10, 3), np.float32)), max_values=2)
    with pytest.raises(sg.SgridError):
        lat.filter(to_dev(np.zeros((10, 3), np.float32)))
    assert lat.n_vertices == 4
