"""Shared helpers of the GPU parity tests (test infrastructure)."""
import numpy as np
import torch

# Tolerances (relative to the magnitude sum_k |w_k v_k| of each output
# element, resp. the sum of absolute values of every term of each gradient
# element; see the design notes for the derivation).
RTOL_FWD = 1e-5
RTOL_BWD = 1e-4
ATOL = 1e-30


def dev():
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def make_grid(w):
    import paper_2305_13220_amd as sg
    bc = to_dev(w["block_coords"], torch.int32)
    g = sg.Grid(bc, float(w["h"]), tuple(float(x) for x in w["origin"]))
    return g


def assert_close_mag(got, want, mag, rtol, what, atol=ATOL):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    mag = np.asarray(mag, np.float64)
    err = np.abs(got - want)
    bound = rtol * mag + atol
    bad = err > bound
    if bad.any():
        i = np.flatnonzero(bad.ravel())[:5]
        raise AssertionError(
            f"{what}: {bad.sum()} of {bad.size} elements out of tolerance; first: "
            + ", ".join(f"[{j}] got {got.ravel()[j]:.9g} want {want.ravel()[j]:.9g} "
                        f"mag {mag.ravel()[j]:.3g}" for j in i))


def check_forward(out_gpu, out_or, rows=None, what="forward"):
    """Compare a GPU forward (torch dict) with an oracle forward (with mags)."""
    sel = slice(None) if rows is None else rows
    ns = out_gpu["nsamples"].cpu().numpy()[sel]
    np.testing.assert_array_equal(ns, out_or["nsamples"], err_msg=f"{what}: nsamples")
    for k in ("feat", "depth", "normal", "wsum"):
        g = out_gpu[k].cpu().numpy()[sel]
        assert_close_mag(g, out_or[k], out_or["mag_" + k], RTOL_FWD, f"{what}: {k}")
    empty = ns == 0
    for k in ("feat", "depth", "normal", "wsum"):
        g = out_gpu[k].cpu().numpy()[sel]
        assert not np.any(g[empty]), f"{what}: {k} of an empty ray is not exactly zero"
