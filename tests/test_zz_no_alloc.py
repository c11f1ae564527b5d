"""The allocation-free mean-field gradient (its workspace is a fixed array
inside the library) against the caller-workspace entry point, through the C
ABI: two calls in a row, the second on a smaller lattice, plus the host-side
rejections (a size beyond the array, an output overlapping the upstream
gradient).

Bars, as for the caller-workspace call against the oracle: g_compat within
1e-3 and g_unary within 1e-4 of the largest magnitude (the two calls run the
same kernels; only the order of the splat's float atomics differs)."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


def _noalloc(lat, unary, mu, iters, gQ):
    from paper_2305_13220_amd import _lib
    n, L = unary.shape
    g_u = torch.empty_like(unary)
    g_mu = torch.empty_like(mu)
    rc = _lib.lib().sg_crf_meanfield_compat_backward_noalloc(
        lat._h, _lib.ptr(unary), L, _lib.ptr(mu), iters, _lib.ptr(gQ), _lib.ptr(g_u),
        _lib.ptr(g_mu), _lib.stream_ptr(unary.device))
    _lib.check(rc, "sg_crf_meanfield_compat_backward_noalloc")
    return g_u, g_mu


def _case(n, d, L, iters, seed):
    import paper_2305_13220_amd as sg
    rng = np.random.default_rng(seed)
    pos = rng.normal(scale=1.5, size=(n, d)).astype(np.float32)
    unary = to_dev(rng.normal(size=(n, L)).astype(np.float32))
    mu = to_dev((-2.0 * np.eye(L) + 0.5 * rng.random((L, L))).astype(np.float32))
    gQ = to_dev(rng.normal(size=(n, L)).astype(np.float32))
    lat = sg.Lattice(to_dev(pos), max_values=L)
    return lat, unary, mu, gQ


def test_noalloc_matches_workspace_call_twice():
    from paper_2305_13220_amd import _lib
    assert _lib.lib().sg_crf_meanfield_compat_backward_noalloc_max_bytes() == 64 << 20
    # second call smaller: a stale tail of the first call's workspace must not matter
    for n, d, L, iters, seed in [(20000, 6, 16, 3, 71), (3001, 3, 5, 2, 72)]:
        print(f"case n={n} d={d} L={L} iters={iters}", flush=True)
        lat, unary, mu, gQ = _case(n, d, L, iters, seed)
        want_u, want_mu = lat.meanfield_backward(unary, mu, iters, gQ)
        g_u, g_mu = _noalloc(lat, unary, mu, iters, gQ)
        torch.cuda.synchronize()
        want_u, want_mu = want_u.cpu().numpy(), want_mu.cpu().numpy()
        g_u, g_mu = g_u.cpu().numpy(), g_mu.cpu().numpy()
        assert np.abs(g_mu - want_mu).max() <= 1e-3 * np.abs(want_mu).max()
        assert np.abs(g_u - want_u).max() <= 1e-4 * np.abs(want_u).max()
        del lat


def test_noalloc_rejects_oversize_and_overlap():
    from paper_2305_13220_amd import _lib
    lat, unary, mu, gQ = _case(3001, 3, 32, 1, 73)
    n, L = unary.shape
    big_iters = 100  # 3001 * 32 * 203 floats > 64 MiB
    assert _lib.lib().sg_crf_meanfield_compat_backward_ws_bytes(n, L, big_iters) > 64 << 20
    g_u = torch.empty_like(unary)
    g_mu = torch.empty_like(mu)
    rc = _lib.lib().sg_crf_meanfield_compat_backward_noalloc(
        lat._h, _lib.ptr(unary), L, _lib.ptr(mu), big_iters, _lib.ptr(gQ), _lib.ptr(g_u),
        _lib.ptr(g_mu), None)
    assert rc == -1 and b"scratch" in _lib.lib().sg_last_error()
    rc = _lib.lib().sg_crf_meanfield_compat_backward_noalloc(
        lat._h, _lib.ptr(unary), L, _lib.ptr(mu), 1, _lib.ptr(gQ), _lib.ptr(gQ),
        _lib.ptr(g_mu), None)
    assert rc == -1 and b"overlap" in _lib.lib().sg_last_error()
    torch.cuda.synchronize()
