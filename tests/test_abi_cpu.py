"""The C ABI without a GPU: the library loads, exports every function that
include/sgrid.h declares, and rejects invalid arguments on the host before
any HIP call (these calls launch nothing)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "sgrid.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sg_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2305_13220_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsgrid.so is not built (run __graft_entry__.build())")
    return _lib.lib()


def test_exports_every_declared_function(L):
    from paper_2305_13220_amd import _lib
    names = _header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), f"{n} declared in sgrid.h but not exported"
    assert set(names) <= set(_lib.exported_symbols())


def test_version_and_empty_error(L):
    assert b"gfx950" in L.sg_version()


def _err(L):
    return L.sg_last_error().decode()


def test_grid_build_validation(L):
    h = ctypes.c_void_p()
    org = (ctypes.c_float * 3)(0, 0, 0)
    assert L.sg_grid_build(None, 10, ctypes.c_float(0.02), org, None, ctypes.byref(h), None) == -1
    assert "d_block_coords" in _err(L)
    fake = ctypes.c_void_p(16)
    assert L.sg_grid_build(fake, 0, ctypes.c_float(0.02), org, None, ctypes.byref(h), None) == -1
    assert L.sg_grid_build(fake, 10, ctypes.c_float(0.0), org, None, ctypes.byref(h), None) == -1
    assert L.sg_grid_build(fake, 10, ctypes.c_float(float("nan")), org, None, ctypes.byref(h),
                           None) == -1
    bad_org = (ctypes.c_float * 3)(0, float("inf"), 0)
    assert L.sg_grid_build(fake, 10, ctypes.c_float(0.02), bad_org, None, ctypes.byref(h),
                           None) == -1
    assert L.sg_grid_build(fake, 10, ctypes.c_float(0.02), org, None, None, None) == -1
    assert h.value is None


def test_grid_handle_validation(L):
    n = ctypes.c_int64()
    assert L.sg_grid_num_blocks(None, ctypes.byref(n)) == -1
    assert L.sg_grid_destroy(None) == 0
    junk = (ctypes.c_uint32 * 64)()  # not a live grid: wrong magic
    assert L.sg_grid_num_blocks(ctypes.byref(junk), ctypes.byref(n)) == -5
    assert L.sg_grid_destroy(ctypes.byref(junk)) == -5
    assert L.sg_grid_lookup(None, None, 0, None, None) == -1


def test_render_validation(L):
    from paper_2305_13220_amd._lib import RenderParamsC
    p = RenderParamsC(0.01, 0.0, 12.0, 0.02, 128)
    fake = ctypes.c_void_p(16)
    assert L.sg_render_forward(None, fake, 3, fake, 10, ctypes.byref(p), fake, fake, fake, fake,
                               None, None, 0, None) == -1
    assert L.sg_render_backward(None, fake, 3, fake, 10, ctypes.byref(p), fake, fake, fake, None,
                                fake, None, 0, None) == -1
    assert L.sg_render_footprint(None, fake, 10, ctypes.byref(p), fake, None, None) == -1
    assert L.sg_query(None, fake, 3, fake, 10, None, None, None, None, None) == -1
    assert L.sg_eikonal(None, fake, 3, fake, 10, ctypes.c_float(1.0), None, None, None) == -1
    assert L.sg_query_backward(None, 3, fake, 10, None, None, None, fake, None) == -1
    assert L.sg_surface_points(None, fake, 3, fake, 10, ctypes.byref(p), fake, fake, None) == -1
    assert L.sg_fuse(None, fake, 1, fake, fake, 3, 4, 4, ctypes.c_float(0.1), 0, fake, None,
                     None) == -1
    assert L.sg_denoise(None, fake, 3, 1, ctypes.c_float(1.0), fake, None) == -1
    lat = ctypes.c_void_p()
    assert L.sg_lattice_build(fake, 10, 25, 4, None, ctypes.byref(lat)) == -1 and not lat.value
    assert L.sg_lattice_build(fake, 10, 3, 33, None, ctypes.byref(lat)) == -1
    assert L.sg_lattice_filter(None, fake, 1, fake, None) == -1
    assert L.sg_crf_meanfield(None, fake, 2, ctypes.c_float(1.0), 1, fake, None) == -1
    assert L.sg_crf_meanfield_compat(None, fake, 2, fake, 1, fake, None) == -1
    assert L.sg_crf_meanfield_compat_backward(None, fake, 2, fake, 1, fake, fake, fake, fake, 1 << 20,
                                              None) == -1
    assert L.sg_crf_meanfield_compat_backward_ws_bytes(0, 4, 1) == 0
    assert L.sg_crf_meanfield_compat_backward_ws_bytes(10, 33, 1) == 0
    assert L.sg_crf_meanfield_compat_backward_ws_bytes(10, 4, -1) == 0
    # marginals of 3 updates (3 x 1600 B), messages of 2 (2 x 1600 B), 2 gradient arrays of
    # 1600 B, each region rounded up to 256 B, + one workgroup's 4x4 partial sums
    assert L.sg_crf_meanfield_compat_backward_ws_bytes(100, 4, 2) == 4864 + 3328 + 2 * 1792 + 256
    assert L.sg_lattice_destroy(None) == 0
    assert L.sg_crf_label_loss(fake, 2, fake, 10, 4, ctypes.c_float(1.0), None, None, 4, None) == -1
    assert L.sg_crf_label_loss(fake, 4, fake, 10, 33, ctypes.c_float(1.0), None, None, 33, None) == -1
    assert L.sg_crf_label_loss(None, 4, None, 0, 4, ctypes.c_float(1.0), None, None, 4, None) == 0
    assert L.sg_crf_property_loss(fake, 2, fake, 10, 3, ctypes.c_float(1.0), None, None, 3,
                                  None) == -1
    assert L.sg_crf_property_loss(None, 3, None, 0, 3, ctypes.c_float(1.0), None, None, 3,
                                  None) == 0
    n = ctypes.c_int64(5)
    org = (ctypes.c_float * 3)(0, 0, 0)
    assert L.sg_alloc_blocks(fake, 1, fake, 4, 4, ctypes.c_float(0.02), org, -1, ctypes.c_float(1),
                             None, 0, ctypes.byref(n), None) == -1 and n.value == 0
    assert L.sg_alloc_blocks(fake, 1, fake, 4, 4, ctypes.c_float(0.0), org, 1, ctypes.c_float(1),
                             None, 0, ctypes.byref(n), None) == -1
    assert L.sg_grid_extend(None, fake, 3, None, None) == -1
    assert L.sg_uniform_points(None, 10, 0, fake, None) == -1
    gh = ctypes.c_void_p()
    assert L.sg_grid_from_depth(fake, 1, fake, 4, 4, ctypes.c_float(0.02), org, 9, ctypes.c_float(1),
                                None, ctypes.byref(gh), None) == -1 and not gh.value
    # zero pixels: nothing to do, no GPU call
    assert L.sg_alloc_blocks(None, 0, None, 4, 4, ctypes.c_float(0.02), org, 1, ctypes.c_float(1),
                             None, 0, ctypes.byref(n), None) == 0 and n.value == 0
    f = ctypes.c_float
    assert L.sg_render_l2_step(None, fake, 3, fake, 10, ctypes.byref(p), fake, fake, fake, f(0.1),
                               f(0.05), f(0.0), fake, fake, fake, fake, None, None, fake, None,
                               0, None) == -1


def test_workspace_size(L):
    """Sample-list workspace: [R][max_samples] (k, block) int32 pairs + [R] counts."""
    from paper_2305_13220_amd._lib import RenderParamsC
    for R, M in ((1, 1), (65536, 128), (1254528, 1024)):
        p = RenderParamsC(0.01, 0.0, 12.0, 0.02, M)
        assert L.sg_render_list_bytes(R, ctypes.byref(p)) == R * M * 8 + R * 4
    p = RenderParamsC(0.01, 0.0, 12.0, 0.02, 128)
    assert L.sg_render_list_bytes(0, ctypes.byref(p)) == 0
    assert L.sg_render_list_bytes(-1, ctypes.byref(p)) == 0
    bad = RenderParamsC(0.01, 0.0, 12.0, 0.02, 0)
    assert L.sg_render_list_bytes(10, ctypes.byref(bad)) == 0
    assert L.sg_render_list_bytes(10, None) == 0


def test_packed_validation(L):
    from paper_2305_13220_amd._lib import RenderParamsC
    from paper_2305_13220_amd.serve import SLOT_DTYPE, SlotC
    p = RenderParamsC(0.01, 0.0, 12.0, 0.02, 128)
    fake = ctypes.c_void_p(16)
    desc = (ctypes.c_ubyte * 512)()
    assert L.sg_packed_grid_desc(None, fake, 3, ctypes.byref(p), desc) == -1
    assert L.sg_render_forward_packed(None, 1, fake, fake, 4, 3, 128, 100, None) == -1
    assert L.sg_render_forward_packed(fake, 0, fake, fake, 4, 3, 128, 100, None) == -1
    assert L.sg_render_forward_packed(fake, 1, fake, fake, 4, 5, 128, 100, None) == -1
    assert L.sg_render_forward_packed(fake, 1, fake, fake, 4, 3, 2000, 100, None) == -1
    assert L.sg_render_forward_slots(None, fake, 3, ctypes.byref(p), fake, fake, 4, 100, None) == -1
    # the numpy slot record matches the C struct layout
    assert SLOT_DTYPE.itemsize == ctypes.sizeof(SlotC) == 136
    assert SLOT_DTYPE.fields["cam"][1] == 32 and SLOT_DTYPE.fields["nsamples"][1] == 128


def test_aux_validation(L):
    fake = ctypes.c_void_p(16)
    f = ctypes.c_float
    assert L.sg_rays_pinhole(fake, 1, fake, -1, fake, None) == -1
    assert L.sg_rays_pinhole(fake, 1, fake, 0, fake, None) == 0  # nothing to do
    assert L.sg_rays_pinhole(None, 1, fake, 5, fake, None) == -1
    assert L.sg_optim_step(5, fake, fake, fake, fake, 10, f(1e-3), f(0.9), f(0.999), f(1e-8), 1,
                           None) == -1
    assert L.sg_optim_step(0, fake, fake, None, fake, 10, f(1e-3), f(0.9), f(0.999), f(1e-8), 1,
                           None) == -1
    assert L.sg_optim_step(0, fake, fake, fake, fake, 10, f(1e-3), f(1.5), f(0.999), f(1e-8), 1,
                           None) == -1
    assert L.sg_optim_step(1, fake, fake, None, fake, 10, f(1e-3), f(0.9), f(0.999), f(1e-8), 0,
                           None) == -1
    assert L.sg_l2_loss_grad(fake, fake, fake, fake, fake, fake, 0, 3, f(0.1), f(0.05), fake, fake,
                             fake, None, None) == -1
    assert L.sg_l2_loss_grad(None, None, fake, fake, fake, fake, 10, 3, f(0.1), f(0.05), None,
                             fake, fake, None, None) == -1


def _plan(L, bmin, bmax, n_blocks, max_cells=None):
    from paper_2305_13220_amd._lib import BuildOptionsC
    lo = (ctypes.c_int32 * 3)(*bmin)
    hi = (ctypes.c_int32 * 3)(*bmax)
    dims = (ctypes.c_int32 * 3)(7, 7, 7)
    cells = ctypes.c_int64(-1)
    opts = None if max_cells is None else ctypes.byref(BuildOptionsC(max_cells))
    rc = L.sg_grid_dense_map_plan(lo, hi, n_blocks, opts, dims, ctypes.byref(cells))
    return rc, tuple(dims), cells.value


def test_dense_map_plan(L):
    """The dense map's size decision on the host, including the box that
    spans the whole coordinate range, (2^21)^3 = 2^63 cells, whose int64
    product once wrapped negative and passed the size check."""
    lim = 1 << 20
    assert _plan(L, (-lim,) * 3, (lim - 1,) * 3, 2) == (0, (0, 0, 0), 0)
    assert _plan(L, (-lim, 0, 0), (lim - 1, 0, 0), 2) == (0, (1 << 21, 1, 1), 1 << 21)
    assert _plan(L, (-lim, -lim, 0), (lim - 1, lim - 1, 0), 2) == (0, (0, 0, 0), 0)
    assert _plan(L, (0, 0, 0), (511, 511, 511), 100) == (0, (512, 512, 512), 1 << 27)
    assert _plan(L, (0, 0, 0), (1023, 1023, 255), 100) == (0, (1024, 1024, 256), 1 << 28)
    assert _plan(L, (0, 0, 0), (1023, 1023, 256), 100) == (0, (0, 0, 0), 0)
    assert _plan(L, (-3, 5, -7), (10, 5, 2), 40) == (0, (14, 1, 10), 140)
    # block indices must fit the map's 23 bits
    assert _plan(L, (0, 0, 0), (9, 9, 9), (1 << 23) - 1)[2] == 1000
    assert _plan(L, (0, 0, 0), (9, 9, 9), 1 << 23)[2] == 0
    # options: 0 disables the map, a limit below the count disables it, < 0 is the default
    assert _plan(L, (0, 0, 0), (9, 9, 9), 5, max_cells=0)[2] == 0
    assert _plan(L, (0, 0, 0), (9, 9, 9), 5, max_cells=999)[2] == 0
    assert _plan(L, (0, 0, 0), (9, 9, 9), 5, max_cells=1000)[2] == 1000
    assert _plan(L, (0, 0, 0), (9, 9, 9), 5, max_cells=-1)[2] == 1000
    assert _plan(L, (0, 0, 0), (lim, 0, 0), 5)[0] == -2
    assert _plan(L, (-lim - 1, 0, 0), (0, 0, 0), 5)[0] == -2
    assert _plan(L, (3, 0, 0), (2, 0, 0), 5)[0] == -1
    assert _plan(L, (0, 0, 0), (2, 0, 0), -1)[0] == -1


def test_lattice_and_workspace_sizes(L):
    """Host-side byte counts of the lattice build and the mean-field
    gradient's workspace, and their limits."""
    def lat(n, d, v):
        cap = 1
        while cap < 2 * n * (d + 1):
            cap <<= 1
        ks = (d + 3) // 4 * 4  # key rows padded to 16 bytes
        return (cap * (8 + 4 * ks + 8 * v + 4) + n * (d + 1) * 8 + n * v * 4
                + 4 * 2 * (d + 1) * n * (d + 1))
    for n, d, v in ((1, 1, 1), (1000, 6, 16), (262144, 6, 16), (5, 16, 32)):
        assert L.sg_lattice_bytes(n, d, v) == lat(n, d, v)
    assert L.sg_lattice_bytes(0, 6, 16) == 0
    assert L.sg_lattice_bytes(10, 0, 16) == 0
    assert L.sg_lattice_bytes(10, 25, 16) == 0
    assert L.sg_lattice_bytes(10, 24, 16) > 0
    assert L.sg_lattice_bytes(10, 6, 33) == 0
    assert L.sg_lattice_bytes((1 << 30) // 7 + 1, 6, 1) == 0  # n (d+1) beyond 2^30
    assert L.sg_lattice_bytes((1 << 30) // 7 - 1, 6, 1) > 0

    def ws(n, lb, t):
        al = lambda b: (b + 255) // 256 * 256
        nl = n * lb * 4
        return (al((t + 1) * nl) + al(t * nl) + al(nl) + al(nl)
                + al((n + 127) // 128 * lb * lb * 4))
    assert L.sg_crf_meanfield_compat_backward_ws_bytes(262144, 16, 5) == ws(262144, 16, 5)
    assert L.sg_crf_meanfield_compat_backward_ws_bytes(1, 1, 0) == ws(1, 1, 0)
    assert L.sg_crf_meanfield_compat_backward_ws_bytes(0, 16, 5) == 0
    assert L.sg_crf_meanfield_compat_backward_ws_bytes(10, 33, 5) == 0
    assert L.sg_crf_meanfield_compat_backward_ws_bytes(10, 16, -1) == 0


def test_grid_generation_and_descriptor_check_validation(L):
    gen = ctypes.c_uint64(7)
    assert L.sg_grid_generation(None, ctypes.byref(gen)) == -1
    assert gen.value == 7
    desc = (ctypes.c_ubyte * 512)()
    assert L.sg_packed_grid_check(None, desc) == -1
    assert L.sg_packed_grid_check(None, None) == -1


def test_extend_refused_while_a_server_holds_the_grid():
    """A render server pins its grids: extend (which moves the grid's memory,
    leaving descriptors and captured launches pointing at freed memory) is
    refused before anything reaches the library, and allowed again after
    the last unpin (it then fails here only on the CPU tensor)."""
    import torch
    import paper_2305_13220_amd as sg
    g = sg.Grid.__new__(sg.Grid)
    g._h = ctypes.c_void_p(0)
    g.device = torch.device("cpu")
    g.pin()
    g.pin()
    coords = torch.zeros((1, 3), dtype=torch.int32)
    with pytest.raises(sg.SgridError, match="pinned"):
        g.extend(coords)
    g.unpin()
    with pytest.raises(sg.SgridError, match="pinned"):
        g.extend(coords)
    g.unpin()
    with pytest.raises(ValueError, match="GPU tensor"):
        g.extend(coords)


def test_binding_rejects_cpu_tensors():
    import torch
    import paper_2305_13220_amd as sg
    with pytest.raises(ValueError, match="GPU tensor"):
        sg.Grid(torch.zeros((4, 3), dtype=torch.int32), 0.02)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and says why,
    before touching a GPU."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
