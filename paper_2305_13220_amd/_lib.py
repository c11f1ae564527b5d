"""ctypes binding of libsgrid.so (include/sgrid.h): argument marshalling only.

Every function here checks tensor device / dtype / shape / contiguity,
passes raw device pointers and the current HIP stream to the C ABI, and
raises SgridError on a non-zero status.  No arithmetic of the method runs
in Python.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgrid.so")


class SgridError(RuntimeError):
    pass


class BuildOptionsC(ctypes.Structure):
    _fields_ = [("dense_map_max_cells", ctypes.c_int64)]


class RenderParamsC(ctypes.Structure):
    _fields_ = [("step", ctypes.c_float), ("t_near", ctypes.c_float), ("t_far", ctypes.c_float),
                ("beta", ctypes.c_float), ("max_samples", ctypes.c_int32)]


_lib = None

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_f = ctypes.c_float

_SIGNATURES = {
    "sg_last_error": ([], ctypes.c_char_p),
    "sg_version": ([], ctypes.c_char_p),
    "sg_grid_build": ([_vp, _i64, _f, _vp, _vp, _vp, _vp], ctypes.c_int),
    "sg_grid_build_ex": ([_vp, _i64, _f, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "sg_grid_dense_map": ([_vp, _vp, _vp], ctypes.c_int),
    "sg_grid_copy_dense_map": ([_vp, _vp, _vp], ctypes.c_int),
    "sg_grid_num_blocks": ([_vp, _vp], ctypes.c_int),
    "sg_grid_geometry": ([_vp, _vp, _vp], ctypes.c_int),
    "sg_grid_generation": ([_vp, _vp], ctypes.c_int),
    "sg_grid_dense_map_plan": ([_vp, _vp, _i64, _vp, _vp, _vp], ctypes.c_int),
    "sg_lattice_bytes": ([_i64, _i32, _i32], ctypes.c_size_t),
    "sg_packed_grid_check": ([_vp, _vp], ctypes.c_int),
    "sg_grid_block_coords": ([_vp, _vp, _vp], ctypes.c_int),
    "sg_grid_neighbors": ([_vp, _vp, _vp], ctypes.c_int),
    "sg_grid_lookup": ([_vp, _vp, _i64, _vp, _vp], ctypes.c_int),
    "sg_grid_destroy": ([_vp], ctypes.c_int),
    "sg_rays_pinhole": ([_vp, _i32, _vp, _i64, _vp, _vp], ctypes.c_int),
    "sg_query": ([_vp, _vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "sg_surface_points": ([_vp, _vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp], ctypes.c_int),
    "sg_query_backward": ([_vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "sg_uniform_points": ([_vp, _i64, ctypes.c_uint64, _vp, _vp], ctypes.c_int),
    "sg_eikonal": ([_vp, _vp, _i32, _vp, _i64, ctypes.c_float, _vp, _vp, _vp], ctypes.c_int),
    "sg_grid_extend": ([_vp, _vp, _i64, _vp, _vp], ctypes.c_int),
    "sg_grid_from_depth": ([_vp, _i32, _vp, _i32, _i32, ctypes.c_float, _vp, _i32, ctypes.c_float,
                            _vp, _vp, _vp], ctypes.c_int),
    "sg_alloc_blocks": ([_vp, _i32, _vp, _i32, _i32, ctypes.c_float, _vp, _i32, ctypes.c_float,
                         _vp, _i64, _vp, _vp], ctypes.c_int),
    "sg_fuse": ([_vp, _vp, _i32, _vp, _vp, _i32, _i32, _i32, ctypes.c_float, _i32, _vp, _vp, _vp],
                ctypes.c_int),
    "sg_denoise": ([_vp, _vp, _i32, _i32, ctypes.c_float, _vp, _vp], ctypes.c_int),
    "sg_lattice_build": ([_vp, _i64, _i32, _i32, _vp, _vp], ctypes.c_int),
    "sg_lattice_num_vertices": ([_vp, _vp], ctypes.c_int),
    "sg_lattice_filter": ([_vp, _vp, _i32, _vp, _vp], ctypes.c_int),
    "sg_crf_meanfield": ([_vp, _vp, _i32, ctypes.c_float, _i32, _vp, _vp], ctypes.c_int),
    "sg_crf_meanfield_compat": ([_vp, _vp, _i32, _vp, _i32, _vp, _vp], ctypes.c_int),
    "sg_crf_meanfield_compat_backward_ws_bytes": ([_i64, _i32, _i32], ctypes.c_size_t),
    "sg_crf_meanfield_compat_backward": ([_vp, _vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp,
                                          ctypes.c_size_t, _vp], ctypes.c_int),
    "sg_crf_meanfield_compat_backward_noalloc_max_bytes": ([], ctypes.c_size_t),
    "sg_crf_meanfield_compat_backward_noalloc": ([_vp, _vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp],
                                                 ctypes.c_int),
    "sg_crf_label_loss": ([_vp, _i64, _vp, _i64, _i32, ctypes.c_float, _vp, _vp, _i64, _vp],
                          ctypes.c_int),
    "sg_crf_property_loss": ([_vp, _i64, _vp, _i64, _i32, ctypes.c_float, _vp, _vp, _i64, _vp],
                             ctypes.c_int),
    "sg_lattice_destroy": ([_vp], ctypes.c_int),
    "sg_render_list_bytes": ([_i64, _vp], ctypes.c_size_t),
    "sg_render_march": ([_vp, _vp, _i64, _vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "sg_render_forward": ([_vp, _vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                           ctypes.c_size_t, _vp], ctypes.c_int),
    "sg_render_backward": ([_vp, _vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                            ctypes.c_size_t, _vp], ctypes.c_int),
    "sg_render_footprint": ([_vp, _vp, _i64, _vp, _vp, _vp, _vp], ctypes.c_int),
    "sg_packed_grid_desc": ([_vp, _vp, _i32, _vp, _vp], ctypes.c_int),
    "sg_render_forward_packed": ([_vp, _i32, _vp, _vp, _i32, _i32, _i32, _i64, _vp], ctypes.c_int),
    "sg_render_forward_slots": ([_vp, _vp, _i32, _vp, _vp, _vp, _i32, _i64, _vp], ctypes.c_int),
    "sg_render_l2_step": ([_vp, _vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp, _f, _f, _f, _vp, _vp, _vp,
                           _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "sg_l2_loss_grad": ([_vp, _vp, _vp, _vp, _vp, _vp, _i64, _i32, _f, _f, _vp, _vp, _vp, _vp, _vp],
                        ctypes.c_int),
    "sg_optim_step": ([_i32, _vp, _vp, _vp, _vp, _i64, _f, _f, _f, _f, _i32, _vp], ctypes.c_int),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2305_13220_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGNATURES)


def check(rc: int, what: str):
    if rc != 0:
        msg = lib().sg_last_error().decode(errors="replace")
        raise SgridError(f"{what} failed (status {rc}): {msg}")


def stream_ptr(device=None):
    return _vp(torch.cuda.current_stream(device).cuda_stream)


def ptr(t):
    return None if t is None else _vp(t.data_ptr())


def want(t, name, dtype, shape=None, device=None):
    """Validate a tensor argument of the C ABI."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor (got {t.device})")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None:
        if t.dim() != len(shape) or any(s is not None and a != s for a, s in zip(t.shape, shape)):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")
    return t
