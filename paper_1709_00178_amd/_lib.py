"""ctypes loader for libpyrit.so (argument marshalling only).

The library must have been built in-tree (``python -m paper_1709_00178_amd.build``
or ``__graft_entry__.build()``).  There is no fallback: a missing library is an
error.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpyrit.so")

_lib = None

c_int, c_u32, c_u64, c_size, c_vp = (ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64,
                                    ctypes.c_size_t, ctypes.c_void_p)
P = ctypes.POINTER

# name -> (restype, argtypes); mirrors include/pyrit.h
SIGNATURES = {
    "pyrit_strerror": (ctypes.c_char_p, [c_int]),
    "pyrit_version": (ctypes.c_char_p, []),
    "pyrit_ring_check": (c_int, [c_int, c_int, c_u32]),
    "pyrit_ring_supported": (c_int, [c_int, c_int, c_u32]),
    "pyrit_lift": (c_int, [c_int, c_int, c_u32, c_u32, P(c_u32)]),
    "pyrit_ring_reduce": (c_int, [c_int, c_int, c_u32, c_u32, P(c_u32)]),
    "pyrit_ring_mul": (c_int, [c_int, c_u32, c_u32, P(c_u32)]),
    "pyrit_gf_mul": (c_int, [c_int, c_u32, c_u32, c_u32, P(c_u32)]),
    "pyrit_cauchy": (c_int, [c_int, c_u32, c_int, c_int, c_vp]),
    "pyrit_cauchy_light": (c_int, [c_int, c_int, c_u32, c_int, c_int, c_vp, c_vp, c_vp, P(c_int)]),
    "pyrit_cauchy_search": (c_int, [c_int, c_int, c_u32, c_int, c_int, c_int, c_vp, c_vp, c_vp,
                                    c_vp, c_vp, P(c_int)]),
    "pyrit_plan_create": (c_int, [c_int, c_int, c_u32, c_int, c_int, c_vp, P(c_vp)]),
    "pyrit_plan_create_ex": (c_int, [c_int, c_int, c_u32, c_int, c_int, c_vp, c_int, P(c_vp)]),
    "pyrit_plan_transform": (c_int, [c_vp, P(c_int)]),
    "pyrit_plan_destroy": (None, [c_vp]),
    "pyrit_plan_params": (c_int, [c_vp, P(c_int), P(c_int), P(c_u32), P(c_int), P(c_int)]),
    "pyrit_plan_lifted": (c_int, [c_vp, c_vp]),
    "pyrit_plan_weight": (c_int, [c_vp, P(c_int)]),
    "pyrit_decode_matrix": (c_int, [c_vp, c_vp, c_int, c_vp, c_vp]),
    "pyrit_encode": (c_int, [c_vp, c_vp, c_vp, c_size, c_vp]),
    "pyrit_encode_ex": (c_int, [c_vp, c_vp, c_vp, c_size, c_size, c_int, c_vp]),
    "pyrit_decode_ex": (c_int, [c_vp, c_vp, c_int, c_vp, c_size, c_size, c_vp]),
    "pyrit_decode": (c_int, [c_vp, c_vp, c_int, c_vp, c_size, c_vp]),
    "pyrit_fill_random": (c_int, [c_vp, c_size, c_size, c_u64, c_vp]),
    "pyrit_fill_random_blocks": (c_int, [c_vp, c_vp, c_vp, c_vp, c_int, c_vp]),
    "pyrit_copy": (c_int, [c_vp, c_vp, c_size, c_vp]),
    "pyrit_to_sliced": (c_int, [c_int, c_vp, c_size, c_vp, c_size, c_vp]),
    "pyrit_from_sliced": (c_int, [c_int, c_vp, c_size, c_size, c_vp, c_vp]),
    "pyrit_batch_create": (c_int, [c_vp, c_int, c_vp, P(c_vp)]),
    "pyrit_batch_launch": (c_int, [c_vp, c_vp]),
    "pyrit_batch_launch_direct": (c_int, [c_vp, c_vp]),
    "pyrit_batch_info": (c_int, [c_vp, P(c_int), P(c_int), P(c_u64), P(c_int), P(c_int)]),
    "pyrit_batch_destroy": (None, [c_vp]),
    "pyrit_batch_describe": (c_int, [c_vp, c_int, c_vp, P(c_int), P(c_int), P(c_u64), P(c_int),
                                     P(c_u64)]),
    "pyrit_batch_run_noalloc": (c_int, [c_vp, c_int, c_vp, c_vp]),
    "pyrit_server_create": (c_int, [c_vp, P(c_vp)]),
    "pyrit_server_pool": (c_vp, [c_vp]),
    "pyrit_server_run": (c_int, [c_vp, c_vp, c_int, c_vp, c_vp]),
    "pyrit_server_destroy": (None, [c_vp]),
}


class BatchItem(ctypes.Structure):
    """pyrit_batch_item"""
    _fields_ = [("plan", c_vp), ("n_erased", c_int), ("erased", P(c_int)),
                ("blocks", P(c_vp)), ("slice_bytes", c_size), ("slice_pitch", c_size)]


class Tune(ctypes.Structure):
    """pyrit_tune"""
    _fields_ = [("mode", c_int), ("tile_bytes", c_int), ("grid", c_int),
                ("wg_threads", c_int), ("xcd_order", c_int), ("split_k", c_int)]


BATCH_MODES = {"grid": 0, "queue": 1, "static": 2}


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1709_00178_amd.build` "
            "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


class Request(ctypes.Structure):
    """pyrit_request"""
    _fields_ = [("arrival_s", ctypes.c_double), ("plan", c_vp), ("n_erased", c_int),
                ("erased", P(c_int)), ("inputs", P(c_vp)), ("slice_bytes", c_size),
                ("slice_pitch", c_size)]


class RequestResult(ctypes.Structure):
    """pyrit_request_result"""
    _fields_ = [("admit_s", ctypes.c_double), ("launch_s", ctypes.c_double),
                ("done_s", ctypes.c_double), ("out_offset", c_u64), ("out_stride", c_u64),
                ("launch", c_int)]


class ServeConfig(ctypes.Structure):
    """pyrit_serve_config"""
    _fields_ = [("pool_bytes", c_size), ("slots", c_int), ("max_batch", c_int),
                ("per_request", c_int), ("release_outputs", c_int), ("block_skew", c_size),
                ("slot_bytes", c_size), ("large_bytes", c_size), ("tune", Tune)]


class ServeStats(ctypes.Structure):
    """pyrit_serve_stats"""
    _fields_ = [("elapsed_s", ctypes.c_double), ("launches", c_int), ("max_batch_seen", c_int),
                ("mean_batch", ctypes.c_double), ("peak_pool_bytes", c_u64),
                ("admission_waits", c_int), ("moved_bytes", c_u64)]
