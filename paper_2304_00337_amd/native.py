"""ctypes binding of libbloch.so (include/bloch.h).  Argument marshalling only: every step
of the computation runs in the library's gfx950 kernels.  Importing works without a GPU;
loading the library fails loudly if it has not been built."""
from __future__ import annotations

import ctypes
import os

__all__ = ["LIB_PATH", "load", "BlGrid", "BlOpts", "BlInfo", "BlProblem", "BlRequest",
           "BlRequestInfo", "BlServerCounters", "EXPORTED", "OPS", "check"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbloch.so")

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_double = ctypes.c_double
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p
P = ctypes.POINTER

BL_OK, BL_EINVAL, BL_ENOMEM, BL_EHIP, BL_ENOCONV, BL_EAGAIN, BL_ESTATE = 0, -1, -2, -3, -4, -5, -6

OPS = {"A": 0, "M": 1, "K": 2, "LIFT": 3, "LHM": 4, "P": 5, "EDGE_SMOOTH": 6,
       "EDGE_SMOOTH_BACK": 7, "NODAL_SMOOTH": 8, "EDGE_VCYCLE": 9, "NODAL_VCYCLE": 10,
       "EDGE_PROLONG": 11, "EDGE_RESTRICT": 12, "NODAL_PROLONG": 13, "NODAL_RESTRICT": 14,
       "PROJECT": 15, "COARSE_EDGE": 16, "COARSE_NODAL": 17, "EIGRES": 18,
       "EDGE_SWEEP": 19, "EDGE_SWEEP_BACK": 20, "NODAL_SWEEP": 21, "NODAL_SWEEP_BACK": 22}


class BlGrid(ctypes.Structure):
    _fields_ = [("n", c_int32), ("m", c_int32), ("a", c_double), ("b", c_double)]


class BlOpts(ctypes.Structure):
    _fields_ = [("nev", c_int32), ("nthrow", c_int32), ("max_iter", c_int32),
                ("levels", c_int32), ("coarsest_min", c_int32), ("nu_pre", c_int32),
                ("nu_post", c_int32), ("nodal_cycles", c_int32), ("variant", c_int32),
                ("precision", c_int32), ("extrap_depth", c_int32), ("autotune", c_int32),
                ("coarse_fuse", c_int32), ("tiled_sweeps", c_int32),
                ("tol", c_double), ("mu", c_double), ("zero_rel", c_double),
                ("engine_streams", c_int32), ("tol_abs", c_int32), ("tol_floor", c_int32),
                ("nested_start", c_int32), ("nested_tol", c_double), ("lock_rel", c_double),
                ("throw_precond", c_int32), ("reserved_opts", c_int32)]


class BlInfo(ctypes.Structure):
    _fields_ = [("n", c_int32), ("m", c_int32), ("p", c_int32), ("nev", c_int32),
                ("levels", c_int32), ("precision", c_int32), ("level_n", c_int32 * 16),
                ("level_m", c_int32 * 16), ("mu", c_double), ("device_bytes", c_size_t),
                ("kernel_launches", c_int64), ("edge_smooth_shape", c_int32 * 3),
                ("nodal_smooth_shape", c_int32 * 3), ("rr_tile", c_int32),
                ("fused_edge_level", c_int32), ("fused_nodal_level", c_int32), ("reserved", c_int32),
                ("autotune_ms", c_double), ("locked_columns", c_int64)]


class BlProblem(ctypes.Structure):
    _fields_ = [("grid", BlGrid), ("eps", P(c_double)), ("nev", c_int32), ("nthrow", c_int32),
                ("nk", c_int32), ("reserved0", c_int32), ("ks", P(c_double)), ("start_dev", c_void_p),
                ("evals", P(c_double)), ("relres", P(c_double)), ("iters", P(c_int32)),
                ("point_ms", P(c_double)), ("evecs_dev", c_void_p), ("status", c_int32),
                ("reserved1", c_int32)]


class BlRequest(ctypes.Structure):
    _fields_ = [("grid", BlGrid), ("eps", P(c_double)), ("nev", c_int32), ("nthrow", c_int32),
                ("nk", c_int32), ("reserved0", c_int32), ("ks", P(c_double)), ("start_dev", c_void_p)]


class BlRequestInfo(ctypes.Structure):
    _fields_ = [("status", c_int32), ("total_iters", c_int32), ("queue_s", c_double),
                ("run_s", c_double), ("latency_s", c_double)]


class BlServerCounters(ctypes.Structure):
    _fields_ = [("rounds", c_int64), ("kernel_launches", c_int64), ("device_bytes", c_size_t),
                ("engines", c_int32), ("queued", c_int32), ("pending", c_int32), ("reserved", c_int32)]


# name -> (restype, argtypes); must match include/bloch.h
EXPORTED = {
    "bl_default_opts": (None, [P(BlOpts), c_int32]),
    "bl_create": (c_int32, [P(BlGrid), P(c_double), P(BlOpts), c_void_p, P(c_void_p)]),
    "bl_destroy": (None, [c_void_p]),
    "bl_footprint_bytes": (c_size_t, [P(BlGrid), P(BlOpts)]),
    "bl_get_info": (c_int32, [c_void_p, P(BlInfo)]),
    "bl_solve_k": (c_int32, [c_void_p, c_double, c_double, c_void_p, P(c_double), P(c_double),
                             P(c_int32), c_void_p]),
    "bl_solve_path": (c_int32, [c_void_p, P(c_double), c_int32, c_void_p, P(c_double),
                                P(c_double), P(c_int32), c_void_p]),
    "bl_reset_history": (c_int32, [c_void_p]),
    "bl_raster_sources": (c_int32, [c_int32, c_int32, c_int32, P(c_int32)]),
    "bl_solve_kgrid": (c_int32, [c_void_p, c_int32, c_void_p, P(c_double), P(c_double), P(c_int32)]),
    "bl_nested_start": (c_int32, [c_void_p, c_double, c_double, c_double, c_void_p, P(c_int32)]),
    "bl_last_residual_history": (c_int32, [c_void_p, P(c_double), c_int32]),
    "bl_set_k": (c_int32, [c_void_p, c_double, c_double]),
    "bl_set_timing": (c_int32, [c_void_p, c_int32]),
    "bl_get_timing": (c_int32, [c_void_p, P(c_double), P(c_int64), P(c_int64), P(c_double)]),
    "bl_apply": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                           c_void_p]),
    "bl_gram": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_int32, c_int64, P(c_double)]),
    "bl_gram_noalloc": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_int32, c_int64, c_void_p]),
    "bl_ritz_small": (c_int32, [c_void_p, P(c_double), P(c_double), c_int32, c_int32, c_double,
                                P(c_double), P(c_double)]),
    "bl_rr_products": (c_int32, [c_void_p, c_void_p, c_int32, P(c_double), P(c_double)]),
    "bl_batch_solve": (c_int32, [P(BlOpts), P(BlProblem), c_int32, c_int32, c_void_p]),
    "bl_batch_create": (c_int32, [P(BlOpts), c_int32, c_size_t, P(c_void_p)]),
    "bl_batch_run": (c_int32, [c_void_p, P(BlProblem), c_int32, c_void_p]),
    "bl_batch_destroy": (None, [c_void_p]),
    "bl_batch_engine_info": (c_int32, [c_void_p, c_int32, P(BlInfo)]),
    "bl_batch_set_timing": (c_int32, [c_void_p, c_int32]),
    "bl_batch_get_timing": (c_int32, [c_void_p, P(c_double), P(c_int64), P(c_int64), P(c_double)]),
    "bl_server_create": (c_int32, [P(BlOpts), c_size_t, c_int32, P(c_void_p)]),
    "bl_server_submit": (c_int32, [c_void_p, P(BlRequest), P(ctypes.c_uint64)]),
    "bl_server_poll": (c_int32, [c_void_p, ctypes.c_uint64, P(c_double), P(c_double), P(c_int32),
                                 P(BlRequestInfo)]),
    "bl_server_stats": (c_int32, [c_void_p, P(BlServerCounters)]),
    "bl_server_destroy": (None, [c_void_p]),
    "bl_strerror": (ctypes.c_char_p, [c_int32]),
    "bl_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load libbloch.so (once) and declare the prototypes; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2304_00337_amd.build` "
                           "(there is no fallback implementation)")
    # PyTorch provides the device memory and streams and ships its own HIP runtime; load it
    # first so that the library binds to the same runtime instance
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTED.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class BlochError(RuntimeError):
    def __init__(self, code, where):
        lib = load()
        msg = lib.bl_last_error().decode(errors="replace")
        super().__init__(f"{where} failed: {lib.bl_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def check(code, where, allow=()):
    if code < 0 and code not in allow:
        raise BlochError(code, where)
    return code
