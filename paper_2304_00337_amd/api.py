"""Python front of the C ABI: the same calls as include/bloch.h, taking NumPy host arrays
and PyTorch device tensors.  Marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np

from . import native
from .native import BlGrid, BlInfo, BlOpts, check

__all__ = ["Solver", "to_device_block", "from_device_block"]


def _torch():
    import torch
    return torch


def to_device_block(X: np.ndarray, dtype=None, device="cuda"):
    """Complex (N, ncols) host array -> planar column block tensor (ncols, 2, N) on the GPU."""
    torch = _torch()
    X = np.asarray(X)
    if X.ndim == 1:
        X = X[:, None]
    planar = np.stack([X.real.T, X.imag.T], axis=1)
    t = torch.from_numpy(np.ascontiguousarray(planar, dtype=np.float64))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device).contiguous()


def from_device_block(t) -> np.ndarray:
    """Planar column block tensor (ncols, 2, N) -> complex (N, ncols) host array."""
    a = t.detach().to("cpu").double().numpy()
    return (a[:, 0, :] + 1j * a[:, 1, :]).T.copy()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Solver:
    """Handle for one grid and permittivity (bl_create).

    Keyword options map to bl_opts fields: nev, nthrow, max_iter, levels, coarsest_min,
    nu_pre, nu_post, nodal_cycles, variant, precision ("fp64" | "mixed" or 0 | 1),
    extrap_depth, tol, mu, zero_rel."""

    def __init__(self, n, m, a, b, eps, nev=8, stream=None, **opts):
        torch = _torch()
        self.lib = native.load()
        self.n, self.m, self.a, self.b = int(n), int(m), float(a), float(b)
        o = BlOpts()
        self.lib.bl_default_opts(ctypes.byref(o), int(nev))
        for k, v in opts.items():
            if k == "precision" and isinstance(v, str):
                v = {"fp64": 0, "mixed": 1}[v]
            if not hasattr(o, k):
                raise TypeError(f"unknown option {k}")
            setattr(o, k, v)
        self.opts = o
        self.grid = BlGrid(self.n, self.m, self.a, self.b)
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        if eps.shape != (self.n * self.m,):
            raise ValueError("eps must hold n*m cell values")
        self._eps = eps
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        check(self.lib.bl_create(ctypes.byref(self.grid), eps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 ctypes.byref(o), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)),
              "bl_create")
        self.h = h
        self.p = o.nev + o.nthrow
        self.nev = o.nev
        self.n_edges = 2 * self.n * self.m
        self.n_nodes = self.n * self.m

    # -- lifetime --------------------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.bl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- queries ---------------------------------------------------------------------------
    def info(self) -> dict:
        inf = BlInfo()
        check(self.lib.bl_get_info(self.h, ctypes.byref(inf)), "bl_get_info")
        L = inf.levels
        return {"n": inf.n, "m": inf.m, "p": inf.p, "nev": inf.nev, "levels": L,
                "precision": inf.precision, "mu": inf.mu, "device_bytes": inf.device_bytes,
                "kernel_launches": inf.kernel_launches,
                "sizes": [(inf.level_n[i], inf.level_m[i]) for i in range(L)]}

    @staticmethod
    def footprint_bytes(n, m, a, b, nev=8, **opts) -> int:
        lib = native.load()
        o = BlOpts()
        lib.bl_default_opts(ctypes.byref(o), int(nev))
        for k, v in opts.items():
            if k == "precision" and isinstance(v, str):
                v = {"fp64": 0, "mixed": 1}[v]
            setattr(o, k, v)
        g = BlGrid(int(n), int(m), float(a), float(b))
        return int(lib.bl_footprint_bytes(ctypes.byref(g), ctypes.byref(o)))

    # -- solves ----------------------------------------------------------------------------
    def _start(self, start):
        if start is None:
            return None
        torch = _torch()
        if isinstance(start, np.ndarray):
            start = to_device_block(start)
        assert start.dtype == torch.float64 and start.is_contiguous()
        assert start.numel() == self.p * 2 * self.n_edges
        return start

    def solve_k(self, k1, k2, start=None, want_vectors=False, allow_noconv=False):
        torch = _torch()
        start = self._start(start)
        ev = np.zeros(self.nev)
        rr = np.zeros(self.nev)
        it = ctypes.c_int32(0)
        vec = torch.empty((self.nev, 2, self.n_edges), dtype=torch.float64, device="cuda") if want_vectors else None
        rc = self.lib.bl_solve_k(self.h, float(k1), float(k2), _ptr(start),
                                 ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 rr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(it),
                                 _ptr(vec))
        check(rc, "bl_solve_k", allow=(native.BL_ENOCONV,) if allow_noconv else ())
        return {"evals": ev, "relres": rr, "iterations": int(it.value), "converged": rc == 0,
                "evecs": vec}

    def solve_path(self, ks, start=None, want_last_vectors=False, allow_noconv=False):
        torch = _torch()
        ks = np.ascontiguousarray(ks, dtype=np.float64).reshape(-1, 2)
        nk = ks.shape[0]
        start = self._start(start)
        ev = np.zeros((nk, self.nev))
        rr = np.zeros((nk, self.nev))
        its = np.zeros(nk, dtype=np.int32)
        vec = torch.empty((self.nev, 2, self.n_edges), dtype=torch.float64, device="cuda") if want_last_vectors else None
        rc = self.lib.bl_solve_path(self.h, ks.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nk,
                                    _ptr(start), ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    rr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    its.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(vec))
        check(rc, "bl_solve_path", allow=(native.BL_ENOCONV,) if allow_noconv else ())
        return {"evals": ev, "relres": rr, "iterations": its, "converged": rc == 0, "evecs": vec}

    def reset_history(self):
        check(self.lib.bl_reset_history(self.h), "bl_reset_history")

    def residual_history(self, cap=1000) -> np.ndarray:
        buf = np.zeros((cap, self.nev))
        rows = check(self.lib.bl_last_residual_history(
            self.h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cap), "bl_last_residual_history")
        return buf[:rows]

    def set_timing(self, enable=True):
        check(self.lib.bl_set_timing(self.h, 1 if enable else 0), "bl_set_timing")

    def timing(self) -> dict:
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        cols = ctypes.c_int64()
        check(self.lib.bl_get_timing(self.h, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(cols)),
              "bl_get_timing")
        return {"total_ms": ms.value, "launches": cnt.value, "columns": cols.value}

    # -- operator level ----------------------------------------------------------------------
    def set_k(self, k1, k2):
        check(self.lib.bl_set_k(self.h, float(k1), float(k2)), "bl_set_k")

    def apply(self, op, x, y=None, out=None, level=0):
        """Run one operator (see bl_apply) on planar device blocks x (ncols, 2, N)."""
        torch = _torch()
        opid = native.OPS[op] if isinstance(op, str) else int(op)
        prec = 1 if x.dtype == torch.float32 else 0
        ncols = x.shape[0]
        if out is None:
            raise ValueError("out must be given (its shape depends on the operator)")
        check(self.lib.bl_apply(self.h, opid, int(level), prec, ncols, _ptr(x), _ptr(y), _ptr(out)),
              f"bl_apply({op})")
        return out

    def gram(self, X, W) -> np.ndarray:
        q, r = X.shape[0], W.shape[0]
        out = np.zeros((q, r, 2))
        check(self.lib.bl_gram(self.h, _ptr(X), q, _ptr(W), r, X.shape[2],
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "bl_gram")
        return out[..., 0] + 1j * out[..., 1]

    def ritz_small(self, G: np.ndarray, H: np.ndarray, want: int, zero_thr: float = -np.inf):
        q = G.shape[0]
        g = np.ascontiguousarray(np.stack([G.real, G.imag], axis=-1), dtype=np.float64)
        h = np.ascontiguousarray(np.stack([H.real, H.imag], axis=-1), dtype=np.float64)
        th = np.zeros(want)
        Y = np.zeros((q, want, 2))
        cnt = check(self.lib.bl_ritz_small(self.h, g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), q, want,
                                           float(zero_thr), th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           Y.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "bl_ritz_small")
        return th[:cnt], (Y[..., 0] + 1j * Y[..., 1])[:, :cnt]
