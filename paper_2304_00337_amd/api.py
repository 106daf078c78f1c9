"""Python front of the C ABI: the same calls as include/bloch.h, taking NumPy host arrays
and PyTorch device tensors.  Marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np

from . import native
from .native import (BlGrid, BlInfo, BlOpts, BlProblem, BlRequest, BlRequestInfo,
                     BlServerCounters, check)

__all__ = ["Solver", "Server", "Batch", "batch_solve", "to_device_block", "from_device_block"]


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


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _make_opts(nev=8, **opts) -> BlOpts:
    lib = native.load()
    o = BlOpts()
    lib.bl_default_opts(ctypes.byref(o), int(nev))
    for k, v in opts.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": 0, "mixed": 1}[v]
        if k == "variant" and isinstance(v, str):
            v = {"gradient": 0, "lobpcg": 1}[v]
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def raster_sources(kappa, i, j):
    """Grid points (i', j') whose blocks give the start block of point (i, j) of the
    kappa x kappa Bloch grid (Section 6), oldest first."""
    lib = native.load()
    buf = (ctypes.c_int32 * 6)()
    c = check(lib.bl_raster_sources(int(kappa), int(i), int(j), buf), "bl_raster_sources")
    return [(buf[2 * q], buf[2 * q + 1]) for q in range(c)]


def _start_block(start, p, n_edges):
    torch = _torch()
    if isinstance(start, np.ndarray):
        start = to_device_block(start)
    if start.dtype != torch.float64 or not start.is_contiguous() or start.numel() != p * 2 * n_edges:
        raise ValueError("start must be a contiguous FP64 planar block of p columns")
    return start


def _info_dict(inf) -> dict:
    L = inf.levels
    return {"n": inf.n, "m": inf.m, "p": inf.p, "nev": inf.nev, "levels": L,
            "precision": inf.precision, "mu": inf.mu, "device_bytes": inf.device_bytes,
            "kernel_launches": inf.kernel_launches,
            "sizes": [(inf.level_n[i], inf.level_m[i]) for i in range(L)],
            "edge_smooth_shape": list(inf.edge_smooth_shape),
            "nodal_smooth_shape": list(inf.nodal_smooth_shape),
            "rr_tile": inf.rr_tile, "autotune_ms": inf.autotune_ms,
            "fused_edge_level": inf.fused_edge_level, "fused_nodal_level": inf.fused_nodal_level,
            "locked_columns": inf.locked_columns}


def _marshal_problems(problems, want_last_vectors):
    torch = _torch()
    keep = []
    arr = (BlProblem * len(problems))()
    outs = []
    for i, pr in enumerate(problems):
        n, m = int(pr["n"]), int(pr["m"])
        nev, nthrow = int(pr["nev"]), int(pr["nthrow"])
        p, ne = nev + nthrow, 2 * n * m
        eps = np.ascontiguousarray(pr["eps"], dtype=np.float64)
        ks = np.ascontiguousarray(pr["ks"], dtype=np.float64).reshape(-1, 2)
        st = _start_block(pr["start"], p, ne) if pr.get("start") is not None else None
        nk = ks.shape[0]
        ev, rr, pm = np.zeros((nk, nev)), np.zeros((nk, nev)), np.zeros(nk)
        its = np.zeros(nk, dtype=np.int32)
        vec = torch.empty((nev, 2, ne), dtype=torch.float64, device="cuda") if want_last_vectors else None
        keep += [eps, ks, st, ev, rr, its, pm, vec]
        b = arr[i]
        b.grid = BlGrid(n, m, float(pr["a"]), float(pr["b"]))
        b.eps = _dptr(eps)
        b.nev, b.nthrow, b.nk = nev, nthrow, nk
        b.ks = _dptr(ks)
        b.start_dev = st.data_ptr() if st is not None else None
        b.evals, b.relres, b.point_ms = _dptr(ev), _dptr(rr), _dptr(pm)
        b.iters = its.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        b.evecs_dev = vec.data_ptr() if vec is not None else None
        outs.append((ev, rr, its, pm, vec))
    return arr, outs, keep


def _unmarshal(arr, outs, rc, where):
    if rc not in (native.BL_OK, native.BL_ENOCONV, native.BL_EINVAL, native.BL_ENOMEM):
        check(rc, where)
    res = []
    for i, (ev, rr, its, pm, vec) in enumerate(outs):
        res.append({"evals": ev, "relres": rr, "iterations": its, "point_ms": pm,
                    "status": int(arr[i].status), "converged": arr[i].status == 0, "evecs": vec})
    return res


def batch_solve(problems, max_slots=0, stream=None, want_last_vectors=False, **opts):
    """bl_batch_solve.  `problems`: sequence of dicts with n, m, a, b, eps (n*m), nev,
    nthrow, ks ((nk, 2) array) and start (host complex (N_e, p) or device planar block).
    Common options as for Solver.  Returns one dict per problem (evals, relres, iterations,
    point_ms, status, evecs)."""
    torch = _torch()
    lib = native.load()
    o = _make_opts(**opts)
    arr, outs, _keep = _marshal_problems(problems, want_last_vectors)
    if stream is None:
        stream = torch.cuda.current_stream()
    rc = lib.bl_batch_solve(ctypes.byref(o), arr, len(problems), int(max_slots), ctypes.c_void_p(stream.cuda_stream))
    return _unmarshal(arr, outs, rc, "bl_batch_solve")


class Batch:
    """bl_batch_*: a batch context whose shape engines persist between runs."""

    def __init__(self, max_slots=0, hbm_budget=0, **opts):
        self.lib = native.load()
        o = _make_opts(**opts)
        h = ctypes.c_void_p()
        check(self.lib.bl_batch_create(ctypes.byref(o), int(max_slots), int(hbm_budget), ctypes.byref(h)),
              "bl_batch_create")
        self.h = h

    def run(self, problems, stream=None, want_last_vectors=False):
        torch = _torch()
        arr, outs, _keep = _marshal_problems(problems, want_last_vectors)
        if stream is None:
            stream = torch.cuda.current_stream()
        rc = self.lib.bl_batch_run(self.h, arr, len(problems), ctypes.c_void_p(stream.cuda_stream))
        return _unmarshal(arr, outs, rc, "bl_batch_run")

    def engines(self) -> list:
        """bl_info of every live engine of the context."""
        out, i = [], 0
        while True:
            inf = BlInfo()
            cnt = check(self.lib.bl_batch_engine_info(self.h, i, ctypes.byref(inf)), "bl_batch_engine_info")
            if i >= cnt:
                return out
            out.append(_info_dict(inf))
            i += 1

    def set_timing(self, enable=True):
        check(self.lib.bl_batch_set_timing(self.h, 1 if enable else 0), "bl_batch_set_timing")

    def timing(self) -> dict:
        ms, cnt, cols, nb = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        check(self.lib.bl_batch_get_timing(self.h, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(cols),
                                           ctypes.byref(nb)), "bl_batch_get_timing")
        return {"total_ms": ms.value, "launches": cnt.value, "columns": cols.value, "alg_bytes": nb.value}

    def close(self):
        if getattr(self, "h", None):
            self.lib.bl_batch_destroy(self.h)
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


class Server:
    """bl_server_*: asynchronous requests with footprint admission and continuous batching.
    Keyword options as for Solver (nev/nthrow come with each request)."""

    def __init__(self, hbm_budget=0, max_slots=0, **opts):
        self.lib = native.load()
        o = _make_opts(**opts)
        h = ctypes.c_void_p()
        check(self.lib.bl_server_create(ctypes.byref(o), int(hbm_budget), int(max_slots), ctypes.byref(h)),
              "bl_server_create")
        self.h = h
        self._keep = {}

    def close(self):
        if getattr(self, "h", None):
            self.lib.bl_server_destroy(self.h)
            self.h = None
            self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, n, m, a, b, eps, nev, nthrow, ks, start) -> int:
        """Queue a request; returns its ticket.  The start block is kept alive until polled."""
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        ks = np.ascontiguousarray(ks, dtype=np.float64).reshape(-1, 2)
        st = _start_block(start, int(nev) + int(nthrow), 2 * int(n) * int(m)) if start is not None else None
        r = BlRequest()
        r.grid = BlGrid(int(n), int(m), float(a), float(b))
        r.eps = _dptr(eps)
        r.nev, r.nthrow, r.nk = int(nev), int(nthrow), ks.shape[0]
        r.ks = _dptr(ks)
        r.start_dev = st.data_ptr() if st is not None else None
        _torch().cuda.current_stream().synchronize()   # the server reads it on its own stream
        t = ctypes.c_uint64()
        check(self.lib.bl_server_submit(self.h, ctypes.byref(r), ctypes.byref(t)), "bl_server_submit")
        self._keep[t.value] = (st, ks.shape[0], int(nev))
        return t.value

    def poll(self, ticket):
        """None while the request runs, else a result dict."""
        st, nk, nev = self._keep[ticket]
        ev = np.zeros((nk, nev))
        rr = np.zeros((nk, nev))
        its = np.zeros(nk, dtype=np.int32)
        info = BlRequestInfo()
        rc = self.lib.bl_server_poll(self.h, ctypes.c_uint64(ticket), _dptr(ev), _dptr(rr),
                                     its.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(info))
        if rc == native.BL_EAGAIN:
            return None
        del self._keep[ticket]
        if rc not in (native.BL_OK, native.BL_ENOCONV):
            check(rc, "bl_server_poll")
        return {"evals": ev, "relres": rr, "iterations": its, "status": int(rc),
                "converged": rc == 0, "queue_s": info.queue_s, "run_s": info.run_s,
                "latency_s": info.latency_s, "total_iters": info.total_iters}

    def stats(self) -> dict:
        c = BlServerCounters()
        rc = self.lib.bl_server_stats(self.h, ctypes.byref(c))
        check(rc, "bl_server_stats")
        return {"rounds": c.rounds, "kernel_launches": c.kernel_launches, "device_bytes": c.device_bytes,
                "engines": c.engines, "queued": c.queued, "pending": c.pending}


class Solver:
    """Handle for one grid and permittivity (bl_create).

    Keyword options map to bl_opts fields: nev, nthrow, max_iter, levels, coarsest_min,
    nu_pre, nu_post, nodal_cycles, variant ("gradient" | "lobpcg" or 0 | 1), precision ("fp64" |
    "mixed" or 0 | 1),
    extrap_depth, tol, mu, zero_rel, lock_rel and the other bl_opts fields by name."""

    def __init__(self, n, m, a, b, eps, nev=8, stream=None, **opts):
        torch = _torch()
        self.lib = native.load()
        self.n, self.m, self.a, self.b = int(n), int(m), float(a), float(b)
        o = BlOpts()
        self.lib.bl_default_opts(ctypes.byref(o), int(nev))
        for k, v in opts.items():
            if k == "precision" and isinstance(v, str):
                v = {"fp64": 0, "mixed": 1}[v]
            if k == "variant" and isinstance(v, str):
                v = {"gradient": 0, "lobpcg": 1}[v]
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
        return _info_dict(inf)

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

    def nested_start(self, k1, k2, tol_levels=1e-3):
        """Start block for a first Bloch parameter by nested iteration (Section 6): returns the
        device block and the iterations spent per level."""
        torch = _torch()
        out = torch.empty((self.p, 2, self.n_edges), dtype=torch.float64, device="cuda")
        L = self.info()["levels"]
        its = np.zeros(L, dtype=np.int32)
        check(self.lib.bl_nested_start(self.h, float(k1), float(k2), float(tol_levels), _ptr(out),
                                       its.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), "bl_nested_start")
        return out, its

    def solve_kgrid(self, kappa, start, allow_noconv=False):
        """Every point k_ij of the kappa x kappa Bloch grid in raster order (Section 6); arrays
        are indexed [j, i]."""
        start = self._start(start)
        if start is None:
            raise ValueError("the grid's first point needs a start block")
        kappa = int(kappa)
        ev = np.zeros((kappa, kappa, self.nev))
        rr = np.zeros((kappa, kappa, self.nev))
        its = np.zeros((kappa, kappa), dtype=np.int32)
        rc = self.lib.bl_solve_kgrid(self.h, kappa, _ptr(start), ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     rr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     its.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        check(rc, "bl_solve_kgrid", allow=(native.BL_ENOCONV,) if allow_noconv else ())
        return {"evals": ev, "relres": rr, "iterations": its, "converged": rc == 0}

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
        ms, cnt, cols, nb = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        check(self.lib.bl_get_timing(self.h, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(cols),
                                     ctypes.byref(nb)), "bl_get_timing")
        return {"total_ms": ms.value, "launches": cnt.value, "columns": cols.value, "alg_bytes": nb.value}

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

    def gram_noalloc(self, X, W, out):
        """bl_gram_noalloc: out (device FP64 tensor of q * r * 2 values) = X^* W, queued on the
        handle's stream with no allocation; returns out."""
        q, r = X.shape[0], W.shape[0]
        if out.numel() < q * r * 2:
            raise ValueError("out must hold q * r complex values")
        check(self.lib.bl_gram_noalloc(self.h, _ptr(X), q, _ptr(W), r, X.shape[2], _ptr(out)), "bl_gram_noalloc")
        return out

    def rr_products(self, S):
        """(S^* M S, S^* A S) for a planar FP64 device block S (q, 2, N_e) (bl_rr_products)."""
        q = S.shape[0]
        G = np.zeros((q, q, 2))
        H = np.zeros((q, q, 2))
        check(self.lib.bl_rr_products(self.h, _ptr(S), q, _dptr(G), _dptr(H)), "bl_rr_products")
        return G[..., 0] + 1j * G[..., 1], H[..., 0] + 1j * H[..., 1]

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
