"""Python binding of libfrnn (include/frnn.h) by ctypes.

Argument marshalling only: every step of the search runs in the HIP library.
PyTorch supplies device memory and the current stream.  Importing this module
loads libfrnn.so and raises if it has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfrnn.so")

WANT_DIST2 = 1
SELF_QUERY = 2
EXCLUDE_SELF = 4

STATUS = {0: "OK", 1: "INVALID_ARG", 2: "NONFINITE", 3: "OOM", 4: "BUDGET", 5: "RADIUS",
          6: "HIP", 7: "INTERNAL", 8: "NOT_READY"}


class FrnnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


# ------------------------------------------------------------- structs
class Opts(ctypes.Structure):
    _fields_ = [("grid_axes_max", ctypes.c_int32), ("cells_per_point", ctypes.c_float),
                ("cell_multiple", ctypes.c_int32), ("cells_per_item", ctypes.c_int32),
                ("queries_per_item", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("row_cap_lds", ctypes.c_int32),
                ("stash_cap", ctypes.c_int32), ("graphs", ctypes.c_int32), ("adapt", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class _CSR(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("indices", ctypes.c_void_p),
                ("dist2", ctypes.c_void_p), ("owner_", ctypes.c_void_p)]


class _HostCSR(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("indices", ctypes.c_void_p),
                ("dist2", ctypes.c_void_p), ("owner_", ctypes.c_void_p)]


class _Edges(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p),
                ("owner_", ctypes.c_void_p)]


class _Event(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("N", ctypes.c_int64),
                ("queries", ctypes.c_void_p), ("M", ctypes.c_int64)]


class IndexInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("D", ctypes.c_int32), ("grid_axes", ctypes.c_int32),
                ("axis", ctypes.c_int32 * 8), ("cells_per_axis", ctypes.c_int32 * 8),
                ("cells", ctypes.c_int64), ("cell_width", ctypes.c_double),
                ("cell_multiple", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int64), ("work_items", ctypes.c_int64),
                ("pairs", ctypes.c_int64), ("long_row_keys", ctypes.c_int64),
                ("stash_cap", ctypes.c_int32), ("adapted", ctypes.c_int32)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int32), ("r", ctypes.c_float), ("K", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("hbm_budget_bytes", ctypes.c_int64),
                ("max_batch_events", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("opts", Opts)]


class Timing(ctypes.Structure):
    _fields_ = [("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("batch_id", ctypes.c_int32), ("batch_events", ctypes.c_int32)]


class TuneReport(ctypes.Structure):
    _fields_ = [("candidates_tried", ctypes.c_int32), ("candidates_rejected", ctypes.c_int32),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double),
                ("from_cache", ctypes.c_int32), ("density_class", ctypes.c_char * 96)]


# ------------------------------------------------------------- loading
def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2609_31980_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_float
    P = ctypes.POINTER
    sig = {
        "frnn_opts_default": (None, [P(Opts)]),
        "frnn_build": (i32, [vp, i64, i32, f32, P(Opts), vp, P(vp)]),
        "frnn_query": (i32, [vp, vp, i64, f32, i32, u32, vp, P(_CSR)]),
        "frnn_index_destroy": (None, [vp]),
        "frnn_index_get_info": (i32, [vp, P(IndexInfo)]),
        "frnn_query_batch": (i32, [P(_Event), i32, i32, f32, i32, u32, P(Opts), vp, P(_CSR)]),
        "frnn_csr_copy": (i32, [P(_CSR), vp, vp, vp, i32, vp]),
        "frnn_csr_release": (None, [P(_CSR)]),
        "frnn_csr_edges": (i32, [P(_CSR), i32, vp, P(_Edges)]),
        "frnn_edges_release": (None, [P(_Edges)]),
        "frnn_edges_copy": (i32, [P(_Edges), vp, vp, i32, vp]),
        "frnn_query_host": (i32, [vp, i64, vp, i64, i32, f32, i32, u32, P(Opts), P(_HostCSR)]),
        "frnn_host_csr_release": (None, [P(_HostCSR)]),
        "frnn_server_opts_default": (None, [P(ServerOpts)]),
        "frnn_server_create": (i32, [P(ServerOpts), P(vp)]),
        "frnn_server_submit": (i32, [vp, vp, i64, P(ctypes.c_uint64)]),
        "frnn_server_wait": (i32, [vp, ctypes.c_uint64, ctypes.c_double, P(_CSR), P(Timing)]),
        "frnn_server_destroy": (None, [vp]),
        "frnn_server_memory": (i32, [vp, P(i64), P(i64)]),
        "frnn_tune": (i32, [vp, i64, i32, f32, i32, u32, vp, P(Opts), P(TuneReport)]),
        "frnn_profile_enable": (None, [i32]),
        "frnn_profile_read": (i32, [P(KernelTime), i32, i32]),
        "frnn_last_stats": (i32, [P(Stats)]),
        "frnn_memory_stats": (None, [P(i64), P(i64)]),
        "frnn_status_str": (ctypes.c_char_p, [i32]),
        "frnn_last_error": (ctypes.c_char_p, []),
        "frnn_test_fail_alloc_after": (None, [i64]),
        "frnn_query_noalloc": (i32, [vp, i64, i32, f32, i32, u32, P(Opts), vp, vp, vp, i64, P(i64), vp]),
        "frnn_measure_valu_rate": (i32, [vp, P(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def _check(st: int):
    if st != 0:
        raise FrnnError(st, (_lib.frnn_last_error() or b"").decode())


def _stream(stream=None):
    import torch
    if stream is not None:
        return ctypes.c_void_p(stream.cuda_stream)
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:  # the handle alone, without a Stream object (a few us less)
        return ctypes.c_void_p(raw(torch.cuda.current_device()))
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _pts(t, D=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("points must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float32 or t.dim() != 2 or not t.is_contiguous():
        raise TypeError("points must be a contiguous float32 [n, D] tensor")
    if D is not None and t.shape[1] != D:
        raise ValueError(f"expected D={D}, got {t.shape[1]}")
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0)


def default_opts(**kw) -> Opts:
    o = Opts()
    _lib.frnn_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


# ------------------------------------------------------------- results
class CSR:
    """Neighbour lists on the device (library-owned until released)."""

    def __init__(self, raw: _CSR, keep=None):
        self._raw = raw
        self._keep = keep   # tensors that must outlive the device work

    @property
    def M(self) -> int:
        return int(self._raw.M)

    @property
    def nnz(self) -> int:
        return int(self._raw.nnz)

    @property
    def has_dist2(self) -> bool:
        return bool(self._raw.dist2)

    def numpy(self, stream=None):
        """(offsets int64 [M+1], indices int32 [nnz], dist2 float32 [nnz] or None)."""
        off = np.empty(self.M + 1, np.int64)
        idx = np.empty(self.nnz, np.int32)
        d2 = np.empty(self.nnz, np.float32) if self.has_dist2 else None
        _check(_lib.frnn_csr_copy(ctypes.byref(self._raw), off.ctypes.data_as(ctypes.c_void_p),
                                  idx.ctypes.data_as(ctypes.c_void_p) if self.nnz else None,
                                  d2.ctypes.data_as(ctypes.c_void_p) if (d2 is not None and self.nnz) else None,
                                  1, _stream(stream)))
        return off, idx, d2

    def torch(self, stream=None):
        """Device copies as torch tensors (offsets, indices, dist2 or None)."""
        import torch
        off = torch.empty(self.M + 1, dtype=torch.int64, device="cuda")
        idx = torch.empty(self.nnz, dtype=torch.int32, device="cuda")
        d2 = torch.empty(self.nnz, dtype=torch.float32, device="cuda") if self.has_dist2 else None
        _check(_lib.frnn_csr_copy(ctypes.byref(self._raw), ctypes.c_void_p(off.data_ptr()),
                                  ctypes.c_void_p(idx.data_ptr()) if self.nnz else None,
                                  ctypes.c_void_p(d2.data_ptr()) if (d2 is not None and self.nnz) else None,
                                  0, _stream(stream)))
        return off, idx, d2

    def edges(self, symmetrized: bool = False, stream=None) -> "Edges":
        """Undirected edges of a self-query CSR (frnn_csr_edges): (i, j) with
        i < j from each row, or with symmetrized also the pairs present in one
        direction only, each once as (min, max)."""
        e = _Edges()
        _check(_lib.frnn_csr_edges(ctypes.byref(self._raw), 1 if symmetrized else 0,
                                   _stream(stream), ctypes.byref(e)))
        return Edges(e)

    def release(self):
        if self._raw.owner_:
            _lib.frnn_csr_release(ctypes.byref(self._raw))
        self._keep = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Index:
    """A built index over device points (frnn_build)."""

    def __init__(self, points, r: float, opts: Opts | None = None, stream=None):
        self.points = points          # keep alive: the index reads it during the build
        self.N, self.D = int(points.shape[0]), int(points.shape[1])
        self.r = float(np.float32(r))
        h = ctypes.c_void_p()
        _check(_lib.frnn_build(_pts(points), self.N, self.D, self.r,
                               ctypes.byref(opts) if opts is not None else None,
                               _stream(stream), ctypes.byref(h)))
        self._h = h

    def query(self, queries=None, r: float | None = None, K: int = 0, exclude_self: bool = False,
              want_dist2: bool = True, stream=None) -> CSR:
        r = self.r if r is None else float(np.float32(r))
        flags = WANT_DIST2 if want_dist2 else 0
        if queries is None:
            flags |= SELF_QUERY
            if exclude_self:
                flags |= EXCLUDE_SELF
            qp, M = None, self.N
        else:
            qp, M = _pts(queries, self.D), int(queries.shape[0])
        out = _CSR()
        _check(_lib.frnn_query(self._h, qp, M, r, int(K), flags, _stream(stream), ctypes.byref(out)))
        return CSR(out, keep=queries)

    def info(self) -> dict:
        inf = IndexInfo()
        _check(_lib.frnn_index_get_info(self._h, ctypes.byref(inf)))
        G = inf.grid_axes
        return {"N": inf.N, "D": inf.D, "grid_axes": G, "axis": list(inf.axis)[:G],
                "cells_per_axis": list(inf.cells_per_axis)[:G], "cells": inf.cells,
                "cell_width": inf.cell_width, "cell_multiple": inf.cell_multiple}

    def close(self):
        if getattr(self, "_h", None):
            _lib.frnn_index_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Edges:
    """Undirected edge list on the device (library-owned until released)."""

    def __init__(self, raw: _Edges):
        self._raw = raw

    @property
    def n(self) -> int:
        return int(self._raw.n)

    def numpy(self, stream=None):
        """(src int32 [n], dst int32 [n]) on the host, src < dst."""
        src = np.empty(self.n, np.int32)
        dst = np.empty(self.n, np.int32)
        _check(_lib.frnn_edges_copy(ctypes.byref(self._raw), src.ctypes.data_as(ctypes.c_void_p),
                                    dst.ctypes.data_as(ctypes.c_void_p), 1, _stream(stream)))
        return src, dst

    def torch(self, stream=None):
        """Device copies (src, dst) as int32 torch tensors."""
        import torch
        src = torch.empty(self.n, dtype=torch.int32, device="cuda")
        dst = torch.empty(self.n, dtype=torch.int32, device="cuda")
        _check(_lib.frnn_edges_copy(ctypes.byref(self._raw), ctypes.c_void_p(src.data_ptr()),
                                    ctypes.c_void_p(dst.data_ptr()), 0, _stream(stream)))
        return src, dst

    def release(self):
        if self._raw.owner_:
            _lib.frnn_edges_release(ctypes.byref(self._raw))

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class HostCSR:
    """Neighbour lists in pinned host memory (frnn_query_host); the numpy
    arrays are views of the library's buffers, valid until release()."""

    def __init__(self, raw: _HostCSR):
        self._raw = raw
        M, nnz = int(raw.M), int(raw.nnz)
        self.offsets = _view(raw.offsets, ctypes.c_int64, M + 1, np.int64)
        self.indices = _view(raw.indices, ctypes.c_int32, nnz, np.int32)
        self.dist2 = _view(raw.dist2, ctypes.c_float, nnz, np.float32) if raw.dist2 else None

    @property
    def M(self) -> int:
        return int(self._raw.M)

    @property
    def nnz(self) -> int:
        return int(self._raw.nnz)

    def numpy(self):
        """Owned copies (offsets, indices, dist2 or None)."""
        return (self.offsets.copy(), self.indices.copy(),
                None if self.dist2 is None else self.dist2.copy())

    def release(self):
        if self._raw.owner_:
            self.offsets = self.indices = self.dist2 = None
            _lib.frnn_host_csr_release(ctypes.byref(self._raw))

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def _view(ptr, ctype, n, dtype):
    if not n or not ptr:
        return np.zeros(n, dtype)
    return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctype)), shape=(n,))


def query_host(points: np.ndarray, r: float, K: int = 0, queries: np.ndarray | None = None,
               exclude_self: bool = False, want_dist2: bool = True,
               opts: Opts | None = None) -> HostCSR:
    """Synchronous search on host float32 arrays; the CSR comes back in
    pinned host memory (frnn_query_host)."""
    x = np.ascontiguousarray(points, dtype=np.float32)
    if x.ndim != 2:
        raise ValueError("points must be [N, D]")
    flags = (WANT_DIST2 if want_dist2 else 0)
    q = None
    if queries is None:
        flags |= SELF_QUERY | (EXCLUDE_SELF if exclude_self else 0)
        M = x.shape[0]
    else:
        if exclude_self:
            raise ValueError("exclude_self needs a self-query")
        q = np.ascontiguousarray(queries, dtype=np.float32)
        if q.ndim != 2 or q.shape[1] != x.shape[1]:
            raise ValueError("queries must be [M, D] with the points' D")
        M = q.shape[0]
    out = _HostCSR()
    _check(_lib.frnn_query_host(x.ctypes.data_as(ctypes.c_void_p), x.shape[0],
                                q.ctypes.data_as(ctypes.c_void_p) if q is not None else None, M,
                                x.shape[1], float(np.float32(r)), int(K), flags,
                                ctypes.byref(opts) if opts is not None else None, ctypes.byref(out)))
    return HostCSR(out)


def build(points, r: float, opts: Opts | None = None, stream=None) -> Index:
    return Index(points, r, opts, stream)


def query_batch(points: list, r: float, K: int = 0, queries: list | None = None,
                exclude_self: bool = False, want_dist2: bool = True, opts: Opts | None = None,
                stream=None) -> list[CSR]:
    """One batched pipeline over many events (self-queries unless queries given)."""
    E = len(points)
    D = int(points[0].shape[1])
    ev = (_Event * E)()
    flags = WANT_DIST2 if want_dist2 else 0
    if queries is None:
        flags |= SELF_QUERY
        if exclude_self:
            flags |= EXCLUDE_SELF
    for e, p in enumerate(points):
        ev[e].points = _pts(p, D)
        ev[e].N = int(p.shape[0])
        if queries is not None:
            ev[e].queries = _pts(queries[e], D)
            ev[e].M = int(queries[e].shape[0])
    outs = (_CSR * E)()
    _check(_lib.frnn_query_batch(ev, E, D, float(np.float32(r)), int(K), flags,
                                 ctypes.byref(opts) if opts is not None else None,
                                 _stream(stream), outs))
    keep = (points, queries)
    return [CSR(outs[e], keep=keep) for e in range(E)]


def query_noalloc(points, r: float, K: int, offsets, indices, dist2=None, exclude_self: bool = False,
                  opts: Opts | None = None, stream=None) -> int:
    """Self-query of one event with no device allocation by the library
    (frnn_query_noalloc): writes the CSR into the caller's tensors (offsets
    int64 [N+1], indices int32 [cap], dist2 float32 [cap] or None) and
    returns the pair count.  A FrnnError of status BUDGET carries the
    needed capacity as `.nnz`."""
    import torch
    n = int(points.shape[0])
    for t, dt, what in ((offsets, torch.int64, "offsets"), (indices, torch.int32, "indices"),
                        (dist2, torch.float32, "dist2")):
        if t is not None and (not t.is_cuda or t.dtype != dt or not t.is_contiguous()):
            raise TypeError(f"{what} must be a contiguous CUDA {dt} tensor")
    if offsets.numel() != n + 1:
        raise ValueError("offsets must hold N + 1 entries")
    cap = int(indices.numel())
    if dist2 is not None and dist2.numel() < cap:
        raise ValueError("dist2 must hold as many entries as indices")
    flags = SELF_QUERY | (WANT_DIST2 if dist2 is not None else 0) | (EXCLUDE_SELF if exclude_self else 0)
    nnz = ctypes.c_int64(0)
    st = _lib.frnn_query_noalloc(_pts(points), n, int(points.shape[1]), float(np.float32(r)), int(K), flags,
                                 ctypes.byref(opts) if opts is not None else None,
                                 ctypes.c_void_p(offsets.data_ptr()),
                                 ctypes.c_void_p(indices.data_ptr() if cap else 0),
                                 ctypes.c_void_p(dist2.data_ptr() if dist2 is not None and cap else 0),
                                 cap, ctypes.byref(nnz), _stream(stream))
    if st != 0:
        e = FrnnError(st, (_lib.frnn_last_error() or b"").decode())
        e.nnz = int(nnz.value)
        raise e
    return int(nnz.value)


# ------------------------------------------------------------- serving
class Server:
    """Continuous-batching request loop (frnn_server_*)."""

    def __init__(self, D: int, r: float, K: int = 0, hbm_budget_bytes: int = 64 << 30,
                 max_batch_events: int = 64, max_inflight: int = 2, want_dist2: bool = True,
                 exclude_self: bool = False, opts: Opts | None = None):
        so = ServerOpts()
        _lib.frnn_server_opts_default(ctypes.byref(so))
        so.D, so.r, so.K = D, float(np.float32(r)), K
        so.flags = (WANT_DIST2 if want_dist2 else 0) | SELF_QUERY | (EXCLUDE_SELF if exclude_self else 0)
        so.hbm_budget_bytes = int(hbm_budget_bytes)
        so.max_batch_events = max_batch_events
        so.max_inflight = max_inflight
        if opts is not None:
            so.opts = opts
        h = ctypes.c_void_p()
        _check(_lib.frnn_server_create(ctypes.byref(so), ctypes.byref(h)))
        self._h = h
        self.D = D

    def submit(self, host_points: np.ndarray) -> int:
        a = np.ascontiguousarray(host_points, dtype=np.float32)
        if a.ndim != 2 or a.shape[1] != self.D:
            raise ValueError("host points must be float32 [N, D]")
        t = ctypes.c_uint64()
        _check(_lib.frnn_server_submit(self._h, a.ctypes.data_as(ctypes.c_void_p), a.shape[0],
                                       ctypes.byref(t)))
        return int(t.value)

    def wait(self, ticket: int, timeout_s: float = -1.0):
        out, tm = _CSR(), Timing()
        _check(_lib.frnn_server_wait(self._h, ticket, float(timeout_s), ctypes.byref(out),
                                     ctypes.byref(tm)))
        return CSR(out), {k: getattr(tm, k) for k, _ in Timing._fields_}

    def memory(self):
        """(held, peak) device bytes charged to the server's budget."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.frnn_server_memory(self._h, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def close(self):
        if getattr(self, "_h", None):
            _lib.frnn_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- tools
def tune(points, r: float, K: int = 0, stream=None):
    """Autotune kernel parameters on this input; returns (Opts, report dict)."""
    best, rep = Opts(), TuneReport()
    _check(_lib.frnn_tune(_pts(points), int(points.shape[0]), int(points.shape[1]),
                          float(np.float32(r)), int(K), WANT_DIST2 | SELF_QUERY,
                          _stream(stream), ctypes.byref(best), ctypes.byref(rep)))
    out = {k: getattr(rep, k) for k, _ in TuneReport._fields_}
    out["density_class"] = out["density_class"].decode()
    return best, out


def profile_enable(on: bool = True):
    _lib.frnn_profile_enable(1 if on else 0)


def profile_read(reset: bool = True) -> dict:
    n = _lib.frnn_profile_read(None, 0, 0)
    arr = (KernelTime * max(n, 1))()
    n = _lib.frnn_profile_read(arr, n, 1 if reset else 0)
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(n)}


def measure_valu_rate(stream=None) -> float:
    """Measured float32 subtract/multiply/add rate of the device (ops/s)."""
    v = ctypes.c_double(0.0)
    _check(_lib.frnn_measure_valu_rate(_stream(stream), ctypes.byref(v)))
    return float(v.value)


def last_stats() -> dict:
    s = Stats()
    _check(_lib.frnn_last_stats(ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in Stats._fields_}


def memory_stats():
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _lib.frnn_memory_stats(ctypes.byref(a), ctypes.byref(b))
    return int(a.value), int(b.value)


def fail_alloc_after(k: int):
    """Test hook: the k-th device allocation from now fails (0 = off)."""
    _lib.frnn_test_fail_alloc_after(int(k))
