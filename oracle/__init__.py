"""CPU oracle for exact fixed-radius neighbour search (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never loads it.  It wraps
`frnn_oracle.c`, the brute-force definition of the relation of Eq. (1) with
the optional K cap of Sec. 1 (see that file's header for the float32
reading).  Its pins live in the test suite.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "frnn_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# -ffp-contract=off: no fused multiply-add; -mfpmath=sse: no x87 excess
# precision; no -ffast-math: subnormals are kept and nothing is reassociated.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
          "-msse2", "-mfpmath=sse", "-fno-fast-math", "-pthread"]


def build(src: str = SRC, out: str = LIB, extra: list[str] | None = None) -> str:
    """Compile the oracle with gcc; always recompiles."""
    cmd = ["gcc", *CFLAGS, *(extra or []), src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


class _CSR(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("offsets", ctypes.POINTER(ctypes.c_int64)),
                ("indices", ctypes.POINTER(ctypes.c_int32)),
                ("dist2", ctypes.POINTER(ctypes.c_float)),
                ("degree", ctypes.POINTER(ctypes.c_int64))]


@dataclass
class CSR:
    offsets: np.ndarray   # int64 [M+1]
    indices: np.ndarray   # int32 [nnz]
    dist2: np.ndarray     # float32 [nnz]
    degree: np.ndarray    # int64 [M], in-radius count before the cap

    @property
    def nnz(self) -> int:
        return int(self.offsets[-1])

    def row(self, i: int):
        a, b = int(self.offsets[i]), int(self.offsets[i + 1])
        return self.indices[a:b], self.dist2[a:b]


class OracleError(RuntimeError):
    pass


_ERRS = {-1: "invalid argument", -2: "non-finite input", -3: "out of memory"}


class Oracle:
    """ctypes front end of one compiled oracle library."""

    def __init__(self, lib_path: str = LIB):
        if not os.path.exists(lib_path):
            build(out=lib_path)
        lib = ctypes.CDLL(lib_path)
        f32p = ctypes.POINTER(ctypes.c_float)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_r2.argtypes = [ctypes.c_float]
        lib.oracle_r2.restype = ctypes.c_float
        lib.oracle_frnn.argtypes = [f32p, ctypes.c_int64, f32p, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_float, ctypes.c_int32, i64p, ctypes.c_int,
                                    ctypes.POINTER(_CSR)]
        lib.oracle_frnn.restype = ctypes.c_int
        lib.oracle_degrees.argtypes = [f32p, ctypes.c_int64, f32p, ctypes.c_int64, ctypes.c_int32,
                                       ctypes.c_float, i64p, ctypes.c_int, i64p]
        lib.oracle_degrees.restype = ctypes.c_int
        lib.oracle_csr_free.argtypes = [ctypes.POINTER(_CSR)]
        lib.oracle_threads_default.restype = ctypes.c_int
        self.lib = lib

    @staticmethod
    def _f32(a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        if a.ndim != 2:
            raise ValueError("expected a 2-D [n, D] array")
        return a

    def r2(self, r: float) -> np.float32:
        return np.float32(self.lib.oracle_r2(float(np.float32(r))))

    def threads(self) -> int:
        return int(self.lib.oracle_threads_default())

    def frnn(self, X, r: float, K: int = 0, Q=None, self_ids=None,
             exclude_self: bool = False, nthreads: int = 0) -> CSR:
        """Rows of the relation for every query (Q defaults to X).

        exclude_self (self-join only) drops j == i; self_ids gives explicit
        per-query reference ids to drop instead (for query subsets)."""
        X = self._f32(X)
        Qa = X if Q is None else self._f32(Q)
        if Qa.shape[1] != X.shape[1]:
            raise ValueError("query and reference dimension differ")
        M, N, D = Qa.shape[0], X.shape[0], X.shape[1]
        ids = None
        if exclude_self:
            if Q is not None and self_ids is None:
                raise ValueError("exclude_self needs a self-join or self_ids")
            self_ids = np.arange(M) if self_ids is None else self_ids
        if self_ids is not None:
            ids = np.ascontiguousarray(self_ids, dtype=np.int64)
            if ids.shape != (M,):
                raise ValueError("self_ids must have one entry per query")
        out = _CSR()
        f32p = ctypes.POINTER(ctypes.c_float)
        st = self.lib.oracle_frnn(
            Qa.ctypes.data_as(f32p), M, X.ctypes.data_as(f32p), N, D,
            float(np.float32(r)), int(K),
            ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if ids is not None else None,
            int(nthreads), ctypes.byref(out))
        if st != 0:
            raise OracleError(_ERRS.get(st, str(st)))
        try:
            nnz = out.nnz
            res = CSR(np.ctypeslib.as_array(out.offsets, (M + 1,)).copy(),
                      np.ctypeslib.as_array(out.indices, (max(nnz, 1),))[:nnz].copy(),
                      np.ctypeslib.as_array(out.dist2, (max(nnz, 1),))[:nnz].copy(),
                      np.ctypeslib.as_array(out.degree, (max(M, 1),))[:M].copy())
        finally:
            self.lib.oracle_csr_free(ctypes.byref(out))
        return res

    def degrees(self, X, r: float, Q=None, self_ids=None, nthreads: int = 0) -> np.ndarray:
        """In-radius counts per query, before any cap."""
        X = self._f32(X)
        Qa = X if Q is None else self._f32(Q)
        M, N, D = Qa.shape[0], X.shape[0], X.shape[1]
        deg = np.zeros(max(M, 1), dtype=np.int64)
        ids = None if self_ids is None else np.ascontiguousarray(self_ids, dtype=np.int64)
        f32p = ctypes.POINTER(ctypes.c_float)
        i64p = ctypes.POINTER(ctypes.c_int64)
        st = self.lib.oracle_degrees(Qa.ctypes.data_as(f32p), M, X.ctypes.data_as(f32p), N, D,
                                     float(np.float32(r)),
                                     ids.ctypes.data_as(i64p) if ids is not None else None,
                                     int(nthreads), deg.ctypes.data_as(i64p))
        if st != 0:
            raise OracleError(_ERRS.get(st, str(st)))
        return deg[:M]


_default: Oracle | None = None


def get() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
