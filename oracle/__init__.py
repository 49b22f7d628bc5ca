"""CPU oracle for C = P^T A P (test infrastructure only).

The oracle is a plain C implementation (ptap_oracle.c) of the definitions in Section 3 of
the paper (Eq. allatonce, Eq. allatoncerow) and of the adjoint of Eq. tripleproduct.  The
product can split its output rows over threads (each row is computed the same way, so the
result is bit-identical to one thread) and can accumulate in long double as a diagnostic of
its own FP64 rounding.  It shares nothing with the GPU library.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg use it.

Parity pins: see tests/test_oracle.py (dense products, Kronecker closed forms, boolean
pattern products, probe identities, the worked row-wise example, finite differences).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ptap_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile the oracle with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"],
                   check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(lib):
    """Declare the C signatures on a loaded oracle library."""
    i32p = ctypes.POINTER(ctypes.c_int32)
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.oracle_rap.restype = ctypes.c_int
    lib.oracle_rap.argtypes = [
        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
        i32p, i32p, f64p, i32p, i32p, f64p, i32p, i32p, f64p,
        i32p, ctypes.c_int32, ctypes.c_int,
        ctypes.POINTER(i32p), ctypes.POINTER(i32p), ctypes.POINTER(f64p), ctypes.POINTER(f64p),
        ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_rap_ex.restype = ctypes.c_int
    lib.oracle_rap_ex.argtypes = [
        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
        i32p, i32p, f64p, i32p, i32p, f64p, i32p, i32p, f64p,
        i32p, ctypes.c_int32, ctypes.c_int, ctypes.c_int32,
        ctypes.POINTER(i32p), ctypes.POINTER(i32p), ctypes.POINTER(f64p), ctypes.POINTER(f64p),
        ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_ptap_backward.restype = ctypes.c_int
    lib.oracle_ptap_backward.argtypes = [
        ctypes.c_int32, ctypes.c_int32, i32p, i32p, f64p, i32p, i32p, f64p, i32p, i32p, f64p,
        f64p, f64p]
    lib.oracle_free.restype = None
    lib.oracle_free.argtypes = [ctypes.c_void_p]
    return lib


class use_library:
    """Context manager that points the wrappers at another build of the oracle source
    (used by the tests that plant a mistake in a copy of the oracle)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _load()
        _lib = _bind(ctypes.CDLL(self.path))
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


@dataclass
class OracleResult:
    """Rows of C (all of them, or the selected ones) with the magnitude bound Cabs."""

    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray | None
    abs: np.ndarray | None
    rows: np.ndarray | None  # the selected rows, or None for all rows

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


def _arrays(M, need_val):
    rp = np.ascontiguousarray(M.rowptr, dtype=np.int32)
    c = np.ascontiguousarray(M.col, dtype=np.int32)
    v = np.ascontiguousarray(M.val, dtype=np.float64) if need_val else None
    return rp, c, v


PATTERN_ONLY = 1
LONG_DOUBLE = 2


def cores() -> int:
    """Threads for the parallel oracle: the CPUs this process may run on, capped by
    OMP_NUM_THREADS when that is set (a host shared between jobs sets it to this job's share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover - not Linux
        n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS", "")
    if cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def rap(Q1, A, Q2, *, rows=None, pattern_only: bool = False, long_double: bool = False,
        threads: int = 1) -> OracleResult:
    """C = Q1^T A Q2 for CSR inputs (objects with n_rows, n_cols, rowptr, col, val).

    long_double: sum each row's terms in long double and round once (diagnostic).
    threads: split the output rows over that many threads (bit-identical to one thread)."""
    lib = _load()
    n = A.n_rows
    if A.n_cols != n or Q1.n_rows != n or Q2.n_rows != n:
        raise ValueError("shape mismatch")
    need = not pattern_only
    Arp, Ac, Av = _arrays(A, need)
    Q1rp, Q1c, Q1v = _arrays(Q1, need)
    Q2rp, Q2c, Q2v = _arrays(Q2, need)
    sel = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
    orp = ctypes.POINTER(ctypes.c_int32)()
    oc = ctypes.POINTER(ctypes.c_int32)()
    ov = ctypes.POINTER(ctypes.c_double)()
    oa = ctypes.POINTER(ctypes.c_double)()
    onnz = ctypes.c_int64()
    flags = (PATTERN_ONLY if pattern_only else 0) | (LONG_DOUBLE if long_double else 0)
    args = (n, Q1.n_cols, Q2.n_cols, _ip(Arp), _ip(Ac), _dp(Av), _ip(Q1rp), _ip(Q1c), _dp(Q1v),
            _ip(Q2rp), _ip(Q2c), _dp(Q2v), _ip(sel) if sel is not None else None,
            0 if sel is None else sel.size)
    outs = (ctypes.byref(orp), ctypes.byref(oc), ctypes.byref(ov), ctypes.byref(oa), ctypes.byref(onnz))
    if flags == (PATTERN_ONLY if pattern_only else 0) and threads == 1:
        rc = lib.oracle_rap(*args, 1 if pattern_only else 0, *outs)
    else:
        rc = lib.oracle_rap_ex(*args, flags, int(threads), *outs)
    if rc != 0:
        raise RuntimeError(f"oracle_rap failed ({rc})")
    nout = Q1.n_cols if sel is None else sel.size
    nnz = onnz.value
    try:
        rowptr = np.ctypeslib.as_array(orp, shape=(nout + 1,)).copy()
        col = np.ctypeslib.as_array(oc, shape=(max(nnz, 1),))[:nnz].copy()
        val = absv = None
        if not pattern_only:
            val = np.ctypeslib.as_array(ov, shape=(max(nnz, 1),))[:nnz].copy()
            absv = np.ctypeslib.as_array(oa, shape=(max(nnz, 1),))[:nnz].copy()
    finally:
        for p in (orp, oc, ov, oa):
            if p:
                lib.oracle_free(ctypes.cast(p, ctypes.c_void_p))
    return OracleResult(rowptr, col, val, absv, sel)


def ptap(A, P, *, rows=None, pattern_only: bool = False, long_double: bool = False,
         threads: int = 1) -> OracleResult:
    """C = P^T A P (Section 3, Eq. tripleproduct), row form of Eq. allatonce."""
    return rap(P, A, P, rows=rows, pattern_only=pattern_only, long_double=long_double,
               threads=threads)


def ptap_backward(A, P, C_rowptr, C_col, W):
    """(dA, dP) of L = sum W o (P^T A P), masked to the patterns of A and P."""
    lib = _load()
    Arp, Ac, Av = _arrays(A, True)
    Prp, Pc, Pv = _arrays(P, True)
    Crp = np.ascontiguousarray(C_rowptr, dtype=np.int32)
    Cc = np.ascontiguousarray(C_col, dtype=np.int32)
    Wv = np.ascontiguousarray(W, dtype=np.float64)
    dA = np.zeros(Ac.size)
    dP = np.zeros(Pc.size)
    rc = lib.oracle_ptap_backward(A.n_rows, P.n_cols, _ip(Arp), _ip(Ac), _dp(Av), _ip(Prp), _ip(Pc),
                                  _dp(Pv), _ip(Crp), _ip(Cc), _dp(Wv), _dp(dA), _dp(dP))
    if rc != 0:
        raise RuntimeError(f"oracle_ptap_backward failed ({rc})")
    return dA, dP
