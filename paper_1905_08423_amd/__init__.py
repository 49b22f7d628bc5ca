"""Python binding of libptap.so, the MI355X library for C = P^T A P (all-at-once, merged
all-at-once and two-step; Section 3 of the paper).

The functions named ptap_* are thin ctypes marshals of the C ABI in include/ptap.h, with the
same names and arguments.  Every computation runs in the library's HIP kernels; PyTorch only
provides device memory (through the plan allocator) and the current stream.  If the library
is not built, loading fails loudly: there is no fallback.

Higher-level helpers: Plan (owns the pattern tensors and the plan handle), ptap() for a
one-shot product, and PtAPFunction, a torch.autograd.Function whose backward calls
ptap_backward.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libptap.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "ptap.h")

# ptap_status
PTAP_OK, PTAP_ERR_INPUT, PTAP_ERR_TOO_LARGE, PTAP_ERR_OOM, PTAP_ERR_HIP, PTAP_ERR_STATE, PTAP_ERR_UNSUPPORTED = range(7)
# ptap_algo
PTAP_ALLATONCE, PTAP_MERGED, PTAP_TWOSTEP = range(3)
# ptap_fold
PTAP_FOLD_AUTO, PTAP_FOLD_ATOMIC, PTAP_FOLD_OWNER = range(3)

ALGOS = {"allatonce": PTAP_ALLATONCE, "merged": PTAP_MERGED, "twostep": PTAP_TWOSTEP}
FOLDS = {"auto": PTAP_FOLD_AUTO, "atomic": PTAP_FOLD_ATOMIC, "owner": PTAP_FOLD_OWNER}


class ptap_allocator(ctypes.Structure):
    _fields_ = [("alloc", ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)),
                ("release", ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)),
                ("ctx", ctypes.c_void_p)]


class ptap_options(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("fold", ctypes.c_int32), ("nblocks", ctypes.c_int32),
                ("tile_entries", ctypes.c_int32), ("hash_slots", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("backward", ctypes.c_int32), ("owner_waves", ctypes.c_int32),
                ("tile_lds", ctypes.c_int32), ("cache", ctypes.c_int32),
                ("owner_kernel", ctypes.c_int32), ("hash_mul", ctypes.c_uint32),
                ("reserved", ctypes.c_int32 * 3)]


class ptap_stats(ctypes.Structure):
    _fields_ = [("nnz_C", ctypes.c_int64), ("nnz_AP", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("peak_bytes", ctypes.c_int64),
                ("pattern_bytes", ctypes.c_int64), ("rows_formed", ctypes.c_int64),
                ("rows_needed", ctypes.c_int64), ("fold_terms", ctypes.c_int64),
                ("n_tiles", ctypes.c_int32), ("fold_used", ctypes.c_int32),
                ("algo", ctypes.c_int32), ("nblocks", ctypes.c_int32),
                ("cache_bytes", ctypes.c_int64), ("block_size", ctypes.c_int64),
                ("staged_tiles", ctypes.c_int64), ("staged_lds_bytes", ctypes.c_int64),
                ("table_slots", ctypes.c_int64), ("tile_entries", ctypes.c_int64),
                ("est_owner_ms", ctypes.c_double), ("est_atomic_ms", ctypes.c_double),
                ("hash_mul", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_SIGNATURES = {
    "ptap_options_default": (None, [ctypes.POINTER(ptap_options)]),
    "ptap_plan_create": (ctypes.c_int, [ctypes.POINTER(_vp), _i32, _i32, _vp, _vp, _i64, _vp, _vp, _i64,
                                        ctypes.POINTER(ptap_options), ctypes.POINTER(ptap_allocator), _vp]),
    "ptap_plan_create_bsr": (ctypes.c_int, [ctypes.POINTER(_vp), _i32, _i32, _i32, _vp, _vp, _i64, _vp, _vp,
                                            _i64, ctypes.POINTER(ptap_options), ctypes.POINTER(ptap_allocator),
                                            _vp]),
    "ptap_symbolic": (ctypes.c_int, [_vp, _vp]),
    "ptap_get_pattern": (ctypes.c_int, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "ptap_copy_pattern": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "ptap_numeric": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "ptap_numeric_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "ptap_backward": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ptap_plan_stats": (ctypes.c_int, [_vp, ctypes.POINTER(ptap_stats)]),
    "ptap_plan_destroy": (None, [_vp]),
    "ptap_batch_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_i32), _i32,
                                         ctypes.POINTER(ptap_allocator), _vp]),
    "ptap_batch_numeric": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]),
    "ptap_batch_destroy": (None, [_vp]),
    "ptap_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ptap_last_hip_error": (_i32, []),
    "ptap_stream_sum": (ctypes.c_int, [_vp, _i64, _vp, _vp]),
}

_lib = None


def header_functions() -> list[str]:
    """Names of the functions declared in include/ptap.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ptap_[a-z_]+)\s*\(", text)) - {"ptap_status", "ptap_algo", "ptap_fold"})


def load_library(path: str = LIB_PATH):
    """Load libptap.so and declare the C signatures.  Raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built: run python -m paper_1905_08423_amd.build "
                               "(there is no fallback implementation)")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


class PtapError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load_library()
        msg = lib.ptap_status_string(status).decode()
        hip = lib.ptap_last_hip_error()
        super().__init__(f"{where}: {msg} (status {status}, hip error {hip})")
        self.status = status


def _check(status: int, where: str):
    if status != PTAP_OK:
        raise PtapError(status, where)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        if not torch.cuda.is_available():
            return None  # argument checks only; nothing can run without a device
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------------------------------------
# Thin marshals with the C names
# ---------------------------------------------------------------------------------------------

def ptap_options_default() -> ptap_options:
    o = ptap_options()
    load_library().ptap_options_default(ctypes.byref(o))
    return o


def ptap_plan_create(n, m, A_rowptr, A_col, A_nnz, P_rowptr, P_col, P_nnz, opts=None, alloc=None,
                     stream=None):
    h = ctypes.c_void_p()
    st = load_library().ptap_plan_create(ctypes.byref(h), n, m, _ptr(A_rowptr), _ptr(A_col), A_nnz,
                                         _ptr(P_rowptr), _ptr(P_col), P_nnz,
                                         ctypes.byref(opts) if opts is not None else None,
                                         ctypes.byref(alloc) if alloc is not None else None,
                                         _stream(stream))
    return st, h


def ptap_plan_create_bsr(nb, mb, bs, A_rowptr, A_col, A_nnzb, P_rowptr, P_col, P_nnzb, opts=None,
                         alloc=None, stream=None):
    h = ctypes.c_void_p()
    st = load_library().ptap_plan_create_bsr(ctypes.byref(h), nb, mb, bs, _ptr(A_rowptr), _ptr(A_col),
                                             A_nnzb, _ptr(P_rowptr), _ptr(P_col), P_nnzb,
                                             ctypes.byref(opts) if opts is not None else None,
                                             ctypes.byref(alloc) if alloc is not None else None,
                                             _stream(stream))
    return st, h


def ptap_symbolic(plan, stream=None):
    return load_library().ptap_symbolic(plan, _stream(stream))


def ptap_get_pattern(plan):
    nnz = _i64()
    rp = ctypes.c_void_p()
    col = ctypes.c_void_p()
    st = load_library().ptap_get_pattern(plan, ctypes.byref(nnz), ctypes.byref(rp), ctypes.byref(col))
    return st, nnz.value, rp.value, col.value


def ptap_copy_pattern(plan, C_rowptr, C_col, stream=None):
    return load_library().ptap_copy_pattern(plan, _ptr(C_rowptr), _ptr(C_col), _stream(stream))


def ptap_numeric(plan, A_val, P_val, C_val, stream=None):
    return load_library().ptap_numeric(plan, _ptr(A_val), _ptr(P_val), _ptr(C_val), _stream(stream))


def ptap_numeric_noalloc(plan, A_val, P_val, C_val, stream=None):
    return load_library().ptap_numeric_noalloc(plan, _ptr(A_val), _ptr(P_val), _ptr(C_val), _stream(stream))


def ptap_backward(plan, A_val, P_val, dC_val, dA_val, dP_val, stream=None):
    return load_library().ptap_backward(plan, _ptr(A_val), _ptr(P_val), _ptr(dC_val), _ptr(dA_val),
                                        _ptr(dP_val), _stream(stream))


def ptap_plan_stats(plan):
    s = ptap_stats()
    st = load_library().ptap_plan_stats(plan, ctypes.byref(s))
    return st, s


def ptap_plan_destroy(plan):
    load_library().ptap_plan_destroy(plan)


def ptap_batch_create(plans, levels=None, alloc=None, stream=None):
    h = ctypes.c_void_p()
    arr = (ctypes.c_void_p * len(plans))(*[p.value if isinstance(p, ctypes.c_void_p) else p for p in plans])
    lv = None if levels is None else (ctypes.c_int32 * len(plans))(*levels)
    st = load_library().ptap_batch_create(ctypes.byref(h), arr, lv, len(plans),
                                          ctypes.byref(alloc) if alloc is not None else None,
                                          _stream(stream))
    return st, h


def ptap_batch_numeric(batch, A_vals, P_vals, C_vals, stream=None):
    k = len(A_vals)
    mk = lambda ts: (ctypes.c_void_p * k)(*[t.data_ptr() for t in ts])  # noqa: E731
    return load_library().ptap_batch_numeric(batch, mk(A_vals), mk(P_vals), mk(C_vals), _stream(stream))


def ptap_batch_destroy(batch):
    load_library().ptap_batch_destroy(batch)


def ptap_status_string(status):
    return load_library().ptap_status_string(status).decode()


def ptap_last_hip_error():
    return load_library().ptap_last_hip_error()


def stream_sum(x, out=None, stream=None):
    """Sum of the FP64 tensor x by the library's streaming-read kernel (a bandwidth probe)."""
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=x.device)
    _check(load_library().ptap_stream_sum(_ptr(x), int(x.numel()), _ptr(out), _stream(stream)),
           "ptap_stream_sum")
    return out


# ---------------------------------------------------------------------------------------------
# Torch-backed allocator: every plan buffer is a torch tensor, so torch's memory statistics
# see the plan's workspace.
# ---------------------------------------------------------------------------------------------
class TorchAllocator:
    """The library releases a buffer as soon as it has enqueued the last launch that uses it, so
    a release is stream-ordered: the tensor is marked as used on the plan's stream
    (record_stream) before it is dropped, and torch's caching allocator does not hand the block
    to another stream until that work is done.  Without an explicit stream the plan runs on
    torch's current stream, where torch already orders reuse."""

    def __init__(self, device=None, stream=None):
        self.device = torch.device("cuda") if device is None else torch.device(device)
        self.stream = stream if isinstance(stream, torch.cuda.Stream) else None
        self.live = {}
        alloc_t = ptap_allocator._fields_[0][1]
        release_t = ptap_allocator._fields_[1][1]

        def _alloc(nbytes, ctx):
            try:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            except RuntimeError:
                return None
            self.live[t.data_ptr()] = t
            return t.data_ptr()

        def _release(ptr, nbytes, ctx):
            t = self.live.pop(ptr, None)
            if t is not None and self.stream is not None:
                t.record_stream(self.stream)

        self.c_alloc = alloc_t(_alloc)
        self.c_release = release_t(_release)
        self.struct = ptap_allocator(self.c_alloc, self.c_release, None)

    @property
    def held_bytes(self):
        return sum(t.numel() for t in self.live.values())


class Plan:
    """A plan for C = P^T A P on fixed patterns of A and P (device tensors).

    algo: "allatonce" | "merged" | "twostep"; fold: "auto" | "atomic" | "owner"; nblocks: K.
    block_size > 1 makes a block-sparse plan (ptap_plan_create_bsr): n, m and the patterns count
    blocks, and values are blocks of block_size^2 doubles (row-major).
    The symbolic phase runs at construction; numeric() may be called many times."""

    def __init__(self, n, m, A_rowptr, A_col, P_rowptr, P_col, *, algo="merged", fold="auto",
                 nblocks=1, tile_entries=0, hash_slots=0, validate=True, xcd_remap=True,
                 backward=False, owner_waves=0, tile_lds=0, cache=False, staged=False, block_size=1,
                 hash_mul=0, allocator=None, stream=None):
        load_library()
        self.n, self.m = int(n), int(m)
        self.A_rowptr, self.A_col = A_rowptr, A_col
        self.P_rowptr, self.P_col = P_rowptr, P_col
        self.A_nnz, self.P_nnz = int(A_col.numel()), int(P_col.numel())
        self.allocator = allocator if allocator is not None else TorchAllocator(A_rowptr.device, stream)
        o = ptap_options_default()
        o.algo = ALGOS[algo] if isinstance(algo, str) else int(algo)
        o.fold = FOLDS[fold] if isinstance(fold, str) else int(fold)
        o.nblocks = int(nblocks)
        o.tile_entries = int(tile_entries)
        o.hash_slots = int(hash_slots)
        # the plan's symbolic phase follows right below, so the check at creation covers it
        o.validate = 2 if validate else 0
        o.xcd_remap = 1 if xcd_remap else 0
        o.backward = 1 if backward else 0
        o.owner_waves = int(owner_waves)
        o.tile_lds = int(tile_lds)
        o.cache = 1 if cache else 0
        o.owner_kernel = 1 if staged else 0
        o.hash_mul = int(hash_mul)
        self.options = o
        self.handle = None
        self.bs = int(block_size)
        if self.bs == 1:
            st, h = ptap_plan_create(self.n, self.m, A_rowptr, A_col, self.A_nnz, P_rowptr, P_col,
                                     self.P_nnz, o, self.allocator.struct, stream)
            _check(st, "ptap_plan_create")
        else:
            st, h = ptap_plan_create_bsr(self.n, self.m, self.bs, A_rowptr, A_col, self.A_nnz, P_rowptr,
                                         P_col, self.P_nnz, o, self.allocator.struct, stream)
            _check(st, "ptap_plan_create_bsr")
        self.handle = h
        _check(ptap_symbolic(self.handle, stream), "ptap_symbolic")
        st, nnz, rp, col = ptap_get_pattern(self.handle)
        _check(st, "ptap_get_pattern")
        self.nnz_C = nnz
        self._rp_ptr, self._col_ptr = rp, col

    @classmethod
    def from_csr(cls, A, P, device="cuda", **kw):
        """Build from host CSR objects (rowptr, col arrays) -- copies the patterns to the device."""
        dev = torch.device(device)
        t = lambda a: torch.as_tensor(a, dtype=torch.int32).to(dev)  # noqa: E731
        plan = cls(A.n_rows, P.n_cols, t(A.rowptr), t(A.col), t(P.rowptr), t(P.col), **kw)
        return plan

    def pattern(self):
        """(C_rowptr, C_col) as new int32 device tensors (copies of the plan-owned arrays)."""
        rp = torch.empty(self.m + 1, dtype=torch.int32, device=self.A_rowptr.device)
        col = torch.empty(max(self.nnz_C, 0), dtype=torch.int32, device=self.A_rowptr.device)
        _check(ptap_copy_pattern(self.handle, rp, col if self.nnz_C else None), "ptap_copy_pattern")
        return rp, col

    def numeric(self, A_val, P_val, C_val=None, stream=None):
        b2 = self.bs * self.bs
        if A_val.numel() != self.A_nnz * b2 or P_val.numel() != self.P_nnz * b2:
            raise ValueError("A_val / P_val do not match the patterns and the block size")
        if C_val is None:
            C_val = torch.empty(self.nnz_C * b2, dtype=torch.float64, device=A_val.device)
        elif C_val.numel() != self.nnz_C * b2:
            raise ValueError("C_val does not match the pattern of C and the block size")
        _check(ptap_numeric(self.handle, A_val, P_val, C_val, stream), "ptap_numeric")
        return C_val

    def backward(self, A_val, P_val, dC_val, need_dA=True, need_dP=True, stream=None):
        dA = torch.empty(self.A_nnz, dtype=torch.float64, device=A_val.device) if need_dA else None
        dP = torch.empty(self.P_nnz, dtype=torch.float64, device=A_val.device) if need_dP else None
        _check(ptap_backward(self.handle, A_val, P_val, dC_val, dA, dP, stream), "ptap_backward")
        return dA, dP

    def stats(self) -> dict:
        st, s = ptap_plan_stats(self.handle)
        _check(st, "ptap_plan_stats")
        return s.as_dict()

    def close(self):
        if self.handle is not None:
            torch.cuda.synchronize()
            ptap_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Batched numeric products over several plans (Plan objects) in one HIP graph.

    levels[k] orders the work: all products of a level run together in one persistent launch,
    after every product of a smaller level (a coarse level's A is the previous level's C).  The
    value tensors passed to the first numeric() call are recorded into the graph: later calls
    must pass the same tensors (their contents may change)."""

    def __init__(self, plans, levels=None, allocator=None, stream=None):
        self.plans = list(plans)
        self.allocator = allocator if allocator is not None else TorchAllocator(stream=stream)
        st, h = ptap_batch_create([p.handle for p in self.plans], levels, self.allocator.struct, stream)
        _check(st, "ptap_batch_create")
        self.handle = h
        self._keep = None

    def numeric(self, A_vals, P_vals, C_vals, stream=None):
        self._keep = (list(A_vals), list(P_vals), list(C_vals))
        _check(ptap_batch_numeric(self.handle, A_vals, P_vals, C_vals, stream), "ptap_batch_numeric")
        return C_vals

    def close(self):
        if self.handle is not None:
            torch.cuda.synchronize()
            ptap_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Option sets tried by tune(): workgroup size and tile budget of the owner fold (the LDS "bins"
# the tiles are sized for), the atomic fold, and the numeric cache.
# Option sets tune() tries: workgroup size (wavefronts), tile budget (LDS bytes and entries), the
# short-row kernel's hash multiplier (the golden ratio forced; by default symbolic may pick another),
# the largest on-chip table of the general kernels, the numeric cache and the fold.  The short-row
# kernel's own table (64 slots, a fine row per 32 lanes) is fixed by its design.
GOLDEN_HASH_MUL = 0x9E3779B1
TUNE_CANDIDATES = (
    {},
    {"owner_waves": 8},
    {"tile_lds": 98304},
    {"tile_lds": 65536},
    {"owner_waves": 4},
    {"tile_entries": 2048},
    {"hash_mul": GOLDEN_HASH_MUL},
    {"hash_slots": 256},
    {"cache": True},
    {"fold": "atomic"},
)


def tune(n, m, A_rowptr, A_col, P_rowptr, P_col, A_val, P_val, *, candidates=TUNE_CANDIDATES,
         reps=3, base=None, stream=None):
    """Choose plan options by measurement: build a plan per candidate option set (merged with
    the given base options), time `reps` numeric products of each on the given values with HIP
    events, and return (best plan, report).  The other plans are destroyed.  The results of all
    candidates are the same product (the options change only how it is computed)."""
    base = dict(base or {})
    report = []
    best = None
    strm = stream if stream is not None else torch.cuda.current_stream()
    for cand in candidates:
        opts = {**base, **cand}
        plan = Plan(n, m, A_rowptr, A_col, P_rowptr, P_col, stream=stream, **opts)
        C = plan.numeric(A_val, P_val, stream=stream)
        plan.numeric(A_val, P_val, C, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(strm)
        for _ in range(reps):
            plan.numeric(A_val, P_val, C, stream=stream)
        e1.record(strm)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        report.append({"options": opts, "numeric_ms": round(ms, 4)})
        if best is None or ms < best[0]:
            if best is not None:
                best[1].close()
            best = (ms, plan, opts)
        else:
            plan.close()
        del C
    best[1].tuned_options = best[2]
    return best[1], report


class PtAPFunction(torch.autograd.Function):
    """C_val = PtAP(A_val, P_val) on a plan's fixed patterns; backward through ptap_backward
    (dA = P dC P^T on A's pattern, dP = A P dC^T + A^T P dC on P's pattern)."""

    @staticmethod
    def forward(ctx, A_val, P_val, plan):
        ctx.plan = plan
        ctx.save_for_backward(A_val, P_val)
        return plan.numeric(A_val.detach(), P_val.detach())

    @staticmethod
    def backward(ctx, dC):
        A_val, P_val = ctx.saved_tensors
        dA, dP = ctx.plan.backward(A_val.detach(), P_val.detach(), dC.contiguous(),
                                   need_dA=ctx.needs_input_grad[0], need_dP=ctx.needs_input_grad[1])
        return dA, dP, None


def ptap(plan, A_val, P_val):
    """Differentiable C values on plan's pattern."""
    return PtAPFunction.apply(A_val, P_val, plan)
