"""The C ABI library: every symbol declared in include/ptap.h is exported (CPU, no compute
calls), plus error handling on the GPU (malformed CSR, call order, allocator failure)."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1905_08423_amd as lib
import ptap_inputs as gen


def test_header_symbols_exported():
    so = ctypes.CDLL(lib.LIB_PATH)
    names = lib.header_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(so, name), name
    assert set(names) <= set(lib._SIGNATURES), "binding lacks a declared function"


def test_status_strings_and_defaults():
    assert lib.ptap_status_string(0) == "ok"
    for s in range(1, 7):
        assert lib.ptap_status_string(s)
    o = lib.ptap_options_default()
    assert (o.algo, o.fold, o.nblocks, o.validate) == (lib.PTAP_MERGED, lib.PTAP_FOLD_AUTO, 1, 1)
    assert ctypes.sizeof(lib.ptap_options) == 16 * 4


def test_null_arguments_rejected_without_gpu():
    # argument checks happen before any device call
    st, h = lib.ptap_plan_create(-1, 2, None, None, 0, None, None, 0)
    assert st == lib.PTAP_ERR_INPUT and not h.value
    assert lib.load_library().ptap_symbolic(None, None) == lib.PTAP_ERR_INPUT
    assert lib.load_library().ptap_numeric(None, None, None, None, None) == lib.PTAP_ERR_INPUT
    lib.ptap_plan_destroy(None)  # accepts NULL


def test_counts_beyond_int32_rejected_without_gpu():
    """nnz(A) or nnz(P) past int32 indexing is PTAP_ERR_TOO_LARGE, reported before any device
    call (the pointers are never read)."""
    fake = ctypes.c_void_p(0x1000)
    L = lib.load_library()
    for a_nnz, p_nnz in [(2**31, 10), (10, 2**31), (2**40, 2**40)]:
        h = ctypes.c_void_p()
        st = L.ptap_plan_create(ctypes.byref(h), 10, 4, fake, fake, a_nnz, fake, fake, p_nnz, None, None, None)
        assert st == lib.PTAP_ERR_TOO_LARGE and not h.value, (a_nnz, p_nnz, st)
        h = ctypes.c_void_p()
        st = L.ptap_plan_create_bsr(ctypes.byref(h), 10, 4, 3, fake, fake, a_nnz, fake, fake, p_nnz,
                                    None, None, None)
        assert st == lib.PTAP_ERR_TOO_LARGE and not h.value, (a_nnz, p_nnz, st)
    assert L.ptap_copy_pattern(None, None, None, None) == lib.PTAP_ERR_INPUT


def test_bad_options_rejected_without_gpu():
    """Option values out of range are PTAP_ERR_INPUT before any device call: an even hash
    multiplier, an unknown owner kernel, a workgroup size other than 4, 8 or 16, a validation
    level other than 0, 1 or 2."""
    fake = ctypes.c_void_p(0x1000)
    L = lib.load_library()
    for field, value in [("hash_mul", 2), ("hash_mul", 0x9E3779B0), ("owner_kernel", 2), ("owner_waves", 12),
                         ("validate", 3), ("validate", -1)]:
        o = lib.ptap_options_default()
        setattr(o, field, value)
        h = ctypes.c_void_p()
        st = L.ptap_plan_create(ctypes.byref(h), 10, 4, fake, fake, 10, fake, fake, 10, ctypes.byref(o), None, None)
        assert st == lib.PTAP_ERR_INPUT and not h.value, (field, value, st)


gpu = pytest.mark.gpu


def _dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).cuda()


def _patterns(A, P):
    """Device copies of the patterns.  The caller must keep the returned tuple alive for the
    life of any plan created on it (the plan keeps raw pointers to these arrays)."""
    return (_dev(A.rowptr, torch.int32), _dev(A.col, torch.int32), _dev(P.rowptr, torch.int32),
            _dev(P.col, torch.int32))


def _create(A, P, keep, opts=None, alloc=None):
    Arp, Ac, Prp, Pc = keep
    return lib.ptap_plan_create(A.n_rows, P.n_cols, Arp, Ac, A.nnz, Prp, Pc, P.nnz, opts, alloc)


@gpu
@pytest.mark.parametrize("defect", ["unsorted", "duplicate", "out_of_range", "rowptr", "nnz"])
def test_malformed_csr_rejected(defect):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A, P = gen.laplacian7(4), gen.trilinear(4)
    col = A.col.copy()
    rp = A.rowptr.copy()
    nnz = A.nnz
    if defect == "unsorted":
        col[1], col[2] = col[2], col[1]
    elif defect == "duplicate":
        col[2] = col[1]
    elif defect == "out_of_range":
        col[5] = A.n_rows + 3
    elif defect == "rowptr":
        rp[3] = rp[4] + 1
    elif defect == "nnz":
        nnz = nnz - 1
    st, h = lib.ptap_plan_create(A.n_rows, P.n_cols, _dev(rp, torch.int32), _dev(col, torch.int32), nnz,
                                 _dev(P.rowptr, torch.int32), _dev(P.col, torch.int32), P.nnz)
    assert st == lib.PTAP_ERR_INPUT and not h.value


@gpu
def test_call_order_and_destroy():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A, P = gen.laplacian7(4), gen.trilinear(4)
    keep = _patterns(A, P)
    st, h = _create(A, P, keep)
    assert st == lib.PTAP_OK
    C = torch.empty(10, dtype=torch.float64, device="cuda")
    Av, Pv = _dev(A.val, torch.float64), _dev(P.val, torch.float64)
    assert lib.ptap_numeric(h, Av, Pv, C) == lib.PTAP_ERR_STATE
    assert lib.ptap_get_pattern(h)[0] == lib.PTAP_ERR_STATE
    assert lib.ptap_symbolic(h) == lib.PTAP_OK
    assert lib.ptap_symbolic(h) == lib.PTAP_ERR_STATE
    # backward was not requested at symbolic time
    assert lib.ptap_backward(h, Av, Pv, C, None, None) == lib.PTAP_ERR_STATE
    lib.ptap_plan_destroy(h)
    del keep


@gpu
def test_allocator_failure_reports_oom():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A, P = gen.stencil27(8), gen.trilinear(8)
    budget = {"left": 1 << 12}
    live = {}
    alloc_t = lib.ptap_allocator._fields_[0][1]
    release_t = lib.ptap_allocator._fields_[1][1]

    def _alloc(nbytes, ctx):
        if nbytes > budget["left"]:
            return None
        budget["left"] -= nbytes
        t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        live[t.data_ptr()] = t
        return t.data_ptr()

    def _release(ptr, nbytes, ctx):
        budget["left"] += nbytes
        live.pop(ptr, None)

    ca, cr = alloc_t(_alloc), release_t(_release)
    al = lib.ptap_allocator(ca, cr, None)
    keep = _patterns(A, P)
    st, h = _create(A, P, keep, None, al)
    assert st == lib.PTAP_OK
    assert lib.ptap_symbolic(h) == lib.PTAP_ERR_OOM
    assert not live, "failed symbolic leaked device memory"
    lib.ptap_plan_destroy(h)
    torch.cuda.synchronize()
    del keep


def test_stream_sum_arguments_rejected_without_gpu():
    f = lib.load_library().ptap_stream_sum
    assert f(None, 4, None, None) == lib.PTAP_ERR_INPUT
    assert f(None, -1, None, None) == lib.PTAP_ERR_INPUT


@gpu
@pytest.mark.parametrize("n", [0, 1, 7, 1 << 20, (1 << 22) + 3])
def test_stream_sum_matches_the_sum(n):
    """The bandwidth probe reads every value once: its sum equals numpy's within the rounding of
    two summation orders (|error| <= n * eps * sum |x|)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    x = np.random.default_rng(n).uniform(-1.0, 1.0, n)
    got = float(lib.stream_sum(torch.as_tensor(x).cuda()).item())
    bound = max(n, 1) * 2.3e-16 * float(np.abs(x).sum())
    assert abs(got - float(x.sum())) <= bound
    odd = torch.as_tensor(np.zeros(3)).cuda()[1:]  # 8-byte aligned view
    assert lib.load_library().ptap_stream_sum(lib._ptr(odd), 2, lib._ptr(odd), None) == lib.PTAP_ERR_INPUT
