"""ptap_numeric_noalloc (the numeric phase without device allocation, its device-memory hash
tables in the library's fixed per-GPU array) against ptap_numeric on the same plans, through the
C ABI: two calls in a row, the second on a smaller problem, for plans whose general kernels keep
hash tables in device memory (a 4x4-block operator, tables capped at 64 slots in LDS), for the
owner fold, the atomic
fold and two-step, and once for a plan that needs no device-memory table."""
import numpy as np
import pytest
import torch

import oracle
import ptap_inputs as gen
from helpers import assert_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


import paper_1905_08423_amd as lib  # noqa: E402
from gpu_util import GpuProblem  # noqa: E402


def _block(s):
    """4x4-block 27-point operator (scalar form) with block smoothed aggregation: rows of AP hold
    up to 108 keys, more than a 64-slot LDS table takes."""
    A = gen.block_stencil27(s, 4, seed=2)
    return A, gen.block_smoothed_aggregation(A, s, 4)


def _both(A, P, **kw):
    g = GpuProblem(A, P)
    plan = g.plan(**kw)
    st = plan.stats()
    ref = plan.numeric(g.A_val, g.P_val).clone()
    C = torch.full((plan.nnz_C,), float("nan"), dtype=torch.float64, device="cuda")
    rc = lib.ptap_numeric_noalloc(plan.handle, g.A_val, g.P_val, C)
    torch.cuda.synchronize()
    assert rc == lib.PTAP_OK, lib.ptap_status_string(rc)
    out = (C.cpu().numpy(), ref.cpu().numpy(), st)
    plan.close()
    return out


@pytest.mark.parametrize("kw", [dict(algo="merged", fold="owner"), dict(algo="merged", fold="atomic"),
                                dict(algo="twostep")], ids=["owner", "atomic", "twostep"])
def test_noalloc_matches_numeric_two_calls(kw):
    # the second call on a smaller problem (300 rows against 1372), also with rows of AP of up to
    # 87 keys, empty rows and zero columns
    cases = [("block_7", _block(7)),
             ("random_300", (gen.random_csr(300, 300, 0.06, seed=31, empty_rows=0.05),
                             gen.random_csr(300, 90, 0.1, seed=32, empty_rows=0.05, zero_cols=3)))]
    for name, (A, P) in cases:
        got, ref, st = _both(A, P, hash_slots=64, **kw)
        assert st["table_slots"] > 0, (name, st)  # the plan does keep tables in device memory
        o = oracle.ptap(A, P)
        assert_close(got, o.val, o.abs, f"noalloc {name}")
        assert_close(got, ref, o.abs, f"noalloc vs numeric {name}")


def test_noalloc_without_device_tables_bit_exact():
    A, P, _ = gen.galerkin_workload("c1")
    got, ref, st = _both(A, P, algo="merged", fold="owner")
    assert st["table_slots"] == 0
    assert np.array_equal(got, ref) and np.array_equal(got, oracle.ptap(A, P).val)
