"""GPU parity at the full sizes of the paper-shaped workloads.

The 128^3 27-point -> 64^3 trilinear product runs in the launch configuration the benchmark times
(merged all-at-once, K = 1, owner fold, default tiles and workgroup size) and in every other
algorithm; the whole C is compared with the oracle: the pattern bit for bit, the values under the
FP64 criterion of tests/helpers.py.  With constant coefficients (diagonal 26, off-diagonal -1) every
product and partial sum is a dyadic rational well inside FP64's range, so there the values must be
bit-exact at full size too.  The 96^3 smoothed-aggregation cases (one and two Jacobi steps) are
compared in full; the 4x4-block case (3.5 M rows, 374 M entries of A) on 2000 sampled rows of C,
which the oracle computes one by one."""
import numpy as np
import pytest
import torch

import oracle
import ptap_inputs as gen
from helpers import assert_close

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


import paper_1905_08423_amd as lib  # noqa: E402
from gpu_util import GpuProblem  # noqa: E402


def _gpu_c(g, **kw):
    plan = g.plan(**kw)
    C = plan.numeric(g.A_val, g.P_val)
    rp, col = plan.pattern()
    torch.cuda.synchronize()
    out = rp.cpu().numpy(), col.cpu().numpy(), C.cpu().numpy(), plan.stats()
    plan.close()
    return out


def _check_full(g, ref, exact=False, **kw):
    rp, col, val, st = _gpu_c(g, **kw)
    assert np.array_equal(rp, ref.rowptr), "C row pointers differ from the oracle"
    assert np.array_equal(col, ref.col), "C column indices differ from the oracle"
    if exact:
        bad = int((val != ref.val).sum())
        assert bad == 0, f"{bad} values not bit-exact, max diff {np.abs(val - ref.val).max()}"
    else:
        assert_close(val, ref.val, ref.abs)
    return st


@pytest.fixture(scope="module")
def c2():
    A, P, _ = gen.galerkin_workload("c2")
    ref = oracle.ptap(A, P)
    yield GpuProblem(A, P), ref


def test_c2_full_benchmark_configuration(c2):
    g, ref = c2
    st = _check_full(g, ref)
    assert st["nnz_C"] == 6_859_000
    assert st["fold_used"] == lib.PTAP_FOLD_OWNER and st["rows_needed"] == g.A.n_rows


@pytest.mark.parametrize("kw", [dict(algo="allatonce", fold="owner", nblocks=8),
                                dict(algo="merged", fold="owner", nblocks=8),
                                dict(algo="merged", fold="atomic"),
                                dict(algo="allatonce", fold="atomic", nblocks=8),
                                dict(algo="twostep"),
                                dict(algo="merged", fold="owner", cache=True)],
                         ids=["allatonce_K8_owner", "merged_K8_owner", "merged_atomic",
                              "allatonce_K8_atomic", "twostep", "merged_owner_cached"])
def test_c2_full_other_algorithms(c2, kw):
    g, ref = c2
    _check_full(g, ref, **kw)


def test_c2_full_constant_coefficients_bit_exact():
    A, P = gen.stencil27(128), gen.trilinear(128)
    ref = oracle.ptap(A, P)
    g = GpuProblem(A, P)
    _check_full(g, ref, exact=True)
    _check_full(g, ref, exact=True, algo="allatonce", fold="owner", nblocks=8)


@pytest.mark.parametrize("side,ranges", [(93, 3), (121, 6)])
def test_owner_tiles_over_uneven_row_ranges(side, ranges):
    """Coarse grids of 47^3 = 103,823 and 61^3 = 226,981 rows: the owner tiles are grown on 3 and
    6 contiguous row ranges (one per 32,768 rows, at most 8) whose sizes differ by one row.  A row
    left out of every tile, or held by two, would show as a wrong entry of C."""
    A, P = gen.stencil27(side, seed=5), gen.trilinear(side)
    m = P.n_cols
    assert min(8, m // 32768) == ranges and m % ranges != 0
    ref = oracle.ptap(A, P)
    g = GpuProblem(A, P)
    st = _check_full(g, ref)
    assert st["n_tiles"] > ranges
    _check_full(g, ref, algo="allatonce", fold="owner", nblocks=8)


def test_rows_beyond_one_thread_per_row_grid_cap():
    """17,000,000 fine and coarse rows: a 1D three-point operator and one smoothed-aggregation
    step over single-node aggregates, so P is tridiagonal and n x n.  The symbolic kernels that
    give one thread to each row (pattern validation, P's column lists, the row work w_I, the
    bounds of C's rows) have to reach rows past 65,536 blocks of 256 threads (16,777,216 rows),
    in A, in P and in C."""
    n = 17_000_000
    A = gen.laplacian7(n, 1, 1)
    P = gen.smoothed_aggregation(A, n, 1, 1, agg=1, steps=1)
    assert A.n_rows > 65536 * 256 and P.n_cols > 65536 * 256
    ref = oracle.ptap(A, P)
    g = GpuProblem(A, P)
    st = _check_full(g, ref)
    assert st["nnz_C"] == len(ref.col)


def test_values_of_A_past_2GiB():
    """216^3 27-point lognormal operator, 269,586,136 entries: A's values take 2.16 GB, beyond the
    2 GiB a 32-bit buffer offset reaches, so the short-row owner kernel reads them by 64-bit
    address.  The whole C against the oracle, for the default form and with the numeric cache."""
    side = 216
    A, P = gen.stencil27(side, seed=6), gen.trilinear(side)
    assert A.nnz * 8 >= 2**31 and A.nnz * 4 < 2**31
    ref = oracle.ptap(A, P)
    g = GpuProblem(A, P)
    _check_full(g, ref)
    _check_full(g, ref, algo="merged", fold="owner", cache=True)


@pytest.mark.parametrize("name", ["c3a", "c3b"])
def test_c3_full_smoothed_aggregation(name):
    """Merged (owner fold), two-step (its short-row kernel walks the rows of P^T, up to 125
    entries, 32 at a time) and the atomic fold, each against the same oracle C."""
    A, P, _ = gen.galerkin_workload(name)
    ref = oracle.ptap(A, P)
    g = GpuProblem(A, P)
    _check_full(g, ref)
    _check_full(g, ref, algo="twostep")
    _check_full(g, ref, algo="merged", fold="atomic")


def test_c3c_block_sampled_rows():
    A, P, _ = gen.galerkin_workload("c3c")
    rows = np.sort(np.random.default_rng(7).choice(P.n_cols, 2000, replace=False)).astype(np.int32)
    ref = oracle.ptap(A, P, rows=rows)
    rp, col, val, st = _gpu_c(GpuProblem(A, P))
    assert st["nnz_C"] == 13_289_344
    lo, hi = rp[rows], rp[rows + 1]
    assert np.array_equal(hi - lo, np.diff(ref.rowptr)), "row lengths differ from the oracle"
    take = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)])
    assert np.array_equal(col[take], ref.col), "C column indices differ from the oracle"
    assert_close(val[take], ref.val, ref.abs)
