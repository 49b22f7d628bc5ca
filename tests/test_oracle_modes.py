"""Pins for the oracle's two extra modes: rows split over threads, and long-double accumulation.

* Threads: every row of C is computed on its own, so any split of the rows over threads must
  give the single-thread result bit for bit (pattern, values and magnitude bounds), including
  selected-row runs, more threads than rows, and inputs with empty rows and zero columns.
* Long double: on dyadic inputs (constant-coefficient stencils with trilinear interpolation)
  every FP64 term and partial sum is exact, so the long-double result must equal the FP64 one
  bit for bit.  On integer inputs whose terms need up to 57 bits, the exact sum of each entry
  (Python integers) fits the 64-bit significand of the x86 extended format, so the long-double
  result must be the exact sum correctly rounded to double, while FP64 accumulation is not.
"""
import numpy as np
import pytest

import oracle
import ptap_inputs as gen
from helpers import close_mask


def _same(a, b):
    assert np.array_equal(a.rowptr, b.rowptr)
    assert np.array_equal(a.col, b.col)
    if a.val is not None:
        assert np.array_equal(a.val.view(np.int64), b.val.view(np.int64))
        assert np.array_equal(a.abs.view(np.int64), b.abs.view(np.int64))


CASES = {
    "stencil27_lognormal_24": lambda: (gen.stencil27(24, seed=1), gen.trilinear(24)),
    "sa_two_steps_12": lambda: (lambda A: (A, gen.smoothed_aggregation(A, 12, 12, 12, steps=2)))(
        gen.stencil27(12, seed=2, eps_z=0.01)),
    "random_empty_rows_zero_cols": lambda: (gen.random_csr(300, 300, 0.03, seed=11, empty_rows=0.2),
                                            gen.random_csr(300, 40, 0.08, seed=12, empty_rows=0.2,
                                                           zero_cols=5, explicit_zeros=0.1)),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("threads", [2, 3, 7, 16])
def test_threads_bit_identical(name, threads):
    A, P = CASES[name]()
    _same(oracle.ptap(A, P), oracle.ptap(A, P, threads=threads))


def test_threads_more_than_rows_and_selected_rows():
    A, P = gen.stencil27(10, seed=3), gen.trilinear(10)
    one = oracle.ptap(A, P)
    _same(one, oracle.ptap(A, P, threads=10_000))
    rows = np.random.default_rng(4).permutation(P.n_cols)[:37].astype(np.int32)
    sel1 = oracle.ptap(A, P, rows=rows)
    sel8 = oracle.ptap(A, P, rows=rows, threads=8)
    _same(sel1, sel8)
    # the selected rows are the full result's rows, in the listed order
    for k, i in enumerate(rows):
        a, b = one.rowptr[i], one.rowptr[i + 1]
        c, d = sel8.rowptr[k], sel8.rowptr[k + 1]
        assert np.array_equal(one.col[a:b], sel8.col[c:d])
        assert np.array_equal(one.val[a:b], sel8.val[c:d])


def test_threads_pattern_only_and_long_double():
    A, P = CASES["sa_two_steps_12"]()
    _same(oracle.ptap(A, P, pattern_only=True), oracle.ptap(A, P, pattern_only=True, threads=5))
    _same(oracle.ptap(A, P, long_double=True), oracle.ptap(A, P, long_double=True, threads=5))


@pytest.mark.parametrize("case", ["c1", "stencil27_const_17", "laplacian7_17"])
def test_long_double_equals_fp64_on_dyadic_inputs(case):
    if case == "c1":
        A, P, _ = gen.galerkin_workload("c1")
    elif case == "stencil27_const_17":
        A, P = gen.stencil27(17), gen.trilinear(17)
    else:
        A, P = gen.laplacian7(17), gen.trilinear(17)
    _same(oracle.ptap(A, P), oracle.ptap(A, P, long_double=True))


def _integer_case(seed):
    rng = np.random.default_rng(seed)
    A = gen.random_csr(60, 60, 0.08, seed=seed, empty_rows=0.05)
    P = gen.random_csr(60, 12, 0.15, seed=seed + 1, empty_rows=0.05)
    lim = 2 ** 19
    A = A.with_values(rng.integers(-lim, lim + 1, A.nnz).astype(np.float64))
    P = P.with_values(rng.integers(-lim, lim + 1, P.nnz).astype(np.float64))
    return A, P


def _exact_ptap(A, P):
    """Dense exact C = P^T A P in Python integers (every entry an integer)."""
    Ad = [[0] * A.n_cols for _ in range(A.n_rows)]
    for r in range(A.n_rows):
        for k in range(A.rowptr[r], A.rowptr[r + 1]):
            Ad[r][int(A.col[k])] = int(A.val[k])
    Pd = [[0] * P.n_cols for _ in range(P.n_rows)]
    for r in range(P.n_rows):
        for k in range(P.rowptr[r], P.rowptr[r + 1]):
            Pd[r][int(P.col[k])] = int(P.val[k])
    n, m = A.n_rows, P.n_cols
    AP = [[sum(Ad[I][J] * Pd[J][j] for J in range(n) if Ad[I][J]) for j in range(m)] for I in range(n)]
    return [[sum(Pd[I][i] * AP[I][j] for I in range(n) if Pd[I][i]) for j in range(m)] for i in range(m)]


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_long_double_is_exact_sum_correctly_rounded(seed):
    A, P = _integer_case(seed)
    exact = _exact_ptap(A, P)
    ld = oracle.ptap(A, P, long_double=True)
    fp = oracle.ptap(A, P)
    assert np.array_equal(ld.col, fp.col)
    # every magnitude sum stays below 2^64, so the extended-precision sums are exact
    assert ld.abs.max() < 2.0 ** 63
    want = np.array([float(exact[i][int(j)]) for i in range(P.n_cols)
                     for j in ld.col[ld.rowptr[i]:ld.rowptr[i + 1]]])
    assert np.array_equal(ld.val, want), "long double result is not the correctly rounded exact sum"
    # FP64 accumulation rounds products of up to 57 bits: it must differ somewhere (else the
    # test above could not tell the modes apart), and stay within the forward-error bound
    assert (fp.val != want).any()
    assert close_mask(fp.val, want, ld.abs).all()
