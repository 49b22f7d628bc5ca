"""Pins for the CPU oracle: facts fixed by the paper and by mathematics, none of which is the
oracle's own formula retyped.

* the worked row-wise example printed in Section 2 (Eq. rowwise), from a golden fixture;
* dense products and brute-force boolean products on tiny inputs (non-symmetric A, empty
  rows, zero columns, explicit zeros);
* Kronecker closed forms for constant-coefficient 7- and 27-point operators with trilinear
  interpolation, bit for bit (all terms are dyadic rationals);
* the hand-derived interior coarse stencil of the 7-point operator;
* the boolean pattern product on all-ones data at larger sizes and the closed-form nnz;
* symmetry of C for symmetric A, probe identities C x = P^T (A (P x));
* finite differences and the dense matrix-calculus gradient for the adjoint.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import ptap_inputs as gen
from helpers import (assert_close, dense, dense_pattern, ones_like_csr, read_golden_sections,
                     rows_of, scipy_csr)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def identity_csr(n):
    return gen.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))


# ------------------------------------------------------------------------------------------
# The worked example of Section 2
# ------------------------------------------------------------------------------------------

def test_toy_rowwise_pattern():
    g = read_golden_sections(os.path.join(GOLDEN, "toy_rowwise.txt"))
    A, P = gen.toy_rowwise(seed=3)
    assert rows_of(A.rowptr, A.col) == g["A"]
    assert rows_of(P.rowptr, P.col) == g["P"]
    # AP through the oracle's general product Q1^T A Q2 with Q1 = I.
    AP = oracle.rap(identity_csr(6), A, P)
    assert rows_of(AP.rowptr, AP.col) == g["AP"]
    # Row 0 of AP combines the rows of P named by row 0 of A.
    assert A.col[A.rowptr[0]:A.rowptr[1]].tolist() == g["row0_uses_P_rows"][0]
    # Remote rows needed by the first process (rows 0-1) under the 3-way split.
    own = set(range(0, 2))
    remote = sorted({int(c) for r in (0, 1) for c in A.col[A.rowptr[r]:A.rowptr[r + 1]] if c not in own})
    assert remote == g["process0_remote_P_rows"][0]
    # P^T A P pattern against a brute-force boolean product.
    C = oracle.ptap(A, P)
    Bp, Ba = dense_pattern(P).astype(int), dense_pattern(A).astype(int)
    brute = (Bp.T @ Ba @ Bp) > 0
    got = np.zeros_like(brute)
    for i, row in enumerate(rows_of(C.rowptr, C.col)):
        got[i, row] = True
    assert np.array_equal(got, brute)
    # values against the dense product
    D = dense(P).T @ dense(A) @ dense(P)
    assert_close(C.val, D[got], (np.abs(dense(P)).T @ np.abs(dense(A)) @ np.abs(dense(P)))[got])


# ------------------------------------------------------------------------------------------
# Dense and brute force on tiny random inputs
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(8))
def test_dense_random(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 40))
    m = int(rng.integers(1, 16))
    A = gen.random_csr(n, n, float(rng.uniform(0.05, 0.4)), seed=seed, empty_rows=0.15,
                       explicit_zeros=0.1)
    P = gen.random_csr(n, m, float(rng.uniform(0.05, 0.5)), seed=1000 + seed, empty_rows=0.2,
                       zero_cols=1 if m > 2 else 0, explicit_zeros=0.1)
    C = oracle.ptap(A, P)
    Ad, Pd = dense(A), dense(P)
    brute = (dense_pattern(P).astype(int).T @ dense_pattern(A).astype(int) @ dense_pattern(P).astype(int)) > 0
    got = np.zeros((m, m), dtype=bool)
    for i, row in enumerate(rows_of(C.rowptr, C.col)):
        assert row == sorted(set(row))
        got[i, row] = True
    assert np.array_equal(got, brute)
    ref = (Pd.T @ Ad @ Pd)[got]
    absref = (np.abs(Pd).T @ np.abs(Ad) @ np.abs(Pd))[got]
    assert_close(C.val, ref, absref)
    np.testing.assert_allclose(C.abs, absref, rtol=1e-13, atol=0)
    # the pattern-only mode returns the same pattern
    Cp = oracle.ptap(A, P, pattern_only=True)
    assert np.array_equal(Cp.rowptr, C.rowptr) and np.array_equal(Cp.col, C.col) and Cp.val is None


@pytest.mark.parametrize("seed", range(4))
def test_general_rap_dense(seed):
    """Q1^T A Q2 with two different interpolations (used by the adjoint identities)."""
    rng = np.random.default_rng(7 + seed)
    n, m1, m2 = 25, 7, 9
    A = gen.random_csr(n, n, 0.2, seed=seed)
    Q1 = gen.random_csr(n, m1, 0.3, seed=50 + seed, empty_rows=0.1)
    Q2 = gen.random_csr(n, m2, 0.3, seed=90 + seed, empty_rows=0.1)
    R = oracle.rap(Q1, A, Q2)
    D = dense(Q1).T @ dense(A) @ dense(Q2)
    mask = (dense_pattern(Q1).astype(int).T @ dense_pattern(A).astype(int) @ dense_pattern(Q2).astype(int)) > 0
    got = np.zeros((m1, m2), dtype=bool)
    for i, row in enumerate(rows_of(R.rowptr, R.col)):
        got[i, row] = True
    assert np.array_equal(got, mask)
    assert_close(R.val, D[mask], (np.abs(dense(Q1)).T @ np.abs(dense(A)) @ np.abs(dense(Q2)))[mask])
    del rng


# ------------------------------------------------------------------------------------------
# Kronecker closed forms (bit-exact)
# ------------------------------------------------------------------------------------------

def _tridiag(k, lo, d, hi):
    return np.diag(np.full(k, d)) + np.diag(np.full(k - 1, lo), -1) + np.diag(np.full(k - 1, hi), 1)


def _csr_to_dense_on_pattern(C, m):
    D = np.zeros((m, m))
    mask = np.zeros((m, m), dtype=bool)
    for i in range(m):
        cols = C.col[C.rowptr[i]:C.rowptr[i + 1]]
        D[i, cols] = C.val[C.rowptr[i]:C.rowptr[i + 1]]
        mask[i, cols] = True
    return D, mask


@pytest.mark.parametrize("side", [5, 9, 16, 17])
def test_kronecker_7pt(side):
    """A = L(x)I(x)I + I(x)L(x)I + I(x)I(x)L with L = tridiag(-1, 2, -1) is the 7-point
    6/-1 Dirichlet operator; with P = p(x)p(x)p,  C = T(x)M(x)M + M(x)T(x)M + M(x)M(x)T where
    T = p^T L p and M = p^T p."""
    A, P = gen.laplacian7(side), gen.trilinear(side)
    p = gen.trilinear_1d(side).toarray()
    L = _tridiag(side, -1.0, 2.0, -1.0)
    T, M = p.T @ L @ p, p.T @ p
    ref = np.kron(T, np.kron(M, M)) + np.kron(M, np.kron(T, M)) + np.kron(M, np.kron(M, T))
    C = oracle.ptap(A, P)
    m = P.n_cols
    D, mask = _csr_to_dense_on_pattern(C, m)
    assert not np.any(ref[~mask])          # every nonzero of the closed form is in the pattern
    assert np.array_equal(D[mask], ref[mask])  # bit for bit
    nc = gen.coarse_side(side)
    assert C.nnz == (3 * nc - 2) ** 3


@pytest.mark.parametrize("side", [5, 9, 16, 17])
def test_kronecker_27pt(side):
    """The 26/-1 27-point operator is 27 I - J(x)J(x)J with J = tridiag(1, 1, 1), so
    C = 27 M(x)M(x)M - Jh(x)Jh(x)Jh with M = p^T p and Jh = p^T J p."""
    A, P = gen.stencil27(side), gen.trilinear(side)
    p = gen.trilinear_1d(side).toarray()
    J = _tridiag(side, 1.0, 1.0, 1.0)
    M, Jh = p.T @ p, p.T @ J @ p
    ref = 27.0 * np.kron(M, np.kron(M, M)) - np.kron(Jh, np.kron(Jh, Jh))
    C = oracle.ptap(A, P)
    m = P.n_cols
    D, mask = _csr_to_dense_on_pattern(C, m)
    assert not np.any(ref[~mask])
    assert np.array_equal(D[mask], ref[mask])
    nc = gen.coarse_side(side)
    assert C.nnz == (3 * nc - 2) ** 3


def test_interior_stencil_7pt():
    """Interior coarse stencil of the 7-point operator under trilinear interpolation, derived
    by hand from the 1D factors: M = p^T p has interior row (1/4, 3/2, 1/4) and T = p^T L p has
    interior row (-1/2, 1, -1/2).  Centre 3*T0*M0^2 = 27/4; face T1*M0^2 + 2*M1*T0*M0 = -3/8;
    edge 2*T1*M1*M0 + M1^2*T0 = -5/16; corner 3*T1*M1^2 = -3/32; the row sums to zero."""
    side = 17
    A, P = gen.laplacian7(side), gen.trilinear(side)
    nc = gen.coarse_side(side)
    c = (4, 4, 4)
    i = c[0] + nc * (c[1] + nc * c[2])
    C = oracle.ptap(A, P, rows=[i])
    cols, vals = C.col, C.val
    assert cols.size == 27
    want = {0: 27 / 4, 1: -3 / 8, 2: -5 / 16, 3: -3 / 32}
    for j, v in zip(cols, vals):
        d = (j % nc - c[0], (j // nc) % nc - c[1], j // (nc * nc) - c[2])
        assert max(abs(t) for t in d) == 1 or d == (0, 0, 0)
        assert v == want[sum(abs(t) for t in d)]
    assert vals.sum() == 0.0


# ------------------------------------------------------------------------------------------
# Structural pattern, symmetry, probes, library cross-check
# ------------------------------------------------------------------------------------------

def _pattern_by_ones(A, P):
    B = (ones_like_csr(P).T @ ones_like_csr(A) @ ones_like_csr(P)).tocsr()
    B.sort_indices()
    return B


@pytest.mark.parametrize("case", ["c2_20", "c3a_12", "c3b_12", "c3c_6", "lap7_odd_13"])
def test_pattern_is_boolean_product(case):
    A, P = _case(case)
    B = _pattern_by_ones(A, P)
    C = oracle.ptap(A, P)
    Cp = oracle.ptap(A, P, pattern_only=True)
    assert np.array_equal(C.rowptr, B.indptr) and np.array_equal(C.col, B.indices)
    assert np.array_equal(Cp.rowptr, B.indptr) and np.array_equal(Cp.col, B.indices)


def _case(case):
    kind, s = case.rsplit("_", 1)
    s = int(s)
    if kind == "c2":
        return gen.stencil27(s, seed=1), gen.trilinear(s)
    if kind in ("c3a", "c3b"):
        A = gen.stencil27(s, seed=2, eps_z=0.01)
        return A, gen.smoothed_aggregation(A, s, s, s, steps=1 if kind == "c3a" else 2)
    if kind == "c3c":
        A = gen.block_stencil27(s, 4, seed=2)
        return A, gen.block_smoothed_aggregation(A, s, 4)
    if kind == "lap7_odd":
        return gen.laplacian7(s), gen.trilinear(s)
    raise KeyError(case)


@pytest.mark.parametrize("case", ["c2_20", "c3a_12", "c3c_6"])
def test_symmetry(case):
    A, P = _case(case)
    As = scipy_csr(A)
    assert abs(As - As.T).max() == 0.0
    C = oracle.ptap(A, P)
    m = P.n_cols
    Cs = sp.csr_matrix((C.val, C.col, C.rowptr), shape=(m, m))
    Cabs = sp.csr_matrix((C.abs, C.col, C.rowptr), shape=(m, m))
    pat = sp.csr_matrix((np.ones(C.nnz), C.col, C.rowptr), shape=(m, m))
    assert (pat != pat.T).nnz == 0
    diff = abs(Cs - Cs.T)
    assert np.all(diff.toarray() <= 1e-14 * Cabs.toarray())


@pytest.mark.parametrize("case", ["c2_20", "c3a_12", "c3b_12", "c3c_6"])
def test_probe_identities(case):
    """C 1 = P^T (A (P 1)) and C x = P^T (A (P x)) for a random x, by sparse mat-vecs."""
    A, P = _case(case)
    C = oracle.ptap(A, P)
    m = P.n_cols
    Cs = sp.csr_matrix((C.val, C.col, C.rowptr), shape=(m, m))
    As, Ps = scipy_csr(A), scipy_csr(P)
    Aa, Pa = abs(As), abs(Ps)
    rng = np.random.default_rng(11)
    for x in (np.ones(m), rng.standard_normal(m)):
        lhs = Cs @ x
        rhs = Ps.T @ (As @ (Ps @ x))
        bound = Pa.T @ (Aa @ (Pa @ np.abs(x)))
        assert np.all(np.abs(lhs - rhs) <= 1e-13 * bound + 1e-300)


@pytest.mark.parametrize("case", ["c2_20", "c3a_12", "c3b_12"])
def test_scipy_values(case):
    A, P = _case(case)
    C = oracle.ptap(A, P)
    S = (scipy_csr(P).T @ scipy_csr(A) @ scipy_csr(P)).tocsr()
    S.sort_indices()
    m = P.n_cols
    Cs = sp.csr_matrix((C.val, C.col, C.rowptr), shape=(m, m))
    ref = np.asarray(S[Cs.nonzero()]).ravel() if Cs.nnz else np.zeros(0)
    got = np.asarray(Cs[Cs.nonzero()]).ravel()
    Cabs = sp.csr_matrix((C.abs, C.col, C.rowptr), shape=(m, m))
    assert_close(got, ref, np.asarray(Cabs[Cs.nonzero()]).ravel())


# ------------------------------------------------------------------------------------------
# Edge cases
# ------------------------------------------------------------------------------------------

def test_edge_single_row():
    A = gen.CSR(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([3.0]))
    P = gen.CSR(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.0]))
    C = oracle.ptap(A, P)
    assert C.rowptr.tolist() == [0, 1] and C.col.tolist() == [0] and C.val.tolist() == [12.0]


def test_edge_empty_matrices():
    A = gen.CSR(3, 3, np.zeros(4, np.int32), np.zeros(0, np.int32), np.zeros(0))
    P = gen.CSR(3, 2, np.array([0, 1, 2, 2], np.int32), np.array([0, 1], np.int32), np.ones(2))
    C = oracle.ptap(A, P)
    assert C.nnz == 0 and C.rowptr.tolist() == [0, 0, 0]


def test_edge_zero_column_and_explicit_zeros():
    # P's column 1 is never used: row and column 1 of C are empty.
    A = gen.CSR(3, 3, np.array([0, 2, 4, 5], np.int32), np.array([0, 2, 0, 1, 2], np.int32),
                np.array([1.0, 0.0, 2.0, -1.0, 4.0]))
    P = gen.CSR(3, 3, np.array([0, 1, 2, 3], np.int32), np.array([0, 2, 2], np.int32),
                np.array([1.0, 0.0, 1.0]))
    C = oracle.ptap(A, P)
    rows = rows_of(C.rowptr, C.col)
    assert rows[1] == [] and all(1 not in r for r in rows)
    # explicit zeros in A and P still create structure: (0,2) exists through A(0,2) = 0.
    assert 2 in rows[0]
    B = _pattern_by_ones(A, P)
    assert np.array_equal(C.rowptr, B.indptr) and np.array_equal(C.col, B.indices)


def test_selected_rows_match_full():
    A, P = _case("c3a_12")
    C = oracle.ptap(A, P)
    sel = np.array([5, 0, 17, P.n_cols - 1, 5])
    R = oracle.ptap(A, P, rows=sel)
    for r, i in enumerate(sel):
        a, b = C.rowptr[i], C.rowptr[i + 1]
        c, d = R.rowptr[r], R.rowptr[r + 1]
        assert np.array_equal(C.col[a:b], R.col[c:d])
        assert np.array_equal(C.val[a:b], R.val[c:d])


# ------------------------------------------------------------------------------------------
# Adjoint
# ------------------------------------------------------------------------------------------

def _loss(A, P, W):
    return float(np.dot(W, oracle.ptap(A, P).val))


@pytest.mark.parametrize("nonsym", [False, True])
def test_backward_dense_gradient(nonsym):
    """dL/dA = P W P^T and dL/dP = A P W^T + A^T P W (dense), masked to the patterns."""
    if nonsym:
        A = gen.random_csr(30, 30, 0.2, seed=5, empty_rows=0.1)
        P = gen.random_csr(30, 8, 0.3, seed=6, empty_rows=0.1, zero_cols=1)
    else:
        A, P = gen.stencil27(6, seed=4), gen.trilinear(6)
    C = oracle.ptap(A, P, pattern_only=True)
    W = gen.loss_weights(C.nnz, seed=5)
    dA, dP = oracle.ptap_backward(A, P, C.rowptr, C.col, W)
    Wd = np.zeros((P.n_cols, P.n_cols))
    for i in range(P.n_cols):
        Wd[i, C.col[C.rowptr[i]:C.rowptr[i + 1]]] = W[C.rowptr[i]:C.rowptr[i + 1]]
    Ad, Pd = dense(A), dense(P)
    gA = Pd @ Wd @ Pd.T
    gP = Ad @ Pd @ Wd.T + Ad.T @ Pd @ Wd
    mA, mP = dense_pattern(A), dense_pattern(P)
    Wa = np.abs(Wd)
    bA = np.abs(Pd) @ Wa @ np.abs(Pd).T
    bP = np.abs(Ad) @ np.abs(Pd) @ Wa.T + np.abs(Ad).T @ np.abs(Pd) @ Wa
    assert_close(dA, gA[mA], bA[mA], "dA")
    assert_close(dP, gP[mP], bP[mP], "dP")


def test_backward_finite_differences():
    """Central differences of L = sum W o C: L is linear in A and quadratic in P, so the
    central difference has no truncation error, only rounding."""
    A, P = gen.stencil27(6, seed=4), gen.trilinear(6)
    C = oracle.ptap(A, P, pattern_only=True)
    W = gen.loss_weights(C.nnz, seed=5)
    dA, dP = oracle.ptap_backward(A, P, C.rowptr, C.col, W)
    rng = np.random.default_rng(6)
    h = 1e-6
    for k in rng.choice(A.nnz, size=20, replace=False):
        vp, vm = A.val.copy(), A.val.copy()
        vp[k] += h; vm[k] -= h
        fd = (_loss(A.with_values(vp), P, W) - _loss(A.with_values(vm), P, W)) / (2 * h)
        assert abs(fd - dA[k]) <= 1e-6 * max(1.0, abs(dA[k]))
    for k in rng.choice(P.nnz, size=20, replace=False):
        vp, vm = P.val.copy(), P.val.copy()
        vp[k] += h; vm[k] -= h
        fd = (_loss(A, P.with_values(vp), W) - _loss(A, P.with_values(vm), W)) / (2 * h)
        assert abs(fd - dP[k]) <= 1e-6 * max(1.0, abs(dP[k]))
