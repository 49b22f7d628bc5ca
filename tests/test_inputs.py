"""Generator checks: well-formed CSR, closed-form sizes, the vertex-centred refinement rule
n_f = 2 n_c - 1 of the paper's model problem (Section 4.1), symmetry, seeded determinism."""
import numpy as np
import pytest
import scipy.sparse as sp

import ptap_inputs as gen


def _p1d_nnz(nf):
    nc = gen.coarse_side(nf)
    return nc + 2 * (nf // 2) - (1 if nf % 2 == 0 else 0)


@pytest.mark.parametrize("side", [2, 3, 8, 9, 16, 17])
def test_trilinear_shape_and_weights(side):
    P = gen.trilinear(side)
    P.check()
    nc = gen.coarse_side(side)
    assert P.n_rows == side ** 3 and P.n_cols == nc ** 3
    assert P.nnz == _p1d_nnz(side) ** 3
    assert set(np.unique(P.val).tolist()) <= {1.0, 0.5, 0.25, 0.125}
    if side % 2 == 1:
        # odd sides: every fine point is a convex combination (rows sum to one) and
        # the refinement is vertex centred, n_f = 2 n_c - 1.
        assert side == 2 * nc - 1
        sums = np.add.reduceat(P.val, P.rowptr[:-1])
        assert np.all(sums == 1.0)


def test_paper_model_problem_sizes():
    # Section 4.1: a 1000^3 coarse grid refined uniformly gives 1999^3 = 7,988,005,999 fine
    # unknowns; 1500^3 gives 2999^3 = 26,973,008,999.
    for nc, nf_total in ((1000, 7_988_005_999), (1500, 26_973_008_999)):
        nf = 2 * nc - 1
        assert gen.coarse_side(nf) == nc and nf ** 3 == nf_total


@pytest.mark.parametrize("side", [3, 7, 16])
def test_laplacian7(side):
    A = gen.laplacian7(side)
    A.check()
    assert A.nnz == 7 * side ** 3 - 6 * side ** 2
    S = sp.csr_matrix((A.val, A.col, A.rowptr))
    assert abs(S - S.T).max() == 0
    assert np.all(S.diagonal() == 6.0)


@pytest.mark.parametrize("side", [3, 7, 16])
def test_stencil27(side):
    A = gen.stencil27(side)
    A.check()
    assert A.nnz == (3 * side - 2) ** 3
    assert set(np.unique(A.val).tolist()) == {-1.0, 26.0}
    B = gen.stencil27(side, seed=1)
    S = sp.csr_matrix((B.val, B.col, B.rowptr))
    assert abs(S - S.T).max() == 0
    # diagonal = sum of the 26 slot weights; the interior row sums to zero
    assert np.all(S.diagonal() > 0)
    assert np.array_equal(B.col, A.col) and np.array_equal(B.rowptr, A.rowptr)


def test_seeded_determinism():
    a = gen.stencil27(10, seed=1).digest()
    b = gen.stencil27(10, seed=1).digest()
    c = gen.stencil27(10, seed=2).digest()
    assert a == b != c


def test_one_dimensional_operator_and_single_node_aggregates():
    """The inputs of the 17 M-row GPU test at a small size: laplacian7(n, 1, 1) is the tridiagonal
    operator (diagonal 6, neighbours -1), and one damped-Jacobi step over single-node aggregates
    gives P = I - (2/3) D^-1 A, tridiagonal and square: diagonal 1/3, neighbours 1/9."""
    n = 50
    A = gen.laplacian7(n, 1, 1)
    A.check()
    S = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(n, n)).toarray()
    T = 6.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    assert A.nnz == 3 * n - 2 and np.array_equal(S, T)
    P = gen.smoothed_aggregation(A, n, 1, 1, agg=1, steps=1)
    P.check()
    assert P.n_rows == n and P.n_cols == n and P.nnz == 3 * n - 2
    D = sp.csr_matrix((P.val, P.col, P.rowptr), shape=(n, n)).toarray()
    assert np.allclose(D, np.eye(n) / 3 + (np.eye(n, k=1) + np.eye(n, k=-1)) / 9, rtol=0, atol=1e-15)


def test_smoothed_aggregation_row_lengths():
    s = 12
    A = gen.stencil27(s, seed=2, eps_z=0.01)
    P1 = gen.smoothed_aggregation(A, s, s, s, steps=1)
    P2 = gen.smoothed_aggregation(A, s, s, s, steps=2)
    P1.check(); P2.check()
    l1, l2 = np.diff(P1.rowptr), np.diff(P2.rowptr)
    assert l1.min() >= 1 and l1.max() == 8
    assert l2.max() == 27
    assert P1.n_cols == (s // 3) ** 3


def test_block_variant():
    B = gen.block_stencil27(5, 4, seed=2)
    B.check()
    S = sp.csr_matrix((B.val, B.col, B.rowptr))
    assert abs(S - S.T).max() == 0
    off = abs(S).sum(axis=1).A.ravel() - np.abs(S.diagonal())
    assert np.all(S.diagonal() > off)
    P = gen.block_smoothed_aggregation(B, 5, 4)
    P.check()
    assert P.n_rows == 4 * 125 and P.n_cols == 4 * 8


def test_random_csr_edge_features():
    M = gen.random_csr(50, 20, 0.3, seed=1, empty_rows=0.3, zero_cols=3, explicit_zeros=0.2)
    M.check()
    lens = np.diff(M.rowptr)
    assert (lens == 0).any()
    assert (M.val == 0.0).any()
    assert np.setdiff1d(np.arange(20), M.col).size >= 3


def test_batch_sides_and_hierarchy():
    s = gen.batch_problem_sides()
    assert s.shape == (64, 3) and s.min() >= 12 and s.max() <= 64
    assert gen.hierarchy_sides(256, 6) == [256, 128, 64, 32, 16, 8]
