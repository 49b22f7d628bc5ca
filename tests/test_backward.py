"""Adjoint of the triple product on the GPU: dA = P dC P^T on A's pattern, dP = A P dC^T + A^T P dC
on P's pattern, for the loss L = sum(W o C).

Checks: the oracle's adjoint (the same adjoint applied to |A|, |P|, |W| bounds the rounding), the
dense matrix-calculus gradient at 8^3, central finite differences of the GPU forward on 200
random entries of each gradient at 64^3 (L is linear in A and quadratic in P, so the central
difference carries rounding only), the adjoint (dot-product) identities at 64^3, and torch's
gradcheck through the autograd function."""
import numpy as np
import pytest
import torch

import oracle
import ptap_inputs as gen
from helpers import assert_close, dense, dense_pattern

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


import paper_1905_08423_amd as lib  # noqa: E402
from gpu_util import GpuProblem  # noqa: E402


def _bounds(A, P, rp, col, W):
    Aa = A.with_values(np.abs(A.val))
    Pa = P.with_values(np.abs(P.val))
    return oracle.ptap_backward(Aa, Pa, rp, col, np.abs(W))


def _gpu_backward(g, plan, W):
    Wd = torch.as_tensor(W).cuda()
    dA, dP = plan.backward(g.A_val, g.P_val, Wd)
    torch.cuda.synchronize()
    return dA.cpu().numpy(), dP.cpu().numpy()


def _grouped(seed=3):
    """Coarse columns in groups of g; every row of C is its whole group (a fine row per group
    holds all g entries, A couples fine rows of one group only).  A fine row with np entries in
    a group of g walks np*g entries of dC, so g = 16 gives walks 16, 64, 128, 192, 256 whose
    segments end exactly on 64-lane pass boundaries, g = 64 one segment per pass, and g = 17,
    65 rows just past 256 (general kernel) beside rows at 255.  Also rows with an empty row of P
    and a row with an empty row of A."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    groups = [(16, [1, 4, 8, 12, 16, 0]), (17, [15, 16, 17]), (64, [1, 2, 4]), (65, [4, 1]),
              (16, [16, 8, 4])]
    prow, pcol, members = [], [], []
    c0 = I = 0
    for g, nps in groups:
        rows = []
        for npi in [g] + nps:
            cols = np.sort(rng.choice(g, size=npi, replace=False)) + c0
            prow += [I] * npi
            pcol += list(cols)
            rows.append(I)
            I += 1
        members.append(rows)
        c0 += g
    n, m = I + 1, c0  # the last fine row has a row of P but none of A
    prow += [I, I]
    pcol += [0, 1]
    P = sp.csr_matrix((rng.uniform(-1, 1, len(prow)), (prow, pcol)), shape=(n, m))
    arow, acol = [], []
    for rows in members:
        for a in rows:
            for b in rows:
                if a == b or rng.random() < 0.5:
                    arow.append(a)
                    acol.append(b)
    A = sp.csr_matrix((rng.uniform(-1, 1, len(arow)), (arow, acol)), shape=(n, n))
    return gen.from_scipy(A), gen.from_scipy(P)


@pytest.mark.parametrize("case", ["random", "c5_8", "c5_12", "c5_12_spill", "sa2_9", "toy", "wide",
                                  "grouped"])
def test_backward_against_oracle(case):
    """Rows with short walks over dC take the short-row kernel, the others the general one;
    c5_12_spill caps on-chip tables at 64 slots, so most rows use device-memory tables."""
    kw = {}
    if case == "random":
        A = gen.random_csr(200, 200, 0.03, seed=3, empty_rows=0.1, explicit_zeros=0.05)
        P = gen.random_csr(200, 40, 0.08, seed=4, empty_rows=0.1, zero_cols=2)
    elif case == "toy":
        A, P = gen.toy_rowwise(seed=1)
    elif case.startswith("sa2"):
        s = int(case.split("_")[1])
        A = gen.stencil27(s, seed=2, eps_z=0.01)
        P = gen.smoothed_aggregation(A, s, s, s, steps=2)
    elif case == "grouped":
        A, P = _grouped()
    elif case == "wide":
        # a small coarse space with long rows of C: a quarter of the rows walk 65..256 entries
        # of dC (two to four passes), the rest walk more and take the general kernel
        A = gen.random_csr(300, 300, 0.01, seed=11, empty_rows=0.05)
        P = gen.random_csr(300, 60, 0.1, seed=12, empty_rows=0.05)
    else:
        s = int(case.split("_")[1])
        A, P = gen.stencil27(s, seed=4), gen.trilinear(s)
        if case.endswith("spill"):
            kw["hash_slots"] = 64
    g = GpuProblem(A, P)
    plan = g.plan(algo="merged", backward=True, **kw)
    rp, col = (t.cpu().numpy() for t in plan.pattern())
    W = gen.loss_weights(plan.nnz_C, seed=5)
    dA, dP = _gpu_backward(g, plan, W)
    rA, rP = oracle.ptap_backward(A, P, rp, col, W)
    bA, bP = _bounds(A, P, rp, col, W)
    assert_close(dA, rA, bA, "dA")
    assert_close(dP, rP, bP, "dP")
    plan.close()


def test_backward_dense_8cubed():
    """Dense gradient at 8^3 (n = 512, m = 64): P W P^T and A P W^T + A^T P W, masked."""
    A, P = gen.stencil27(8, seed=4), gen.trilinear(8)
    g = GpuProblem(A, P)
    plan = g.plan(algo="merged", backward=True)
    rp, col = (t.cpu().numpy() for t in plan.pattern())
    W = gen.loss_weights(plan.nnz_C, seed=5)
    dA, dP = _gpu_backward(g, plan, W)
    Wd = np.zeros((P.n_cols, P.n_cols))
    for i in range(P.n_cols):
        Wd[i, col[rp[i]:rp[i + 1]]] = W[rp[i]:rp[i + 1]]
    Ad, Pd = dense(A), dense(P)
    gA = (Pd @ Wd @ Pd.T)[dense_pattern(A)]
    gP = (Ad @ Pd @ Wd.T + Ad.T @ Pd @ Wd)[dense_pattern(P)]
    Wa = np.abs(Wd)
    bA = (np.abs(Pd) @ Wa @ np.abs(Pd).T)[dense_pattern(A)]
    bP = (np.abs(Ad) @ np.abs(Pd) @ Wa.T + np.abs(Ad).T @ np.abs(Pd) @ Wa)[dense_pattern(P)]
    assert_close(dA, gA, bA, "dA")
    assert_close(dP, gP, bP, "dP")
    plan.close()


@pytest.fixture(scope="module")
def c5():
    """64^3 27-point lognormal (seed 4), trilinear to 32^3, W ~ N(0,1) on C's pattern (seed 5)."""
    A, P = gen.stencil27(64, seed=4), gen.trilinear(64)
    g = GpuProblem(A, P)
    plan = g.plan(algo="merged", backward=True)
    rp, col = (t.cpu().numpy() for t in plan.pattern())
    W = gen.loss_weights(plan.nnz_C, seed=5)
    dA, dP = _gpu_backward(g, plan, W)
    yield g, plan, rp, col, W, dA, dP
    plan.close()


def _fd(plan, g, which, k, rows_mask, h=1e-6):
    """Central difference of L on the C entries the perturbation can change."""
    vals = g.A_val if which == "A" else g.P_val
    base = vals[k].item()
    C = []
    for sgn in (1.0, -1.0):
        vals[k] = base + sgn * h
        C.append(plan.numeric(g.A_val, g.P_val))
    vals[k] = base
    torch.cuda.synchronize()
    diff = (C[0] - C[1])[rows_mask]
    return diff


def test_backward_full_64cubed_against_oracle(c5):
    """Every entry of dA and dP at the differentiation workload's size against the oracle's
    adjoint, under the FP64 criterion with the adjoint of |A|, |P|, |W| as the scale."""
    g, plan, rp, col, W, dA, dP = c5
    rA, rP = oracle.ptap_backward(g.A, g.P, rp, col, W)
    bA, bP = _bounds(g.A, g.P, rp, col, W)
    assert_close(dA, rA, bA, "dA")
    assert_close(dP, rP, bP, "dP")


def test_backward_finite_differences_64cubed(c5):
    g, plan, rp, col, W, dA, dP = c5
    A, P = g.A, g.P
    h = 1e-6
    Wt = torch.as_tensor(W).cuda()
    rng = np.random.default_rng(6)
    m = P.n_cols
    rowid = np.repeat(np.arange(m), np.diff(rp))
    rowid_t = torch.as_tensor(rowid).cuda()
    col_t = torch.as_tensor(col).cuda()
    worst = 0.0
    for k in rng.choice(A.nnz, size=200, replace=False):
        I = int(np.searchsorted(A.rowptr, k, side="right") - 1)
        J = int(A.col[k])
        rows_i = torch.as_tensor(P.col[P.rowptr[I]:P.rowptr[I + 1]]).cuda()
        cols_j = torch.as_tensor(P.col[P.rowptr[J]:P.rowptr[J + 1]]).cuda()
        mask = torch.isin(rowid_t, rows_i) & torch.isin(col_t, cols_j)
        diff = _fd(plan, g, "A", int(k), mask, h)
        fd = float((Wt[mask] * diff).sum().item()) / (2 * h)
        err = abs(fd - dA[k]) / max(1.0, abs(dA[k]))
        worst = max(worst, err)
        assert err <= 1e-6, (k, fd, dA[k])
    for k in rng.choice(P.nnz, size=200, replace=False):
        kk = int(P.col[k])
        mask = (rowid_t == kk) | (col_t == kk)
        diff = _fd(plan, g, "P", int(k), mask, h)
        fd = float((Wt[mask] * diff).sum().item()) / (2 * h)
        err = abs(fd - dP[k]) / max(1.0, abs(dP[k]))
        worst = max(worst, err)
        assert err <= 1e-6, (k, fd, dP[k])
    print(f"finite differences: worst relative error {worst:.2e}")


def test_adjoint_identities_64cubed(c5):
    """<dA, dAx> = <W, P^T dAx P> and <dP, dPx> = <W, dPx^T A P + P^T A dPx> for random
    directions on the patterns; the right-hand sides come from the oracle's general Q1^T A Q2."""
    g, plan, rp, col, W, dA, dP = c5
    A, P = g.A, g.P
    rng = np.random.default_rng(8)
    dAx = rng.standard_normal(A.nnz)
    rhs_A = float(np.dot(W, oracle.ptap(A.with_values(dAx), P).val))
    lhs_A = float(np.dot(dA, dAx))
    dPx = rng.standard_normal(P.nnz)
    Px = P.with_values(dPx)
    r1 = oracle.rap(Px, A, P)
    r2 = oracle.rap(P, A, Px)
    assert np.array_equal(r1.col, col) and np.array_equal(r2.col, col)
    rhs_P = float(np.dot(W, r1.val + r2.val))
    lhs_P = float(np.dot(dP, dPx))
    Aa, Pa = A.with_values(np.abs(A.val)), P.with_values(np.abs(P.val))
    Wa = np.abs(W)
    scale_A = float(np.dot(Wa, oracle.ptap(A.with_values(np.abs(dAx)), Pa).val))
    Pxa = P.with_values(np.abs(dPx))
    scale_P = float(np.dot(Wa, oracle.rap(Pxa, Aa, Pa).val + oracle.rap(Pa, Aa, Pxa).val))
    assert abs(lhs_A - rhs_A) <= 1e-12 * scale_A, (lhs_A, rhs_A, scale_A)
    assert abs(lhs_P - rhs_P) <= 1e-12 * scale_P, (lhs_P, rhs_P, scale_P)


def test_autograd_function_and_gradcheck():
    A, P = gen.stencil27(4, seed=9), gen.trilinear(4)
    g = GpuProblem(A, P)
    plan = g.plan(algo="merged", backward=True)
    W = torch.as_tensor(gen.loss_weights(plan.nnz_C, seed=2)).cuda()
    Av = g.A_val.clone().requires_grad_(True)
    Pv = g.P_val.clone().requires_grad_(True)
    C = lib.ptap(plan, Av, Pv)
    (C * W).sum().backward()
    dA, dP = plan.backward(g.A_val, g.P_val, W)
    # dA has no atomics (bitwise repeatable); dP gathers its terms with device-wide atomic adds,
    # so two calls may differ in the order of the additions, i.e. in rounding only
    assert torch.equal(Av.grad, dA)
    assert float((Pv.grad - dP).abs().max()) <= 1e-13 * float(dP.abs().max())
    # C is linear in A and quadratic in P: central differences are exact for any step, so a large
    # step keeps the rounding noise of the forward (its atomic order varies) far below atol
    f = lambda a, p: lib.ptap(plan, a, p)  # noqa: E731
    assert torch.autograd.gradcheck(f, (Av.detach().clone().requires_grad_(True),
                                        Pv.detach().clone().requires_grad_(True)),
                                    eps=1e-3, atol=1e-9, rtol=1e-7, nondet_tol=1e-12)
    plan.close()
