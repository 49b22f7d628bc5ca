"""GPU parity at the full sizes of the paper-shaped workloads.

The 128^3 27-point -> 64^3 trilinear product runs in the launch configuration the benchmark times
(merged all-at-once, K = 1, owner fold, default tiles and workgroup size) and in every other
algorithm; the whole C is compared with the oracle: the pattern bit for bit, the values under the
FP64 criterion of tests/helpers.py.  With constant coefficients (diagonal 26, off-diagonal -1) every
product and partial sum is a dyadic rational well inside FP64's range, so there the values must be
bit-exact at full size too.  The 96^3 smoothed-aggregation cases (one and two Jacobi steps) are
compared in full, and so is the 4x4-block case (3.5 M rows, 374 M entries of A), whose rows take the
general owner kernel; the oracle runs over the host's threads (each row of C on its own, so the
result is the same as on one thread).  Every comparison prints how many entries lie beyond a plain
1e-12 relative test (tests/helpers.py parity_report; run with -s), beside the criterion applied."""
import numpy as np
import pytest
import torch

import oracle
import ptap_inputs as gen
from helpers import assert_close, parity_report

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


def _check_full(g, ref, exact=False, ref_ld=None, name="", **kw):
    rp, col, val, st = _gpu_c(g, **kw)
    assert np.array_equal(rp, ref.rowptr), "C row pointers differ from the oracle"
    assert np.array_equal(col, ref.col), "C column indices differ from the oracle"
    if exact:
        bad = int((val != ref.val).sum())
        assert bad == 0, f"{bad} values not bit-exact, max diff {np.abs(val - ref.val).max()}"
    else:
        assert_close(val, ref.val, ref.abs)
    parity_report(name or "full " + ",".join(f"{k}={v}" for k, v in kw.items()), val, ref, ref_ld)
    return st


def _oracle(A, P, long_double=False):
    return oracle.ptap(A, P, threads=oracle.cores(), long_double=long_double)


@pytest.fixture(scope="module")
def c2():
    A, P, _ = gen.galerkin_workload("c2")
    yield GpuProblem(A, P), _oracle(A, P), _oracle(A, P, long_double=True)


def test_c2_full_benchmark_configuration(c2):
    g, ref, ld = c2
    st = _check_full(g, ref, ref_ld=ld, name="c2 merged owner (benchmark configuration)")
    assert st["nnz_C"] == 6_859_000
    assert st["fold_used"] == lib.PTAP_FOLD_OWNER and st["rows_needed"] == g.A.n_rows


def test_c2_owner_fold_run_twice(c2):
    """The owner fold adds the contributions of a tile's wavefronts into its LDS rows in the order
    the wavefronts arrive, so two runs on non-dyadic values may differ in the last bits (both
    within the criterion); the count of differing entries is printed.  On dyadic values every
    order gives the same bits (tests elsewhere require bit-exact results there)."""
    g, ref, _ = c2
    plan = g.plan(algo="merged", fold="owner")
    a = plan.numeric(g.A_val, g.P_val).clone()
    b = plan.numeric(g.A_val, g.P_val)
    torch.cuda.synchronize()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    plan.close()
    assert_close(a, ref.val, ref.abs)
    assert_close(b, ref.val, ref.abs)
    print(f"PARITY c2 owner fold run twice: {int((a != b).sum())} of {a.size} entries differ in bits, "
          f"max rel {float(np.abs(a - b).max() / np.abs(ref.val).max()):.3g} of max |C|")


@pytest.mark.parametrize("kw", [dict(algo="allatonce", fold="owner", nblocks=8),
                                dict(algo="merged", fold="owner", nblocks=8),
                                dict(algo="merged", fold="atomic"),
                                dict(algo="allatonce", fold="atomic", nblocks=8),
                                dict(algo="twostep"),
                                dict(algo="merged", fold="owner", cache=True)],
                         ids=["allatonce_K8_owner", "merged_K8_owner", "merged_atomic",
                              "allatonce_K8_atomic", "twostep", "merged_owner_cached"])
def test_c2_full_other_algorithms(c2, kw):
    g, ref, ld = c2
    _check_full(g, ref, ref_ld=ld, **kw)


def test_c2_full_constant_coefficients_bit_exact():
    A, P = gen.stencil27(128), gen.trilinear(128)
    ref = _oracle(A, P)
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
    ref = _oracle(A, P)
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
    ref = _oracle(A, P)
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
    ref = _oracle(A, P)
    g = GpuProblem(A, P)
    _check_full(g, ref)
    _check_full(g, ref, algo="merged", fold="owner", cache=True)


@pytest.mark.parametrize("name", ["c3a", "c3b"])
def test_c3_full_smoothed_aggregation(name):
    """Merged (owner fold), two-step (its short-row kernel walks the rows of P^T, up to 125
    entries, 32 at a time) and the atomic fold, each against the same oracle C."""
    A, P, _ = gen.galerkin_workload(name)
    ref = _oracle(A, P)
    ld = _oracle(A, P, long_double=True)
    g = GpuProblem(A, P)
    _check_full(g, ref, ref_ld=ld, name=f"{name} merged owner")
    _check_full(g, ref, ref_ld=ld, name=f"{name} twostep", algo="twostep")
    _check_full(g, ref, ref_ld=ld, name=f"{name} merged atomic", algo="merged", fold="atomic")


def test_c3c_block_full():
    """The 4x4-block workload in its scalar form: every row of C has 108 entries, so every tile
    takes the general owner kernel (four wavefronts per workgroup).  The whole C against the
    oracle."""
    A, P, _ = gen.galerkin_workload("c3c")
    ref = _oracle(A, P)
    g = GpuProblem(A, P)
    st = _check_full(g, ref, name="c3c scalar merged owner (general kernel)")
    assert st["nnz_C"] == 13_289_344


def test_hierarchy_256_six_levels_bit_exact():
    """The six-level hierarchy of the batched workload: a 256^3 7-point Laplacian (117 M entries)
    with trilinear interpolations 256 -> 128 -> 64 -> 32 -> 16 -> 8.  Level l + 1 multiplies the
    previous level's C.  All values are dyadic, so every level must equal the oracle, applied
    level by level, bit for bit: for the plain numeric of every level and for the batched graph
    (replayed twice)."""
    sides = gen.hierarchy_sides(256, 6)
    A0 = gen.laplacian7(sides[0])
    Ps = [gen.trilinear(s) for s in sides[:-1]]
    refs, A = [], A0
    for P in Ps:
        r = _oracle(A, P)
        refs.append(r)
        A = gen.CSR(P.n_cols, P.n_cols, r.rowptr, r.col, r.val)
    d = lambda a, t: torch.as_tensor(np.ascontiguousarray(a), dtype=t).cuda()  # noqa: E731
    A_rowptr, A_col = d(A0.rowptr, torch.int32), d(A0.col, torch.int32)
    plans, keep, P_vals = [], [], []
    for P in Ps:
        Prp, Pc = d(P.rowptr, torch.int32), d(P.col, torch.int32)
        plan = lib.Plan(P.n_rows, P.n_cols, A_rowptr, A_col, Prp, Pc, algo="merged")
        plans.append(plan)
        keep.append((A_rowptr, A_col, Prp, Pc))
        P_vals.append(d(P.val, torch.float64))
        A_rowptr, A_col = plan.pattern()
    C = [torch.empty(p.nnz_C, dtype=torch.float64, device="cuda") for p in plans]
    A_vals = [d(A0.val, torch.float64)] + C[:-1]
    # plain numerics, level by level
    for l, plan in enumerate(plans):
        rp, col = plan.pattern()
        assert np.array_equal(rp.cpu().numpy(), refs[l].rowptr) and np.array_equal(col.cpu().numpy(), refs[l].col)
        plan.numeric(A_vals[l], P_vals[l], C[l])
        torch.cuda.synchronize()
        assert np.array_equal(C[l].cpu().numpy(), refs[l].val), f"plain level {l}"
    batch = lib.Batch(plans, levels=list(range(len(plans))))
    for rep in range(2):
        for c in C:
            c.fill_(np.nan)
        batch.numeric(A_vals, P_vals, C)
        torch.cuda.synchronize()
        for l in range(len(plans)):
            assert np.array_equal(C[l].cpu().numpy(), refs[l].val), f"batched level {l} replay {rep}"
    batch.close()
    for p in plans:
        p.close()


def test_auto_fold_choice():
    """PTAP_FOLD_AUTO takes the fold the cost model estimates faster (the owner fold where few
    rows of AP are formed twice, the atomic fold where many are or the rows are long), and the
    product is the same: the 128^3 and 96^3 two-step-smoothed-aggregation workloads keep the owner
    fold, the 48^3 two-step smoothed aggregation and the 4x4-block operator at 40^3 nodes take the
    atomic fold; each against the oracle."""
    A2 = gen.stencil27(48, seed=2, eps_z=0.01)
    cases = [("c2", *gen.galerkin_workload("c2")[:2], lib.PTAP_FOLD_OWNER),
             ("c3b", *gen.galerkin_workload("c3b")[:2], lib.PTAP_FOLD_OWNER),
             ("sa2_48", A2, gen.smoothed_aggregation(A2, 48, 48, 48, steps=2), lib.PTAP_FOLD_ATOMIC)]
    Ab = gen.block_stencil27(40, 4, seed=2)
    cases.append(("block_40", Ab, gen.block_smoothed_aggregation(Ab, 40, 4), lib.PTAP_FOLD_ATOMIC))
    for name, A, P, want in cases:
        g = GpuProblem(A, P)
        st = _check_full(g, _oracle(A, P), name=f"{name} auto fold", algo="merged", fold="auto")
        assert st["fold_used"] == want, (name, st["est_owner_ms"], st["est_atomic_ms"])
        assert st["est_owner_ms"] > 0 and st["est_atomic_ms"] > 0
        print(f"PARITY {name}: auto fold {'atomic' if want == lib.PTAP_FOLD_ATOMIC else 'owner'}, "
              f"estimates owner {st['est_owner_ms']:.3f} ms, atomic {st['est_atomic_ms']:.3f} ms")
