"""Batched form: several plans in one persistent launch per level, recorded once into a HIP
graph and replayed.  Results must match the plain per-plan numeric on the same GPU and the
oracle."""
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


def _independent(count, lo, hi, seed):
    sides = gen.batch_problem_sides(count, seed=seed, lo=lo, hi=hi)
    probs = []
    for k, (nx, ny, nz) in enumerate(sides):
        A = gen.stencil27(int(nx), int(ny), int(nz), seed=100 + k)
        P = gen.trilinear(int(nx), int(ny), int(nz))
        probs.append(GpuProblem(A, P))
    return probs


@pytest.mark.parametrize("count,lo,hi", [(6, 3, 12), (16, 5, 20)])
def test_independent_problems(count, lo, hi):
    probs = _independent(count, lo, hi, seed=3)
    plans = [g.plan(algo="merged") for g in probs]
    plain = [p.numeric(g.A_val, g.P_val) for p, g in zip(plans, probs)]
    C = [torch.full((p.nnz_C,), np.nan, dtype=torch.float64, device="cuda") for p in plans]
    batch = lib.Batch(plans)
    batch.numeric([g.A_val for g in probs], [g.P_val for g in probs], C)
    torch.cuda.synchronize()
    for g, p, c, c0 in zip(probs, plans, C, plain):
        ref = oracle.ptap(g.A, g.P)
        got = c.cpu().numpy()
        assert_close(got, ref.val, ref.abs)
        assert_close(got, c0.cpu().numpy(), ref.abs)
    batch.close()
    for p in plans:
        p.close()


def test_graph_replays_with_new_values():
    """The graph is recorded once; every replay (with eager work and synchronisation between
    them) must give the result of the current values."""
    probs = _independent(5, 4, 10, seed=7)
    plans = [g.plan(algo="merged") for g in probs]
    C = [torch.empty(p.nnz_C, dtype=torch.float64, device="cuda") for p in plans]
    batch = lib.Batch(plans)
    rng = np.random.default_rng(11)
    for rep in range(4):
        vals = []
        for g in probs:
            Av = rng.uniform(-1, 1, g.A.nnz)
            Pv = rng.uniform(-1, 1, g.P.nnz)
            g.A_val.copy_(torch.from_numpy(Av))
            g.P_val.copy_(torch.from_numpy(Pv))
            vals.append((Av, Pv))
        torch.cuda.synchronize()
        x = torch.randn(1000, device="cuda").sum()  # unrelated eager work between replays
        batch.numeric([g.A_val for g in probs], [g.P_val for g in probs], C)
        torch.cuda.synchronize()
        del x
        for g, c, (Av, Pv) in zip(probs, C, vals):
            ref = oracle.ptap(g.A.with_values(Av), g.P.with_values(Pv))
            assert_close(c.cpu().numpy(), ref.val, ref.abs, f"replay {rep}")
    batch.close()
    for p in plans:
        p.close()


def test_hierarchy_levels_bit_exact():
    """A geometric hierarchy from a 17^3 7-point Laplacian with trilinear interpolations: level
    l+1 multiplies the previous level's C.  All values are dyadic, so every level must match the
    oracle (applied level by level to its own results) bit for bit."""
    sides = gen.hierarchy_sides(17, 4)  # 17, 9, 5, 3
    A0 = gen.laplacian7(sides[0])
    Ps = [gen.trilinear(s) for s in sides[:-1]]
    d = lambda a, t: torch.as_tensor(np.ascontiguousarray(a), dtype=t).cuda()  # noqa: E731
    plans, A_rowptr, A_col, keep = [], d(A0.rowptr, torch.int32), d(A0.col, torch.int32), []
    P_dev = []
    for l, P in enumerate(Ps):
        Prp, Pc, Pv = d(P.rowptr, torch.int32), d(P.col, torch.int32), d(P.val, torch.float64)
        plan = lib.Plan(P.n_rows, P.n_cols, A_rowptr, A_col, Prp, Pc, algo="merged")
        plans.append(plan)
        keep.append((A_rowptr, A_col, Prp, Pc))
        P_dev.append(Pv)
        A_rowptr, A_col = plan.pattern()
    C = [torch.empty(p.nnz_C, dtype=torch.float64, device="cuda") for p in plans]
    A_vals = [d(A0.val, torch.float64)] + C[:-1]
    batch = lib.Batch(plans, levels=list(range(len(plans))))
    for rep in range(2):
        batch.numeric(A_vals, P_dev, C)
        torch.cuda.synchronize()
        A = A0
        for l, P in enumerate(Ps):
            ref = oracle.ptap(A, P)
            got = C[l].cpu().numpy()
            assert np.array_equal(got, ref.val), f"level {l} replay {rep}"
            A = gen.CSR(P.n_cols, P.n_cols, ref.rowptr, ref.col, ref.val)
    batch.close()
    for p in plans:
        p.close()


def test_batch_with_general_tiles():
    """A plan whose rows exceed the short-row limits (smoothed aggregation with two smoothing
    steps) runs its tiles in the general kernel inside the same graph."""
    s = 9
    A = gen.stencil27(s, seed=2, eps_z=0.01)
    P = gen.smoothed_aggregation(A, s, s, s, steps=2)
    probs = [GpuProblem(A, P)] + _independent(3, 4, 8, seed=5)
    plans = [g.plan(algo="merged") for g in probs]
    C = [torch.empty(p.nnz_C, dtype=torch.float64, device="cuda") for p in plans]
    batch = lib.Batch(plans)
    batch.numeric([g.A_val for g in probs], [g.P_val for g in probs], C)
    torch.cuda.synchronize()
    for g, c in zip(probs, C):
        ref = oracle.ptap(g.A, g.P)
        assert_close(c.cpu().numpy(), ref.val, ref.abs)
    batch.close()
    for p in plans:
        p.close()


@pytest.mark.slow
def test_batch_with_A_values_past_2GiB():
    """A 216^3 plan (269,586,136 entries of A: its values are read by 64-bit address) in one level
    with three small plans: it is launched on its own inside the graph, the small ones through the
    batched kernel, and every C matches the oracle."""
    A = gen.stencil27(216, seed=7)
    P = gen.trilinear(216)
    assert A.nnz * 8 >= 2**31
    probs = [GpuProblem(A, P)] + _independent(3, 4, 8, seed=6)
    plans = [g.plan(algo="merged") for g in probs]
    C = [torch.full((p.nnz_C,), np.nan, dtype=torch.float64, device="cuda") for p in plans]
    batch = lib.Batch(plans)
    batch.numeric([g.A_val for g in probs], [g.P_val for g in probs], C)
    torch.cuda.synchronize()
    for g, c in zip(probs, C):
        ref = oracle.ptap(g.A, g.P)
        assert_close(c.cpu().numpy(), ref.val, ref.abs)
    batch.close()
    for p in plans:
        p.close()


def test_batch_rejects_changed_pointers_and_bad_plans():
    probs = _independent(2, 4, 6, seed=9)
    plans = [g.plan(algo="merged") for g in probs]
    C = [torch.empty(p.nnz_C, dtype=torch.float64, device="cuda") for p in plans]
    batch = lib.Batch(plans)
    batch.numeric([g.A_val for g in probs], [g.P_val for g in probs], C)
    C2 = [torch.empty_like(c) for c in C]
    st = lib.ptap_batch_numeric(batch.handle, [g.A_val for g in probs], [g.P_val for g in probs], C2)
    assert st == lib.PTAP_ERR_INPUT
    batch.close()
    two = probs[0].plan(algo="twostep")
    st, h = lib.ptap_batch_create([two.handle])
    assert st == lib.PTAP_ERR_UNSUPPORTED and not h.value
    two.close()
    for p in plans:
        p.close()


def test_tune_picks_a_measured_plan_with_the_same_product():
    """tune(): every candidate plan computes the same product; the returned plan is the fastest
    candidate of the report and its result matches the oracle."""
    import oracle
    from helpers import assert_close
    A, P = gen.stencil27(20, seed=3), gen.trilinear(20)
    d = lambda a, t: torch.as_tensor(np.ascontiguousarray(a), dtype=t).cuda()  # noqa: E731
    Av, Pv = d(A.val, torch.float64), d(P.val, torch.float64)
    plan, report = lib.tune(A.n_rows, P.n_cols, d(A.rowptr, torch.int32), d(A.col, torch.int32),
                            d(P.rowptr, torch.int32), d(P.col, torch.int32), Av, Pv, reps=2)
    assert len(report) == len(lib.TUNE_CANDIDATES)
    best = min(report, key=lambda r: r["numeric_ms"])
    assert plan.tuned_options == best["options"]
    C = plan.numeric(Av, Pv).cpu().numpy()
    ref = oracle.ptap(A, P)
    assert_close(C, ref.val, ref.abs)
    plan.close()
