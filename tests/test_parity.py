"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

The C pattern must be bit-exact (row pointers and sorted columns).  Values are bit-exact on
dyadic inputs (constant-coefficient stencils with trilinear interpolation: every product and
partial sum is exact in FP64) and otherwise within the FP64 criterion of tests/helpers.py."""
import numpy as np
import pytest
import torch

import oracle
import ptap_inputs as gen

pytestmark = pytest.mark.gpu

ALGO_FOLD = [("merged", "owner"), ("allatonce", "owner"), ("merged", "atomic"),
             ("allatonce", "atomic"), ("twostep", "auto")]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


from gpu_util import check_against_oracle  # noqa: E402


@pytest.mark.parametrize("algo,fold", ALGO_FOLD)
@pytest.mark.parametrize("K", [1, 3, 8])
def test_c1_bit_exact(algo, fold, K):
    A, P, _ = gen.galerkin_workload("c1")
    check_against_oracle(A, P, exact=True, algo=algo, fold=fold, nblocks=K)


@pytest.mark.parametrize("fold", ["owner", "atomic"])
@pytest.mark.parametrize("K", [5000, 600000])
def test_two_pass_more_blocks_than_rows(fold, K):
    """All-at-once with more ownership blocks than fine rows (most entries of P off-block): the
    block index takes 32-bit arithmetic at K = 5000 (n K < 2^31) and 64-bit at K = 600000."""
    A, P, _ = gen.galerkin_workload("c1")
    assert A.n_rows * 5000 < 2**31 <= A.n_rows * 600000
    check_against_oracle(A, P, exact=True, algo="allatonce", fold=fold, nblocks=K)


@pytest.mark.parametrize("algo,fold", ALGO_FOLD)
def test_toy_rowwise(algo, fold):
    A, P = gen.toy_rowwise(seed=4)
    check_against_oracle(A, P, algo=algo, fold=fold, nblocks=3)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("algo,fold", ALGO_FOLD)
def test_random_fuzz(seed, algo, fold):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(1, 300))
    m = int(rng.integers(1, 60))
    A = gen.random_csr(n, n, float(rng.uniform(0.005, 0.05)), seed=seed, empty_rows=0.1,
                       explicit_zeros=0.05)
    P = gen.random_csr(n, m, float(rng.uniform(0.01, 0.15)), seed=900 + seed, empty_rows=0.15,
                       zero_cols=2 if m > 4 else 0, explicit_zeros=0.05)
    check_against_oracle(A, P, algo=algo, fold=fold, nblocks=int(rng.integers(1, 5)))


@pytest.mark.parametrize("algo,fold", ALGO_FOLD)
@pytest.mark.parametrize("case", ["c2_20", "c3a_12", "c3b_9", "c3c_6"])
def test_workloads_reduced(algo, fold, case):
    A, P = _case(case)
    check_against_oracle(A, P, algo=algo, fold=fold)


@pytest.mark.parametrize("algo,fold", [("merged", "owner"), ("merged", "atomic"), ("twostep", "auto"),
                                       ("allatonce", "owner")])
@pytest.mark.parametrize("case", ["c3c_7", "random_long"])
def test_forced_spill(algo, fold, case):
    """Hash tables capped at 64 slots: rows of AP with more than 32 keys (up to 108 for the
    4x4-block operator, 87 for the random one) go to tables in device memory; the plan reports
    the slots it keeps there."""
    if case == "random_long":
        A = gen.random_csr(300, 300, 0.06, seed=31, empty_rows=0.05)
        P = gen.random_csr(300, 90, 0.1, seed=32, empty_rows=0.05, zero_cols=3)
    else:
        A, P = _case(case)
    st = check_against_oracle(A, P, algo=algo, fold=fold, hash_slots=64, nblocks=3 if algo == "allatonce" else 1)
    assert st["table_slots"] > 0, st


@pytest.mark.parametrize("te", [1593, 2105, 2361, 2729])
def test_general_owner_kernel_odd_tile_size(te):
    """The general owner kernel with an odd tile size: its LDS regions once sat back to back, so an
    odd number of tile entries put the wavefront scratch and the tables' FP64 values at addresses
    4 mod 8 (the failing runs had 1593 or 2729 entries).  The 4x4-block operator's rows of A hold
    108 entries, so every scratch slot is used."""
    A = gen.block_stencil27(12, 4, seed=2)
    P = gen.block_smoothed_aggregation(A, 12, 4)
    st = check_against_oracle(A, P, algo="merged", fold="owner", tile_entries=te)
    assert st["tile_entries"] == te and te % 2 == 1


@pytest.mark.parametrize("tile_entries", [16, 100, 700])
def test_owner_tile_sizes(tile_entries):
    """Small tiles: many tiles, rows longer than a tile go to device-memory tiles."""
    A, P = _case("c3b_9")
    check_against_oracle(A, P, algo="merged", fold="owner", tile_entries=tile_entries)
    A, P, _ = gen.galerkin_workload("c1")
    check_against_oracle(A, P, exact=True, algo="allatonce", fold="owner", nblocks=4,
                         tile_entries=tile_entries)


@pytest.mark.parametrize("xcd", [False, True])
def test_xcd_remap_same_result(xcd):
    A, P, _ = gen.galerkin_workload("c1")
    check_against_oracle(A, P, exact=True, algo="merged", fold="owner", xcd_remap=xcd, tile_entries=300)


def test_edge_single_and_empty():
    A = gen.CSR(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([3.0]))
    P = gen.CSR(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.0]))
    for algo, fold in ALGO_FOLD:
        check_against_oracle(A, P, exact=True, algo=algo, fold=fold)
    # A with no entries: C has no entries at all
    A = gen.CSR(5, 5, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0))
    P = gen.random_csr(5, 3, 0.5, seed=1)
    for algo, fold in ALGO_FOLD:
        check_against_oracle(A, P, algo=algo, fold=fold)


def test_repeated_numeric_new_values():
    """One symbolic, several numerics with new values (Section 4.1 runs 1 + 11)."""
    from gpu_util import GpuProblem
    A, P = _case("c2_20")
    g = GpuProblem(A, P)
    plan = g.plan(algo="merged")
    rng = np.random.default_rng(3)
    for _ in range(3):
        Av = rng.uniform(-1, 1, A.nnz)
        Pv = rng.uniform(-1, 1, P.nnz)
        g.A_val.copy_(torch.from_numpy(Av))
        g.P_val.copy_(torch.from_numpy(Pv))
        C = plan.numeric(g.A_val, g.P_val).cpu().numpy()
        ref = oracle.ptap(A.with_values(Av), P.with_values(Pv))
        from helpers import assert_close
        assert_close(C, ref.val, ref.abs)
    plan.close()


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
    raise KeyError(case)


@pytest.mark.parametrize("waves", [4, 8, 16])
@pytest.mark.parametrize("algo,K", [("merged", 1), ("allatonce", 4)])
def test_owner_waves(waves, algo, K):
    """The short-row owner kernel with each workgroup size (and the two-pass form)."""
    A, P, _ = gen.galerkin_workload("c1")
    check_against_oracle(A, P, exact=True, algo=algo, fold="owner", nblocks=K, owner_waves=waves)
    A, P = _case("c2_20")
    check_against_oracle(A, P, algo=algo, fold="owner", nblocks=K, owner_waves=waves, tile_entries=500)


@pytest.mark.parametrize("case", ["c1", "c2_20", "c3a_12", "c3b_9", "c3c_6", "fuzz"])
def test_numeric_cache(case):
    """Numeric cache (packed extents of the rows of P per entry of A, Section 4.2's caching of
    intermediate data): same results as without it, and its size is reported."""
    from gpu_util import GpuProblem
    if case == "c1":
        A, P, _ = gen.galerkin_workload("c1")
    elif case == "fuzz":
        A = gen.random_csr(250, 250, 0.04, seed=11, empty_rows=0.1, explicit_zeros=0.05)
        P = gen.random_csr(250, 40, 0.08, seed=12, empty_rows=0.15, zero_cols=2, explicit_zeros=0.05)
    else:
        A, P = _case(case)
    exact = case == "c1"
    for algo, K in [("merged", 1), ("allatonce", 3)]:
        st = check_against_oracle(A, P, exact=exact, algo=algo, fold="owner", nblocks=K, cache=True)
        assert st["cache_bytes"] in (0, 4 * A.nnz)
    st = check_against_oracle(A, P, exact=exact, algo="merged", fold="owner", cache=True, tile_entries=120)
    if case in ("c1", "c2_20"):
        assert st["cache_bytes"] == 4 * A.nnz  # every tile takes the short-row kernel here
    g = GpuProblem(A, P)
    plain = g.plan(algo="merged", fold="owner")
    assert plain.stats()["cache_bytes"] == 0
    plain.close()



def test_forced_hash_multiplier_same_product():
    """ptap_options.hash_mul: any odd multiplier of the short-row kernel's R_I hash gives the same
    C (bit-exact on dyadic C1; under the value criterion on a lognormal operator), and the stats
    report the multiplier in use."""
    from gpu_util import GpuProblem
    from helpers import assert_close
    for A, P, exact in [(gen.laplacian7(16), gen.trilinear(16), True),
                        (gen.stencil27(20, seed=3), gen.trilinear(20), False)]:
        g = GpuProblem(A, P)
        ref = oracle.ptap(A, P)
        for mul in (0x9E3779B1, 0x00000001, 0x7FFFFFFF, 0xDEADBEEF):
            plan = g.plan(fold="owner", hash_mul=mul)
            assert plan.stats()["hash_mul"] == mul
            C = plan.numeric(g.A_val, g.P_val).cpu().numpy()
            if exact:
                assert np.array_equal(C, ref.val)
            else:
                assert_close(C, ref.val, ref.abs)
            plan.close()



def _mixed_long_short(seed):
    """Fine rows n = 3000, coarse m = 400: a banded A (7 entries a row) with every 1500th row dense
    (600 random columns), and a P whose rows mostly take one to three nearby coarse columns while
    every 700th row takes 30 random ones.  Most rows stay short; the long ones outgrow the
    symbolic phase's one-pass tables (|R_I| beyond 31 keys, C(i,:) beyond 191 columns, the fine
    rows S_i reached through A beyond 447), so the class launches that take over run beside the
    one-pass kernels in one plan."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    n, m = 3000, 400
    rows, cols = [], []
    for i in range(n):
        c = set(range(max(0, i - 3), min(n, i + 4)))
        if i % 1500 == 0:
            c |= set(rng.choice(n, size=600, replace=False).tolist())
        rows += [i] * len(c)
        cols += sorted(c)
    A = sp.csr_matrix((rng.uniform(-1, 1, len(rows)), (rows, cols)), shape=(n, n))
    rows, cols = [], []
    for I in range(n):
        base = I * m // n
        c = set(range(base, min(m, base + 1 + I % 3)))
        if I % 700 == 0:
            c |= set(rng.choice(m, size=30, replace=False).tolist())
        rows += [I] * len(c)
        cols += sorted(c)
    P = sp.csr_matrix((rng.uniform(-1, 1, len(rows)), (rows, cols)), shape=(n, m))
    return gen.from_scipy(A), gen.from_scipy(P)


@pytest.mark.parametrize("algo,fold,K", [("merged", "owner", 1), ("allatonce", "owner", 3),
                                         ("merged", "atomic", 1), ("twostep", "auto", 1),
                                         ("merged", "auto", 1)])
def test_symbolic_fallback_rows(algo, fold, K):
    import scipy.sparse as sp
    A, P = _mixed_long_short(seed=11)
    # the input reaches every path: rows of C within the row store (<= 32), longer rows within the
    # one-pass table (<= 191), rows beyond it, S_i beyond 447 and R_I beyond 31 keys
    Ab = sp.csr_matrix((np.ones(A.nnz), A.col, A.rowptr), shape=(A.n_rows, A.n_rows))
    Pb = sp.csr_matrix((np.ones(P.nnz), P.col, P.rowptr), shape=(P.n_rows, P.n_cols))
    c_len = np.diff((Pb.T @ Ab @ Pb).tocsr().indptr)
    assert (c_len <= 32).any() and ((c_len > 32) & (c_len <= 191)).any() and (c_len > 191).any()
    assert np.diff((Pb.T @ Ab).tocsr().indptr).max() > 447
    assert np.diff((Ab @ Pb).tocsr().indptr).max() > 31
    check_against_oracle(A, P, algo=algo, fold=fold, nblocks=K)
