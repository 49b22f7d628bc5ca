"""Block-sparse (BSR) plans: C = P^T A P on dense bs x bs blocks.

The oracle is the scalar one: the block matrices are expanded to scalar CSR (every entry of every
stored block stored), the oracle forms C, and the library's block result, expanded the same way,
must have exactly the oracle's pattern and values within the FP64 criterion of tests/helpers.py.
With dense blocks the structural scalar product fills whole blocks, so the two patterns agree
entry for entry."""
import numpy as np
import pytest
import torch

import oracle
import ptap_inputs as gen
from helpers import assert_close


def test_block_layout_round_trip():
    """CPU: the layout helpers the block tests rely on (no arithmetic of the product)."""
    A = gen.block_stencil27(4, 4, seed=2)
    B = gen.csr_to_bsr(A, 4)
    A2 = gen.bsr_to_csr(B)
    assert np.array_equal(A2.rowptr, A.rowptr) and np.array_equal(A2.col, A.col)
    assert np.array_equal(A2.val, A.val)
    R = gen.random_bsr(40, 15, 3, 0.1, seed=1, empty_rows=0.2)
    C = gen.bsr_to_csr(R)
    C.check()
    R2 = gen.csr_to_bsr(C, 3)
    assert np.array_equal(R2.rowptr, R.rowptr) and np.array_equal(R2.col, R.col)
    assert np.array_equal(R2.val, R.val)
    with pytest.raises(ValueError):
        gen.csr_to_bsr(gen.random_csr(8, 8, 0.3, seed=3), 2)


gpu = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bsr_plan(A, P, **kw):
    import paper_1905_08423_amd as lib
    d = lambda a, t: torch.as_tensor(np.ascontiguousarray(a), dtype=t).cuda()  # noqa: E731
    plan = lib.Plan(A.nb, P.mb, d(A.rowptr, torch.int32), d(A.col, torch.int32), d(P.rowptr, torch.int32),
                    d(P.col, torch.int32), block_size=A.bs, **kw)
    keep = [d(A.val.reshape(-1), torch.float64), d(P.val.reshape(-1), torch.float64)]
    return plan, keep


def _gpu_bsr(A, P, **kw):
    plan, (Av, Pv) = _bsr_plan(A, P, **kw)
    C = plan.numeric(Av, Pv)
    rp, col = plan.pattern()
    torch.cuda.synchronize()
    st = plan.stats()
    out = gen.BSR(P.mb, P.mb, A.bs, rp.cpu().numpy(), col.cpu().numpy(),
                  C.cpu().numpy().reshape(-1, A.bs, A.bs))
    plan.close()
    return out, st


def _check_bsr(A, P, **kw):
    Cb, st = _gpu_bsr(A, P, **kw)
    ref = oracle.ptap(gen.bsr_to_csr(A), gen.bsr_to_csr(P))
    Cs = gen.bsr_to_csr(Cb)
    assert np.array_equal(Cs.rowptr, ref.rowptr), "expanded C row pointers differ from the oracle"
    assert np.array_equal(Cs.col, ref.col), "expanded C columns differ from the oracle"
    assert_close(Cs.val, ref.val, ref.abs)
    assert st["block_size"] == A.bs
    return st


@gpu
def test_block_stencil_reduced():
    """4x4-block anisotropic 27-point operator on 6^3 nodes, block smoothed aggregation."""
    _need_gpu()
    A = gen.block_stencil27(6, 4, seed=2)
    P = gen.block_smoothed_aggregation(A, 6, 4)
    _check_bsr(gen.csr_to_bsr(A, 4), gen.csr_to_bsr(P, 4))


@gpu
@pytest.mark.parametrize("bs", [1, 2, 3, 4, 5, 8])
@pytest.mark.parametrize("seed", [0, 1])
def test_random_blocks(bs, seed):
    """Random block patterns with empty rows, every block size the kernel instantiates."""
    _need_gpu()
    rng = np.random.default_rng(40 + seed)
    nb = int(rng.integers(20, 120))
    mb = int(rng.integers(5, 30))
    A = gen.random_bsr(nb, nb, bs, float(rng.uniform(0.02, 0.08)), seed=seed, empty_rows=0.1)
    P = gen.random_bsr(nb, mb, bs, float(rng.uniform(0.05, 0.2)), seed=100 + seed, empty_rows=0.1)
    _check_bsr(A, P)


@gpu
def test_long_rows_accumulate_in_device_memory():
    """8x8 blocks with dense coupling: rows of C longer than the LDS accumulator take the
    device-atomic path; both paths must agree with the oracle."""
    _need_gpu()
    A = gen.random_bsr(150, 150, 8, 0.25, seed=5)
    P = gen.random_bsr(150, 160, 8, 0.3, seed=6)
    _check_bsr(A, P)


@gpu
@pytest.mark.parametrize("nb,mb,da,dp,seed", [(100, 30, 0.5, 0.2, 11), (60, 380, 0.6, 0.15, 12)])
def test_block4_long_rows(nb, mb, da, dp, seed):
    """4x4 blocks with rows of A longer than the 32 entries whose blocks the 4x4 kernel stages
    at a time (several chunks per fine row); the second case also has rows of C longer than the
    LDS accumulator, which take the device-atomic path."""
    _need_gpu()
    A = gen.random_bsr(nb, nb, 4, da, seed=seed, empty_rows=0.05)
    P = gen.random_bsr(nb, mb, 4, dp, seed=50 + seed, empty_rows=0.05)
    assert np.diff(A.rowptr).max() > 32
    _check_bsr(A, P)


@gpu
def test_block4_chunk_and_batch_boundaries():
    """4x4 blocks, rows of A with exactly 0, 1, 31, 32, 33, 64 and 65 blocks (the 4x4 kernel
    stages 32 entries of A(I,:) at a time) and rows of P that are empty or up to 12 blocks long,
    so that segments of the product walk are empty, end exactly at a 32-product batch or cross
    one."""
    _need_gpu()
    rng = np.random.default_rng(77)
    nb, mb = 140, 24
    lens = np.array([0, 1, 31, 32, 33, 64, 65])[np.arange(nb) % 7]
    rowptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.concatenate([np.sort(rng.choice(nb, size=k, replace=False)) for k in lens]).astype(np.int64)
    A = gen.BSR(nb, nb, 4, rowptr, col, rng.uniform(-1.0, 1.0, size=(len(col), 4, 4)))
    plens = rng.integers(0, 13, size=nb)
    plens[rng.random(nb) < 0.2] = 0
    prow = np.concatenate([[0], np.cumsum(plens)]).astype(np.int64)
    pcol = np.concatenate([np.sort(rng.choice(mb, size=k, replace=False)) for k in plens]).astype(np.int64)
    P = gen.BSR(nb, mb, 4, prow, pcol, rng.uniform(-1.0, 1.0, size=(len(pcol), 4, 4)))
    _check_bsr(A, P)


@gpu
def test_block_plan_errors_and_repeat():
    _need_gpu()
    import paper_1905_08423_amd as lib
    A = gen.random_bsr(30, 30, 2, 0.1, seed=8)
    P = gen.random_bsr(30, 10, 2, 0.2, seed=9)
    for bad in (0, 9):
        with pytest.raises(lib.PtapError) as e:
            plan, _ = _bsr_plan(gen.BSR(A.nb, A.nb, bad, A.rowptr, A.col, A.val),
                                gen.BSR(P.nb, P.mb, bad, P.rowptr, P.col, P.val))
        assert e.value.status == lib.PTAP_ERR_INPUT
    with pytest.raises(lib.PtapError) as e:
        _bsr_plan(A, P, algo="twostep")
    assert e.value.status == lib.PTAP_ERR_UNSUPPORTED
    with pytest.raises(lib.PtapError) as e:
        _bsr_plan(A, P, backward=True)
    assert e.value.status == lib.PTAP_ERR_UNSUPPORTED
    # one symbolic, numerics with new values; value arrays of the wrong size are refused
    plan, (Av, Pv) = _bsr_plan(A, P)
    rng = np.random.default_rng(2)
    for _ in range(2):
        A.val[:] = rng.uniform(-1, 1, A.val.shape)
        P.val[:] = rng.uniform(-1, 1, P.val.shape)
        Av.copy_(torch.from_numpy(A.val.reshape(-1)))
        Pv.copy_(torch.from_numpy(P.val.reshape(-1)))
        C = plan.numeric(Av, Pv).cpu().numpy()
        ref = oracle.ptap(gen.bsr_to_csr(A), gen.bsr_to_csr(P))
        rp, col = plan.pattern()
        Cs = gen.bsr_to_csr(gen.BSR(P.mb, P.mb, 2, rp.cpu().numpy(), col.cpu().numpy(), C.reshape(-1, 2, 2)))
        assert np.array_equal(Cs.col, ref.col)
        assert_close(Cs.val, ref.val, ref.abs)
    with pytest.raises(ValueError):
        plan.numeric(Av[:-1], Pv)
    plan.close()


@gpu
@pytest.mark.slow
def test_block_full_size_sampled():
    """The 4x4-block workload at full size (96^3 nodes, 3.5 M scalar rows): 2000 sampled block
    rows of C against the oracle's rows (computed one by one on the scalar expansion)."""
    _need_gpu()
    A, P, _ = gen.galerkin_workload("c3c")
    Ab, Pb = gen.csr_to_bsr(A, 4), gen.csr_to_bsr(P, 4)
    Cb, st = _gpu_bsr(Ab, Pb)
    assert Cb.nnzb * 16 == 13_289_344
    brows = np.sort(np.random.default_rng(7).choice(Pb.mb, 500, replace=False))
    rows = (brows[:, None] * 4 + np.arange(4)[None, :]).ravel().astype(np.int32)
    ref = oracle.ptap(A, P, rows=rows)
    got_cols, got_vals = [], []
    for bi in brows:
        for g in range(4):
            ks = range(Cb.rowptr[bi], Cb.rowptr[bi + 1])
            got_cols.append(np.concatenate([Cb.col[k] * 4 + np.arange(4) for k in ks]))
            got_vals.append(np.concatenate([Cb.val[k, g, :] for k in ks]))
    got_cols, got_vals = np.concatenate(got_cols), np.concatenate(got_vals)
    assert np.array_equal(got_cols, ref.col), "sampled rows: columns differ from the oracle"
    assert_close(got_vals, ref.val, ref.abs)
