"""Helpers for the GPU parity tests: run the HIP library through its C ABI binding and compare
with the CPU oracle."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import paper_1905_08423_amd as lib
from helpers import assert_close


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


class GpuProblem:
    """A and P resident on the device."""

    def __init__(self, A, P):
        self.A, self.P = A, P
        self.A_rowptr = dev(A.rowptr, torch.int32)
        self.A_col = dev(A.col, torch.int32)
        self.A_val = dev(A.val, torch.float64)
        self.P_rowptr = dev(P.rowptr, torch.int32)
        self.P_col = dev(P.col, torch.int32)
        self.P_val = dev(P.val, torch.float64)

    def plan(self, **kw):
        return lib.Plan(self.A.n_rows, self.P.n_cols, self.A_rowptr, self.A_col, self.P_rowptr,
                        self.P_col, **kw)


def run(A, P, **kw):
    """(rowptr, col, val, stats) of C from the GPU library."""
    g = GpuProblem(A, P)
    plan = g.plan(**kw)
    C = plan.numeric(g.A_val, g.P_val)
    rp, col = plan.pattern()
    torch.cuda.synchronize()
    out = (rp.cpu().numpy(), col.cpu().numpy(), C.cpu().numpy(), plan.stats())
    plan.close()
    return out


def check_against_oracle(A, P, ref=None, exact=False, **kw):
    rp, col, val, stats = run(A, P, **kw)
    ref = ref if ref is not None else oracle.ptap(A, P)
    assert np.array_equal(rp, ref.rowptr), "C row pointers differ from the oracle"
    assert np.array_equal(col, ref.col), "C column indices differ from the oracle"
    if exact:
        assert np.array_equal(val, ref.val), f"values not bit-exact: max diff {np.abs(val - ref.val).max()}"
    else:
        assert_close(val, ref.val, ref.abs)
    return stats
