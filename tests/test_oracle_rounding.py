"""The oracle's own FP64 rounding at the full workload sizes, against its long-double mode.

Section 3's Eq. allatonce fixes C = P^T A P exactly; any summation order is a valid FP64
evaluation of it, so the oracle is not the exact C either.  The long-double mode (64-bit
significand, one rounding per entry at the end) shows how far the FP64 sums are from the exact
ones: every entry must stay within the forward-error bound the parity criterion uses
(1e-14 |P|^T |A| |P|, about 90 unit roundoffs of the sum of term magnitudes), and the number of
entries the FP64 oracle itself puts beyond 1e-12 relative is reported.  Those entries are the
cancelling sums for which a strict 1e-12 per-entry test would reject a correct result; the GPU
parity tests print the same counts for the library (tests/helpers.py parity_report)."""
import numpy as np
import pytest

import oracle
import ptap_inputs as gen
from helpers import ABS_FRAC, close_mask, parity_report


@pytest.mark.parametrize("name", ["c2", "c3b"])
def test_fp64_oracle_against_long_double(name):
    A, P, _ = gen.galerkin_workload(name)
    t = oracle.cores()
    fp = oracle.ptap(A, P, threads=t)
    ld = oracle.ptap(A, P, long_double=True, threads=t)
    assert np.array_equal(fp.rowptr, ld.rowptr) and np.array_equal(fp.col, ld.col)
    assert np.array_equal(fp.abs, ld.abs)  # magnitudes are summed in FP64 in both modes
    assert close_mask(fp.val, ld.val, ld.abs, rel=0.0, abs_frac=ABS_FRAC).all()
    rep = parity_report(f"oracle_fp64_vs_long_double_{name}", fp.val, ld)
    # the FP64 sums stay well inside the criterion's bound (a few unit roundoffs of the sum of
    # magnitudes), while some entries are beyond 1e-12 relative: cancelling sums
    assert rep["max_err_over_Cabs"] < ABS_FRAC / 2
    assert rep["beyond_1e-12"] > 0
