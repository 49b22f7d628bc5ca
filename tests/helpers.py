"""Shared test helpers: the FP64 acceptance criterion and small dense utilities."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# Acceptance criterion for an FP64 entry (i, j) of C against the oracle:
#   |got - ref| <= max(REL * |ref|, ABS_FRAC * Cabs(i, j)),  Cabs = |P|^T |A| |P|.
# REL is the per-entry relative tolerance.  Where a sum cancels heavily, two valid summation
# orders already differ by more than REL relative; there the forward-error bound of recursive
# summation, a small multiple of the unit roundoff times the sum of the term magnitudes,
# governs instead (ABS_FRAC = 1e-14 is about 90 unit roundoffs).
REL = 1e-12
ABS_FRAC = 1e-14


def close_mask(got, ref, ref_abs, rel=REL, abs_frac=ABS_FRAC):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(got - ref)
    return (err <= rel * np.abs(ref)) | (err <= abs_frac * np.asarray(ref_abs))


def assert_close(got, ref, ref_abs, what="values", rel=REL, abs_frac=ABS_FRAC):
    ok = close_mask(got, ref, ref_abs, rel, abs_frac)
    if not ok.all():
        bad = np.flatnonzero(~ok)[:8]
        raise AssertionError(
            f"{what}: {int((~ok).sum())} of {ok.size} entries outside tolerance; first {bad.tolist()}: "
            f"got {np.asarray(got)[bad].tolist()} ref {np.asarray(ref)[bad].tolist()} "
            f"abs {np.asarray(ref_abs)[bad].tolist()}")


def strict_report(got, ref):
    """Count of entries beyond the plain 1e-12 relative criterion and the worst relative error
    (an entry whose reference is exactly 0 counts as infinitely far off unless it is 0 too)."""
    got = np.asarray(got); ref = np.asarray(ref)
    err = np.abs(got - ref)
    rel = np.where(ref != 0, err / np.where(ref != 0, np.abs(ref), 1.0), np.where(err > 0, np.inf, 0.0))
    return int((rel > REL).sum()), float(rel.max() if rel.size else 0.0)


def parity_report(name, got, ref, ref_ld=None):
    """One line on how a result compares with the oracle under the plain 1e-12 relative test,
    beside the criterion the tests apply: entries beyond 1e-12 relative, the worst relative error,
    the worst error as a fraction of |P|^T |A| |P| (the criterion's second bound), and the same
    against the oracle's long-double sums when given.  Printed (run pytest with -s to see it) and
    returned as a dict."""
    got = np.asarray(got, dtype=np.float64)
    n, worst = strict_report(got, ref.val)
    frac = float((np.abs(got - ref.val) / np.where(ref.abs > 0, ref.abs, 1.0)).max()) if got.size else 0.0
    out = {"entries": int(got.size), "beyond_1e-12": n, "max_rel": worst, "max_err_over_Cabs": frac}
    if ref_ld is not None:
        n2, w2 = strict_report(got, ref_ld.val)
        n3, w3 = strict_report(ref.val, ref_ld.val)
        out.update({"beyond_1e-12_vs_long_double": n2, "max_rel_vs_long_double": w2,
                    "oracle_fp64_beyond_1e-12_vs_long_double": n3, "oracle_fp64_max_rel_vs_long_double": w3})
    print(f"PARITY {name}: " + ", ".join(f"{k}={v:.3g}" if isinstance(v, float) else f"{k}={v}"
                                         for k, v in out.items()))
    return out


def dense(M) -> np.ndarray:
    D = np.zeros((M.n_rows, M.n_cols))
    for r in range(M.n_rows):
        for k in range(M.rowptr[r], M.rowptr[r + 1]):
            D[r, M.col[k]] = M.val[k]
    return D


def dense_pattern(M) -> np.ndarray:
    D = np.zeros((M.n_rows, M.n_cols), dtype=bool)
    for r in range(M.n_rows):
        D[r, M.col[M.rowptr[r]:M.rowptr[r + 1]]] = True
    return D


def ones_like_csr(M) -> sp.csr_matrix:
    """The pattern of M as a scipy matrix of ones (no value can cancel)."""
    return sp.csr_matrix((np.ones(M.nnz), M.col, M.rowptr), shape=(M.n_rows, M.n_cols))


def scipy_csr(M) -> sp.csr_matrix:
    return sp.csr_matrix((M.val, M.col, M.rowptr), shape=(M.n_rows, M.n_cols))


def rows_of(rowptr, col):
    return [col[rowptr[i]:rowptr[i + 1]].tolist() for i in range(len(rowptr) - 1)]


def read_golden_sections(path):
    out, cur = {}, None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                out[cur] = []
            else:
                out[cur].append([int(t) for t in line.split()])
    return out
