"""The oracle's pins must catch plausible mistakes.

Each case copies the oracle source, plants one mistake (a dropped factor, a wrong index, a
transposed operand, a lost term, a flipped sign), builds the copy with gcc into a temporary
directory, and checks that at least one pin from test_oracle.py fails against it.  Nothing
here touches the GPU."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import ptap_inputs as gen
from helpers import close_mask, dense, dense_pattern

SRC = os.path.join(os.path.dirname(oracle.__file__), "ptap_oracle.c")

MUTATIONS = {
    "drop_left_weight": ("acc[j] += w * (a * p);", "acc[j] += (a * p);"),
    "square_right_weight": ("acc[j] += w * (a * p);", "acc[j] += w * (a * w);"),
    "transpose_A": ("int32_t J = A_col[ka];\n        double a = pattern_only ? 0.0 : A_val[ka];",
                    "int32_t J = I; double a = pattern_only ? 0.0 : A_val[ka]; (void)A_col;"),
    "skip_last_P_entry": ("for (int32_t kp = Q2_rowptr[J]; kp < Q2_rowptr[J + 1]; ++kp) {\n          int32_t j = Q2_col[kp];\n          if (!mark[j])",
                          "for (int32_t kp = Q2_rowptr[J]; kp < Q2_rowptr[J + 1] - 1; ++kp) {\n          int32_t j = Q2_col[kp];\n          if (!mark[j])"),
    "backward_drop_second_term": ("dP[kk] += s;", "dP[kk] += 0.0 * s;"),
    "backward_sign_second_term": ("dP[kk] += s;", "dP[kk] -= s;"),
    "backward_transpose_W_in_dA": ("s += P_val[ki] * w_at(C_rowptr, C_col, W, i, j) * P_val[kj];",
                                   "s += P_val[ki] * w_at(C_rowptr, C_col, W, j, i) * P_val[kj];"),
    # the long-double mode: a term rounded to double before it is added
    "modes_long_double_rounds_terms": (
        "accl[j] += (long double)w * ((long double)a * (long double)p);",
        "accl[j] += (double)((long double)w * ((long double)a * (long double)p));"),
    # the threaded mode: the last range of rows loses its last row to the next-to-last range
    "modes_thread_ranges_shifted": (
        "parts[k].r0 = (int32_t)(((int64_t)nrows_out * k) / nthreads);",
        "parts[k].r0 = (int32_t)(((int64_t)nrows_out * k) / nthreads) + (k == nthreads - 1 && k > 0);"),
}


def _build_mutant(tmp_path, name):
    old, new = MUTATIONS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, name
    src = tmp_path / f"{name}.c"
    src.write_text(text.replace(old, new))
    lib = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", str(lib), str(src), "-lm"],
                   check=True)
    return str(lib)


def _forward_pins_pass():
    """A compact subset of the forward pins: dense products on a non-symmetric random case and
    the bit-exact Kronecker form.  Returns True when all of them pass."""
    A = gen.random_csr(20, 20, 0.25, seed=1, empty_rows=0.1)
    P = gen.random_csr(20, 6, 0.35, seed=2, empty_rows=0.1)
    C = oracle.ptap(A, P)
    brute = (dense_pattern(P).astype(int).T @ dense_pattern(A).astype(int) @ dense_pattern(P).astype(int)) > 0
    got = np.zeros_like(brute)
    for i in range(P.n_cols):
        got[i, C.col[C.rowptr[i]:C.rowptr[i + 1]]] = True
    if not np.array_equal(got, brute):
        return False
    Ad, Pd = dense(A), dense(P)
    ref = (Pd.T @ Ad @ Pd)[got]
    bound = (np.abs(Pd).T @ np.abs(Ad) @ np.abs(Pd))[got]
    if not close_mask(C.val, ref, bound).all():
        return False
    p = gen.trilinear_1d(9).toarray()
    L = np.diag(np.full(9, 2.0)) - np.diag(np.ones(8), 1) - np.diag(np.ones(8), -1)
    T, M = p.T @ L @ p, p.T @ p
    kref = np.kron(T, np.kron(M, M)) + np.kron(M, np.kron(T, M)) + np.kron(M, np.kron(M, T))
    C = oracle.ptap(gen.laplacian7(9), gen.trilinear(9))
    D = np.zeros_like(kref)
    for i in range(kref.shape[0]):
        D[i, C.col[C.rowptr[i]:C.rowptr[i + 1]]] = C.val[C.rowptr[i]:C.rowptr[i + 1]]
    return np.array_equal(D, kref)


def _backward_pins_pass():
    A = gen.random_csr(24, 24, 0.2, seed=5, empty_rows=0.1)
    P = gen.random_csr(24, 7, 0.3, seed=6, empty_rows=0.1)
    C = oracle.ptap(A, P, pattern_only=True)
    W = gen.loss_weights(C.nnz, seed=5)
    dA, dP = oracle.ptap_backward(A, P, C.rowptr, C.col, W)
    Wd = np.zeros((P.n_cols, P.n_cols))
    for i in range(P.n_cols):
        Wd[i, C.col[C.rowptr[i]:C.rowptr[i + 1]]] = W[C.rowptr[i]:C.rowptr[i + 1]]
    Ad, Pd = dense(A), dense(P)
    gA = (Pd @ Wd @ Pd.T)[dense_pattern(A)]
    gP = (Ad @ Pd @ Wd.T + Ad.T @ Pd @ Wd)[dense_pattern(P)]
    bA = (np.abs(Pd) @ np.abs(Wd) @ np.abs(Pd).T)[dense_pattern(A)]
    bP = (np.abs(Ad) @ np.abs(Pd) @ np.abs(Wd).T + np.abs(Ad).T @ np.abs(Pd) @ np.abs(Wd))[dense_pattern(P)]
    return bool(close_mask(dA, gA, bA).all() and close_mask(dP, gP, bP).all())


def _modes_pins_pass():
    """The pins of the long-double and threaded modes (tests/test_oracle_modes.py)."""
    import test_oracle_modes as tm

    try:
        tm.test_long_double_is_exact_sum_correctly_rounded(21)
        tm.test_threads_bit_identical("stencil27_lognormal_24", 3)
    except AssertionError:
        return False
    return True


def test_unmutated_oracle_passes_the_subset():
    assert _forward_pins_pass()
    assert _backward_pins_pass()
    assert _modes_pins_pass()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(tmp_path, name):
    lib = _build_mutant(tmp_path, name)
    with oracle.use_library(lib):
        if name.startswith("backward"):
            caught = not _backward_pins_pass()
        elif name.startswith("modes"):
            caught = not _modes_pins_pass()
        else:
            caught = not _forward_pins_pass()
    assert caught, f"planted mistake {name} was not caught"
