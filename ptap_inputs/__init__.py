"""Seeded synthetic inputs for the triple product C = P^T A P.

This module builds the fine operators A and interpolations P that both the
CPU oracle and the GPU library consume.  It holds none of the triple
product's arithmetic: it only assembles stencil matrices on structured grids,
trilinear and smoothed-aggregation interpolations, and small random CSR
matrices for edge cases.  Every array is returned in the CSR layout the
library takes (int32 row pointers and column indices, sorted and unique
within each row, float64 values).

Grid numbering is lexicographic with x fastest: index = x + nx*(y + ny*z).

The shapes follow the paper's workloads (Section 4.1: a structured 3D grid,
one unknown per point, linear interpolation with 2x coarsening per dimension;
Section 4.2: algebraic interpolations whose rows have 0..12 entries and
coarse operators whose rows have up to a few hundred entries).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

__all__ = [
    "CSR", "laplacian7", "stencil27", "trilinear_1d", "trilinear", "coarse_side",
    "smoothed_aggregation", "block_stencil27", "block_smoothed_aggregation",
    "random_csr", "toy_rowwise", "galerkin_workload", "batch_problem_sides",
    "hierarchy_sides", "loss_weights", "to_scipy", "from_scipy", "BSR", "csr_to_bsr", "bsr_to_csr",
    "random_bsr",
]


@dataclass
class CSR:
    """A compressed-sparse-row matrix with int32 indices and float64 values."""

    n_rows: int
    n_cols: int
    rowptr: np.ndarray  # int32 [n_rows + 1]
    col: np.ndarray     # int32 [nnz], sorted and unique within each row
    val: np.ndarray     # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def check(self) -> None:
        """Raise ValueError unless the arrays form a well-formed CSR matrix."""
        rp, c = self.rowptr, self.col
        if rp.dtype != np.int32 or c.dtype != np.int32 or self.val.dtype != np.float64:
            raise ValueError("dtype")
        if rp.shape != (self.n_rows + 1,) or rp[0] != 0 or c.shape != (rp[-1],) or self.val.shape != c.shape:
            raise ValueError("shape")
        if np.any(np.diff(rp) < 0):
            raise ValueError("rowptr not monotone")
        if c.size:
            if c.min() < 0 or c.max() >= self.n_cols:
                raise ValueError("column out of range")
            d = np.diff(c.astype(np.int64))
            row_start = np.zeros(c.size, dtype=bool)
            starts = rp[:-1][np.diff(rp) > 0]
            row_start[starts] = True
            if np.any(d[~row_start[1:]] <= 0):
                raise ValueError("columns not strictly increasing within a row")

    def digest(self) -> str:
        """SHA-256 over the raw bytes of the three arrays and the shape."""
        h = hashlib.sha256()
        h.update(np.array([self.n_rows, self.n_cols], dtype=np.int64).tobytes())
        for a in (self.rowptr, self.col, self.val):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()

    def with_values(self, val: np.ndarray) -> "CSR":
        return CSR(self.n_rows, self.n_cols, self.rowptr, self.col, np.ascontiguousarray(val, dtype=np.float64))


def to_scipy(M: CSR) -> sp.csr_matrix:
    return sp.csr_matrix((M.val, M.col, M.rowptr), shape=(M.n_rows, M.n_cols))


def from_scipy(M) -> CSR:
    M = sp.csr_matrix(M)
    M.sum_duplicates()
    M.sort_indices()
    return CSR(M.shape[0], M.shape[1], M.indptr.astype(np.int32), M.indices.astype(np.int32),
               M.data.astype(np.float64))


def _check_int32(nnz: int) -> None:
    if nnz >= 2**31:
        raise ValueError("matrix too large for int32 indices")


# --------------------------------------------------------------------------------------------
# Stencil operators on a structured grid
# --------------------------------------------------------------------------------------------

def _offsets(points: int):
    """Stencil offsets (dx, dy, dz) in an order that makes columns ascending within a row."""
    if points == 7:
        return [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    if points == 27:
        return [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    raise ValueError(points)


def _assemble(nx: int, ny: int, nz: int, points: int, offdiag, diag) -> CSR:
    """Assemble a stencil matrix row by row.

    offdiag(idx, nbr, (dx,dy,dz)) -> values of the coupling idx->nbr (only called for in-grid nbr);
    diag(idx, valid_masks) -> diagonal values.
    """
    n = nx * ny * nz
    offs = _offsets(points)
    idx = np.arange(n, dtype=np.int64)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    cols = np.empty((n, points), dtype=np.int32)
    vals = np.empty((n, points), dtype=np.float64)
    mask = np.empty((n, points), dtype=bool)
    valid_list = []
    for s, (dx, dy, dz) in enumerate(offs):
        ok = ((x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny) & (z + dz >= 0) & (z + dz < nz))
        mask[:, s] = ok
        nbr = idx + dx + nx * (dy + ny * dz)
        cols[:, s] = np.where(ok, nbr, 0)
        if (dx, dy, dz) == (0, 0, 0):
            center = s
            vals[:, s] = 0.0
        else:
            v = np.zeros(n)
            v[ok] = offdiag(idx[ok], nbr[ok], (dx, dy, dz))
            vals[:, s] = v
            valid_list.append(((dx, dy, dz), ok))
    vals[:, center] = diag(idx, valid_list)
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    _check_int32(int(rowptr[-1]))
    return CSR(n, n, rowptr.astype(np.int32), cols[mask], vals[mask])


def laplacian7(nx: int, ny: int | None = None, nz: int | None = None) -> CSR:
    """3D 7-point Laplacian with Dirichlet boundaries: diagonal 6, off-diagonal -1.

    Out-of-grid neighbours are dropped; the diagonal stays 6 everywhere.
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return _assemble(nx, ny, nz, 7, lambda i, j, d: -1.0, lambda i, valid: 6.0)


def stencil27(nx: int, ny: int | None = None, nz: int | None = None, *, seed: int | None = None,
              eps_z: float = 1.0) -> CSR:
    """3D 27-point operator with per-cell coefficients.

    With seed=None every coefficient is 1, giving diagonal 26 and off-diagonal -1.
    Otherwise k_i ~ lognormal(0, 1) per grid point (numpy default_rng(seed)) and
      A(i,j) = -w(d) * (k_i + k_j) / 2 for each in-grid neighbour j,
      A(i,i) = sum over the 26 stencil slots of w(d) * (k_i + k_j*) / 2, with k_j* = k_i out of grid,
    where w(d) = eps_z for offsets with a z component and 1 otherwise.  A is symmetric.
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    n = nx * ny * nz
    k = np.ones(n) if seed is None else np.random.default_rng(seed).lognormal(0.0, 1.0, size=n)

    def w(d):
        return eps_z if d[2] != 0 else 1.0

    def off(i, j, d):
        return -w(d) * 0.5 * (k[i] + k[j])

    def diag(idx, valid_list):
        s = np.zeros(n)
        for d, ok in valid_list:
            nbr = idx + d[0] + nx * (d[1] + ny * d[2])
            kj = np.where(ok, k[np.where(ok, nbr, 0)], k)
            s += w(d) * 0.5 * (k + kj)
        return s

    return _assemble(nx, ny, nz, 27, off, diag)


# --------------------------------------------------------------------------------------------
# Interpolations
# --------------------------------------------------------------------------------------------

def coarse_side(nf: int) -> int:
    """Coarse points per dimension for vertex-centred 2x coarsening: ceil(nf / 2).

    Odd sides reproduce n_f = 2 n_c - 1 exactly (the paper's model problem, Section 4.1)."""
    return (nf + 1) // 2


def trilinear_1d(nf: int) -> sp.csr_matrix:
    """1D linear interpolation from ceil(nf/2) coarse points to nf fine points.

    Coarse point c sits at fine point 2c.  An even fine point f takes (f/2, 1); an odd fine
    point takes ((f-1)/2, 1/2) and ((f+1)/2, 1/2), dropping coarse indices beyond the last
    point (homogeneous Dirichlet value there)."""
    nc = coarse_side(nf)
    rows, cols, vals = [], [], []
    for f in range(nf):
        if f % 2 == 0:
            rows.append(f); cols.append(f // 2); vals.append(1.0)
        else:
            for c in ((f - 1) // 2, (f + 1) // 2):
                if c < nc:
                    rows.append(f); cols.append(c); vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def trilinear(nx: int, ny: int | None = None, nz: int | None = None) -> CSR:
    """Trilinear interpolation P = p_z (x) p_y (x) p_x with weights 1, 1/2, 1/4, 1/8."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    P = sp.kron(trilinear_1d(nz), sp.kron(trilinear_1d(ny), trilinear_1d(nx), format="csr"), format="csr")
    return from_scipy(P)


def _aggregates(nx: int, ny: int, nz: int, a: int) -> tuple[np.ndarray, int, tuple[int, int, int]]:
    n = nx * ny * nz
    idx = np.arange(n)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    cx, cy, cz = -(-nx // a), -(-ny // a), -(-nz // a)
    agg = (x // a) + cx * ((y // a) + cy * (z // a))
    return agg, cx * cy * cz, (cx, cy, cz)


def smoothed_aggregation(A: CSR, nx: int, ny: int, nz: int, *, agg: int = 3, steps: int = 1,
                         omega: float = 2.0 / 3.0) -> CSR:
    """Smoothed-aggregation interpolation: tentative P = 1 on each node's agg^3 aggregate,
    followed by `steps` damped-Jacobi smoothing steps P <- (I - omega D^-1 A) P, D = diag(A)."""
    aggs, m, _ = _aggregates(nx, ny, nz, agg)
    n = A.n_rows
    T = sp.csr_matrix((np.ones(n), (np.arange(n), aggs)), shape=(n, m))
    As = to_scipy(A)
    Dinv = sp.diags(1.0 / As.diagonal())
    S = sp.identity(n, format="csr") - omega * (Dinv @ As)
    P = T
    for _ in range(steps):
        P = S @ P
    P = sp.csr_matrix(P)
    P.eliminate_zeros()
    return from_scipy(P)


def block_stencil27(nx: int, G: int, *, seed: int, eps_z: float = 0.01) -> CSR:
    """Block variant of the anisotropic 27-point operator with G coupled components per node,
    expanded to scalar CSR (row = node*G + g).

    Off-diagonal node blocks B_ij = w(d) (k_i + k_j)/2 * U_ij with U uniform in [-1, 1] and
    B_ji = B_ij^T.  Diagonal block: symmetric uniform [-1, 1] whose diagonal is raised to the
    absolute row sum of all other entries of its scalar row plus 1 (dominant diagonal)."""
    rng = np.random.default_rng(seed)
    nn = nx ** 3
    k = rng.lognormal(0.0, 1.0, size=nn)
    idx = np.arange(nn, dtype=np.int64)
    x, y, z = idx % nx, (idx // nx) % nx, idx // (nx * nx)
    offs = _offsets(27)
    # Couplings for "forward" offsets only; backward ones are the transposed blocks.
    fwd = [d for d in offs if (d[2], d[1], d[0]) > (0, 0, 0)]
    blocks = {}
    for d in fwd:
        ok = ((x + d[0] >= 0) & (x + d[0] < nx) & (y + d[1] >= 0) & (y + d[1] < nx) & (z + d[2] >= 0) & (z + d[2] < nx))
        i = idx[ok]
        j = i + d[0] + nx * (d[1] + nx * d[2])
        w = eps_z if d[2] != 0 else 1.0
        U = rng.uniform(-1.0, 1.0, size=(i.size, G, G))
        blocks[d] = (i, j, (w * 0.5 * (k[i] + k[j]))[:, None, None] * U)
    D = rng.uniform(-1.0, 1.0, size=(nn, G, G))
    D = 0.5 * (D + D.transpose(0, 2, 1))
    rows, cols, vals = [], [], []
    gg = np.arange(G)
    for d, (i, j, B) in blocks.items():
        for (ri, rj, M) in ((i, j, B), (j, i, B.transpose(0, 2, 1))):
            r = (ri[:, None, None] * G + gg[None, :, None]).repeat(G, axis=2)
            c = (rj[:, None, None] * G + gg[None, None, :]).repeat(G, axis=1)
            rows.append(r.ravel()); cols.append(c.ravel()); vals.append(M.ravel())
    offsum = np.zeros(nn * G)
    for r, v in zip(rows, vals):
        np.add.at(offsum, r, np.abs(v))
    Dd = D.copy()
    diag_idx = np.arange(G)
    Dd[:, diag_idx, diag_idx] = 0.0
    offsum += np.abs(Dd).sum(axis=2).ravel()
    Dd[:, diag_idx, diag_idx] = (offsum + 1.0).reshape(nn, G)
    r = (idx[:, None, None] * G + gg[None, :, None]).repeat(G, axis=2)
    c = (idx[:, None, None] * G + gg[None, None, :]).repeat(G, axis=1)
    rows.append(r.ravel()); cols.append(c.ravel()); vals.append(Dd.ravel())
    M = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nn * G, nn * G))
    return from_scipy(M)


def block_smoothed_aggregation(A: CSR, nx: int, G: int, *, agg: int = 3, steps: int = 1,
                               omega: float = 2.0 / 3.0) -> CSR:
    """Block tentative interpolation (identity per component on each aggregate, coarse dof
    = aggregate*G + g) followed by damped-Jacobi smoothing with the pointwise diagonal."""
    aggs, m, _ = _aggregates(nx, nx, nx, agg)
    nn = nx ** 3
    rows = np.arange(nn * G)
    cols = aggs.repeat(G) * G + np.tile(np.arange(G), nn)
    T = sp.csr_matrix((np.ones(nn * G), (rows, cols)), shape=(nn * G, m * G))
    As = to_scipy(A)
    S = sp.identity(nn * G, format="csr") - omega * (sp.diags(1.0 / As.diagonal()) @ As)
    P = T
    for _ in range(steps):
        P = S @ P
    P = sp.csr_matrix(P)
    P.eliminate_zeros()
    return from_scipy(P)


# --------------------------------------------------------------------------------------------
# Block-sparse (BSR) layout: dense bs x bs blocks on a block pattern
# --------------------------------------------------------------------------------------------

@dataclass
class BSR:
    """Block CSR: nb x mb blocks of bs x bs; val[k] is block k, row-major (nnzb x bs x bs)."""

    nb: int
    mb: int
    bs: int
    rowptr: np.ndarray  # int32 [nb + 1]
    col: np.ndarray     # int32 [nnzb], sorted and unique within each block row
    val: np.ndarray     # float64 [nnzb, bs, bs]

    @property
    def nnzb(self) -> int:
        return int(self.rowptr[-1])


def csr_to_bsr(M: CSR, bs: int) -> BSR:
    """The block layout of a scalar CSR matrix whose stored entries fill whole bs x bs blocks
    (row = node*bs + g).  In such a matrix the bs scalar rows of block row bi hold the same
    block columns, bs consecutive entries per block.  Raises ValueError otherwise."""
    if M.n_rows % bs or M.n_cols % bs:
        raise ValueError("shape is not a multiple of the block size")
    nb, mb = M.n_rows // bs, M.n_cols // bs
    rp = M.rowptr.astype(np.int64)
    lens = np.diff(rp).reshape(nb, bs)
    if np.any(lens % bs) or np.any(lens != lens[:, :1]):
        raise ValueError("a block of the pattern is not complete")
    nblk = lens[:, 0] // bs
    browptr = np.concatenate([[0], np.cumsum(nblk)]).astype(np.int64)
    nnzb = int(browptr[-1])
    bi = np.repeat(np.arange(nb), nblk)
    q = np.arange(nnzb) - browptr[bi]
    g = np.arange(bs)
    # start of block k's row g in the scalar arrays, then its bs consecutive entries
    base = rp[bi[:, None] * bs + g[None, :]] + q[:, None] * bs
    idx = base[:, :, None] + g[None, None, :]
    cols = M.col[idx]
    bcol = cols[:, 0, 0] // bs
    if np.any(cols != bcol[:, None, None] * bs + g[None, None, :]):
        raise ValueError("a block of the pattern is not complete")
    return BSR(nb, mb, bs, browptr.astype(np.int32), bcol.astype(np.int32),
               np.ascontiguousarray(M.val[idx], dtype=np.float64))


def bsr_to_csr(B: BSR) -> CSR:
    """Scalar CSR expansion of a BSR matrix (every entry of every stored block is stored)."""
    bs = B.bs
    brow = np.repeat(np.arange(B.nb), np.diff(B.rowptr))
    g = np.arange(bs)
    rows = (brow[:, None, None] * bs + g[None, :, None]).repeat(bs, axis=2)
    cols = (B.col[:, None, None].astype(np.int64) * bs + g[None, None, :]).repeat(bs, axis=1)
    order = np.lexsort((cols.ravel(), rows.ravel()))
    r, c, v = rows.ravel()[order], cols.ravel()[order], B.val.reshape(-1)[order]
    rowptr = np.zeros(B.nb * bs + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    return CSR(B.nb * bs, B.mb * bs, np.cumsum(rowptr).astype(np.int32), c.astype(np.int32),
               np.ascontiguousarray(v, dtype=np.float64))


def random_bsr(nb: int, mb: int, bs: int, density: float, *, seed: int, empty_rows: float = 0.0) -> BSR:
    """Random block pattern (as random_csr) with dense blocks of uniform [-1, 1] values."""
    pat = random_csr(nb, mb, density, seed=seed, empty_rows=empty_rows)
    rng = np.random.default_rng(seed + 7919)
    val = rng.uniform(-1.0, 1.0, size=(pat.nnz, bs, bs))
    return BSR(nb, mb, bs, pat.rowptr, pat.col, val)


# --------------------------------------------------------------------------------------------
# Small matrices for edge cases
# --------------------------------------------------------------------------------------------

def random_csr(n_rows: int, n_cols: int, density: float, *, seed: int, empty_rows: float = 0.0,
               zero_cols: int = 0, explicit_zeros: float = 0.0, max_row: int | None = None) -> CSR:
    """Random CSR matrix with uniform values in [-1, 1].

    empty_rows: fraction of rows forced empty; zero_cols: number of columns never used;
    explicit_zeros: fraction of stored entries whose value is 0.0 (kept as structure);
    max_row: cap on entries per row."""
    rng = np.random.default_rng(seed)
    allowed = np.arange(n_cols)
    if zero_cols:
        dead = rng.choice(n_cols, size=min(zero_cols, n_cols), replace=False)
        allowed = np.setdiff1d(allowed, dead)
    rowptr = [0]
    cols, vals = [], []
    for _ in range(n_rows):
        if rng.random() < empty_rows or allowed.size == 0:
            rowptr.append(rowptr[-1])
            continue
        cnt = rng.binomial(allowed.size, density)
        if max_row is not None:
            cnt = min(cnt, max_row)
        c = np.sort(rng.choice(allowed, size=cnt, replace=False))
        v = rng.uniform(-1.0, 1.0, size=cnt)
        if explicit_zeros:
            v[rng.random(cnt) < explicit_zeros] = 0.0
        cols.append(c); vals.append(v)
        rowptr.append(rowptr[-1] + cnt)
    col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    val = np.concatenate(vals) if vals else np.zeros(0)
    return CSR(n_rows, n_cols, np.array(rowptr, dtype=np.int32), col, val)


# Sparsity patterns of the worked example of the row-wise product (Section 2, Eq. rowwise):
# a 6x6 A times a 6x4 P, rows partitioned over three processes (two rows each).
TOY_A_ROWS = [[0, 1, 4], [1, 2, 4], [0, 3, 4], [1, 3], [3, 4], [1, 4, 5]]
TOY_P_ROWS = [[0, 3], [1], [2, 3], [2], [1, 3], [2]]


def toy_rowwise(seed: int = 0) -> tuple[CSR, CSR]:
    """The worked example's A (6x6) and P (6x4) patterns with seeded uniform [-1,1] values."""
    rng = np.random.default_rng(seed)

    def build(rows, ncols):
        rp = np.zeros(len(rows) + 1, dtype=np.int32)
        rp[1:] = np.cumsum([len(r) for r in rows])
        col = np.array([c for r in rows for c in r], dtype=np.int32)
        return CSR(len(rows), ncols, rp, col, rng.uniform(-1.0, 1.0, size=col.size))

    return build(TOY_A_ROWS, 6), build(TOY_P_ROWS, 4)


# --------------------------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------------------------

def galerkin_workload(name: str, scale: int | None = None) -> tuple[CSR, CSR, dict]:
    """Return (A, P, info) for a named workload.

    c1: 16^3 7-point Laplacian (6/-1, Dirichlet), trilinear to 8^3.
    c2: 128^3 27-point lognormal (seed 1), trilinear to 64^3.
    c3a/c3b: 96^3 anisotropic 27-point (eps 0.01 in z, lognormal seed 2), smoothed aggregation
             3x3x3 with one (c3a) or two (c3b) damped-Jacobi steps.
    c3c: block variant G=4 of c3a (seed 2).
    c5: 64^3 27-point lognormal (seed 4), trilinear to 32^3.
    `scale` overrides the fine grid side (for reduced-size tests)."""
    if name == "c1":
        s = scale or 16
        A, P = laplacian7(s), trilinear(s)
    elif name == "c2":
        s = scale or 128
        A, P = stencil27(s, seed=1), trilinear(s)
    elif name in ("c3a", "c3b"):
        s = scale or 96
        A = stencil27(s, seed=2, eps_z=0.01)
        P = smoothed_aggregation(A, s, s, s, steps=1 if name == "c3a" else 2)
    elif name == "c3c":
        s = scale or 96
        A = block_stencil27(s, 4, seed=2)
        P = block_smoothed_aggregation(A, s, 4)
    elif name == "c5":
        s = scale or 64
        A, P = stencil27(s, seed=4), trilinear(s)
    else:
        raise KeyError(name)
    return A, P, {"name": name, "side": s, "n": A.n_rows, "m": P.n_cols}


def batch_problem_sides(count: int = 64, *, seed: int = 3, lo: int = 12, hi: int = 64) -> np.ndarray:
    """Grid sides (nx, ny, nz) of independent problems, i.i.d. uniform integers in [lo, hi]."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=(count, 3))


def hierarchy_sides(finest: int = 256, levels: int = 6) -> list[int]:
    """Fine-grid sides of a geometric hierarchy with 2x vertex-centred coarsening."""
    out = [finest]
    for _ in range(levels - 1):
        out.append(coarse_side(out[-1]))
    return out


def loss_weights(nnz: int, *, seed: int) -> np.ndarray:
    """W ~ N(0, 1) on the stored entries of C, for the loss L = sum(W o C)."""
    return np.random.default_rng(seed).standard_normal(nnz)
