"""Seeded sparse test matrices (CSR: int64 row pointers, int32 sorted distinct
column indices, float64 values).

Every generator draws from ``numpy.random.Generator(PCG64(seed))`` in a fixed
order, in fixed-size row chunks, so a given (shape, seed) always yields the
same bytes.  The shapes and distributions follow the paper's workload classes
(Section 4, Table of test matrices): rectangular least-squares matrices with
tiny smallest-gap ratios, irregular graph-like matrices, and PDE operators.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

_CHUNK = 65536


def to_csr(A) -> sp.csr_matrix:
    """Canonical CSR: sorted, summed duplicates, int64 indptr, int32 indices."""
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int64)
    A.indices = A.indices.astype(np.int32)
    return A


def _csr_from_rows(m, n, lengths, cols, vals) -> sp.csr_matrix:
    indptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lengths, out=indptr[1:])
    A = sp.csr_matrix((vals, cols.astype(np.int32), indptr), shape=(m, n))
    A.indptr = indptr
    A.indices = A.indices.astype(np.int32)
    A.sort_indices()
    return A


def _distinct_columns(rng, lengths, n):
    """Uniform distinct columns per row (row lengths << n).  Duplicates inside a
    row are redrawn until none is left; the result is sorted per row."""
    lengths = np.asarray(lengths, dtype=np.int64)
    total = int(lengths.sum())
    row = np.repeat(np.arange(lengths.size, dtype=np.int64), lengths)
    col = rng.integers(0, n, size=total, dtype=np.int64)
    while True:
        order = np.lexsort((col, row))
        col = col[order]
        row = row[order]
        dup = np.zeros(total, dtype=bool)
        dup[1:] = (row[1:] == row[:-1]) & (col[1:] == col[:-1])
        nd = int(dup.sum())
        if nd == 0:
            return col
        col[dup] = rng.integers(0, n, size=nd, dtype=np.int64)


def random_uniform_rows(m, n, lengths, seed) -> sp.csr_matrix:
    """Rows with the given lengths at uniform random distinct columns, N(0,1)
    values.  Columns are drawn for all rows first, then the values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lengths = np.broadcast_to(np.asarray(lengths, dtype=np.int64), (m,)).copy()
    if np.any(lengths > n):
        raise ValueError("row longer than the number of columns")
    cols = np.empty(int(lengths.sum()), dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(lengths)])
    for r0 in range(0, m, _CHUNK):
        r1 = min(m, r0 + _CHUNK)
        cols[starts[r0]:starts[r1]] = _distinct_columns(rng, lengths[r0:r1], n)
    vals = rng.standard_normal(cols.size)
    return _csr_from_rows(m, n, lengths, cols, vals)


def uniform_workload(seed=1001, m=2000, n=1000, nnz_per_row=10) -> sp.csr_matrix:
    """2000 x 1000, 10 nonzeros per row at uniform random columns, N(0,1)."""
    return random_uniform_rows(m, n, nnz_per_row, seed)


def banded_scaled(m, n, seed, band=64, per_row=16, log_lo=-4.0, log_hi=0.0):
    """Banded rectangular matrix times a random column scaling.

    Row i draws ``per_row`` distinct columns inside a ``band``-wide window that
    starts at clip(floor(i*n/m) - band/2, 0, n - band); values are N(0,1).
    Then A <- A * diag(10**U(log_lo, log_hi)) with one scale per column, drawn
    after all values from the same generator.
    """
    if n < band:
        raise ValueError("n must be at least the band width")
    rng = np.random.Generator(np.random.PCG64(seed))
    cols = np.empty((m, per_row), dtype=np.int64)
    for r0 in range(0, m, _CHUNK):
        r1 = min(m, r0 + _CHUNK)
        keys = rng.random((r1 - r0, band))
        pick = np.sort(np.argpartition(keys, per_row - 1, axis=1)[:, :per_row], axis=1)
        i = np.arange(r0, r1, dtype=np.int64)
        start = np.clip(i * n // m - band // 2, 0, n - band)
        cols[r0:r1] = start[:, None] + pick
    vals = np.empty(m * per_row)
    for r0 in range(0, m, _CHUNK):
        r1 = min(m, r0 + _CHUNK)
        vals[r0 * per_row:r1 * per_row] = rng.standard_normal((r1 - r0) * per_row)
    scale = 10.0 ** rng.uniform(log_lo, log_hi, size=n)
    cols = cols.reshape(-1)
    vals *= scale[cols]
    return _csr_from_rows(m, n, np.full(m, per_row), cols, vals)


def banded_workload(m=1_000_000, n=500_000, seed=1002):
    """Banded (64 wide, 16 per row) times log-uniform column scaling in
    [1e-4, 1]; least-squares-like with tiny smallest-gap ratios."""
    return banded_scaled(m, n, seed)


def powerlaw_rows(m, n, seed, exponent=2.1, lmin=3.924, lmax=2000):
    """Row lengths from a power law with density ~ L**(-exponent) on
    [lmin, lmax] (mean about 20 for the defaults), rounded; uniform distinct
    columns; N(0,1) values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = exponent - 1.0
    u = rng.random(m)
    tail = 1.0 - (lmin / lmax) ** a
    L = lmin * (1.0 - u * tail) ** (-1.0 / a)
    lengths = np.clip(np.rint(L), 1, min(lmax, n)).astype(np.int64)
    cols = np.empty(int(lengths.sum()), dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(lengths)])
    for r0 in range(0, m, _CHUNK):
        r1 = min(m, r0 + _CHUNK)
        cols[starts[r0]:starts[r1]] = _distinct_columns(rng, lengths[r0:r1], n)
    vals = np.empty(cols.size)
    for s0 in range(0, cols.size, _CHUNK * 16):
        s1 = min(cols.size, s0 + _CHUNK * 16)
        vals[s0:s1] = rng.standard_normal(s1 - s0)
    return _csr_from_rows(m, n, lengths, cols, vals)


def powerlaw_workload(m=2_000_000, n=1_000_000, seed=1003):
    """Power-law row lengths (mean 20, max 2000, exponent 2.1), N(0,1)."""
    return powerlaw_rows(m, n, seed)


def batched_problem(i, seed_base=4000, mmin=5000, mmax=200000, lmin=8, lmax=12):
    """Problem i of the batched workload: rows U{mmin..mmax}, cols rows/2,
    U{lmin..lmax} nonzeros per row, N(0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed_base + i))
    m = int(rng.integers(mmin, mmax + 1))
    n = m // 2
    lengths = rng.integers(lmin, lmax + 1, size=m)
    sub_seed = int(rng.integers(0, 2**62))
    return random_uniform_rows(m, n, lengths, sub_seed)


def _smooth_field(ng, seed, nmodes=4):
    """Log-coefficient field: 16 low Fourier modes (kx, ky in 1..4) with
    amplitude ~ N(0,1)/(kx^2+ky^2) and uniform phases, on the (ng+2)^2 grid
    including the boundary, normalised to zero mean and unit variance."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / (ng + 1)
    x = np.arange(ng + 2) * h
    X, Y = np.meshgrid(x, x, indexing="xy")  # Y varies along axis 0 (iy)
    g = np.zeros_like(X)
    for kx in range(1, nmodes + 1):
        for ky in range(1, nmodes + 1):
            amp = rng.standard_normal() / (kx * kx + ky * ky)
            phase = rng.uniform(0.0, 2.0 * np.pi)
            g += amp * np.cos(2.0 * np.pi * (kx * X + ky * Y) + phase)
    g = (g - g.mean()) / g.std()
    return g


def convection_diffusion(ng, seed, peclet=10.0, drop_rows=None):
    """h^2-scaled 5-point discretisation of -div(a grad u) + beta . grad u on
    the unit square, Dirichlet zero, ng x ng interior nodes, h = 1/(ng+1),
    row = iy*ng + ix.  Face coefficients are the arithmetic mean of a at the two
    nodes; convection is first-order upwind with beta = Pe*mean(a)*(1,1)/sqrt(2)
    (global Peclet number Pe on the unit length).  a = exp(0.5*g) with g the
    smooth random field above.  The last ``drop_rows`` rows (whole grid lines)
    are removed, which makes the matrix rectangular (m < n)."""
    h = 1.0 / (ng + 1)
    a = np.exp(0.5 * _smooth_field(ng, seed))  # (ng+2, ng+2), [iy, ix]
    abar = a[1:-1, 1:-1].mean()
    bx = by = peclet * abar / np.sqrt(2.0)
    aP = a[1:-1, 1:-1]
    aE = 0.5 * (aP + a[1:-1, 2:])
    aW = 0.5 * (aP + a[1:-1, :-2])
    aN = 0.5 * (aP + a[2:, 1:-1])
    aS = 0.5 * (aP + a[:-2, 1:-1])
    N = ng * ng
    idx = np.arange(N).reshape(ng, ng)
    diag = (aE + aW + aN + aS + h * (bx + by)).ravel()
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [diag]
    # east (ix+1), west (ix-1), north (iy+1), south (iy-1)
    rows.append(idx[:, :-1].ravel()); cols.append(idx[:, 1:].ravel()); vals.append(-aE[:, :-1].ravel())
    rows.append(idx[:, 1:].ravel()); cols.append(idx[:, :-1].ravel()); vals.append((-aW - h * bx)[:, 1:].ravel())
    rows.append(idx[:-1, :].ravel()); cols.append(idx[1:, :].ravel()); vals.append(-aN[:-1, :].ravel())
    rows.append(idx[1:, :].ravel()); cols.append(idx[:-1, :].ravel()); vals.append((-aS - h * by)[1:, :].ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    A = to_csr(A)
    if drop_rows:
        A = to_csr(A[: N - drop_rows])
    return A


def convdiff_workload(ng=1024, seed=5000, drop_rows=None):
    """1024^2 convection-diffusion, Pe = 10, last 4 grid lines (4096 rows)
    dropped: 1,044,480 x 1,048,576."""
    if drop_rows is None:
        drop_rows = 4 * ng
    return convection_diffusion(ng, seed, drop_rows=drop_rows)


def _haar_orthonormal(rng, rows, cols):
    Z = rng.standard_normal((rows, cols))
    Q, R = np.linalg.qr(Z)
    return Q * np.sign(np.diag(R))


def prescribed_dense(m, n, sigma, seed):
    """Dense A = P diag(sigma) Q^T (m >= n) with Haar-random orthonormal P
    (m x n) and Q (n x n); returned as CSR together with sigma sorted
    ascending, P and Q."""
    sigma = np.asarray(sigma, dtype=np.float64)
    if m < n or sigma.size != n:
        raise ValueError("need m >= n and len(sigma) == n")
    rng = np.random.Generator(np.random.PCG64(seed))
    P = _haar_orthonormal(rng, m, n)
    Q = _haar_orthonormal(rng, n, n)
    A = (P * sigma) @ Q.T
    return to_csr(sp.csr_matrix(A)), np.sort(sigma), P, Q


def _givens_round(rng, size):
    """Sparse orthogonal matrix applying independent random plane rotations to
    random disjoint index pairs (a possible odd index left alone)."""
    perm = rng.permutation(size)
    npair = size // 2
    i = perm[:npair]
    j = perm[npair:2 * npair]
    th = rng.uniform(0.0, 2.0 * np.pi, size=npair)
    c, s = np.cos(th), np.sin(th)
    rows = np.concatenate([i, i, j, j])
    cols = np.concatenate([i, j, i, j])
    vals = np.concatenate([c, -s, s, c])
    if size % 2:
        k = perm[-1:]
        rows = np.concatenate([rows, k]); cols = np.concatenate([cols, k]); vals = np.concatenate([vals, [1.0]])
    return sp.csr_matrix((vals, (rows, cols)), shape=(size, size))


def prescribed_givens(m, n, sigma, seed, rounds=2):
    """Sparse matrix with exactly known singular values: diag(sigma) (m x n,
    m >= n) multiplied on both sides by ``rounds`` layers of random disjoint
    plane rotations.  Orthogonal transforms keep the singular values, so they
    equal ``sigma`` up to rounding at any size."""
    sigma = np.asarray(sigma, dtype=np.float64)
    if m < n or sigma.size != n:
        raise ValueError("need m >= n and len(sigma) == n")
    rng = np.random.Generator(np.random.PCG64(seed))
    D = sp.csr_matrix((sigma, (np.arange(n), np.arange(n))), shape=(m, n))
    A = D
    for _ in range(rounds):
        A = _givens_round(rng, m) @ A
    for _ in range(rounds):
        A = A @ _givens_round(rng, n).T
    return to_csr(A), np.sort(sigma)


def one_per_row(m, n, seed):
    """One nonzero per row (m >= n, every column hit).  A^T A is diagonal,
    so the singular values are the column 2-norms."""
    if m < n:
        raise ValueError("need m >= n")
    rng = np.random.Generator(np.random.PCG64(seed))
    col = np.concatenate([np.arange(n), rng.integers(0, n, size=m - n)])
    col = rng.permutation(col)
    val = rng.standard_normal(m)
    return to_csr(sp.csr_matrix((val, (np.arange(m), col)), shape=(m, n)))


def block_diagonal(nblocks, mb, nb, seed):
    """Block-diagonal matrix of ``nblocks`` dense N(0,1) blocks of shape
    (mb, nb), mb >= nb; returns (A, blocks).  Its singular values are the union
    of the blocks' singular values."""
    if mb < nb:
        raise ValueError("need mb >= nb")
    rng = np.random.Generator(np.random.PCG64(seed))
    blocks = rng.standard_normal((nblocks, mb, nb))
    A = sp.block_diag(list(blocks), format="csr")
    return to_csr(A), blocks
