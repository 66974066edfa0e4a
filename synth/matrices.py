"""Seeded synthetic sparse matrices in CSR form.

This module only *draws* inputs: sparsity patterns, values and right-hand-side
seeds.  It holds none of the solver arithmetic (no products, no features, no
Krylov steps), so both the CPU oracle and the GPU path can take their inputs
from here without sharing any of the method's code.

Every generator returns a :class:`CSR` with int32 row pointers and column
indices (columns strictly increasing inside each row) and float64 values.
Randomness comes only from ``numpy.random.default_rng(seed)`` (PCG64).

The families stand in for the SuiteSparse matrices the paper trains and tests
on (dataset construction, and the test-matrix table of the evaluation): the
collection is not available here, so stencil, power-law, block-diagonal,
uniform-random, graph-Laplacian and convection-diffusion patterns with the
same range of sizes (769 to 2.06M rows) and row lengths (about 6 to 424 nonzeros
per row) replace it.
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np


@dataclass
class CSR:
    n: int                 # rows
    ncols: int             # columns
    rp: np.ndarray         # int32[n+1]
    col: np.ndarray        # int32[nnz]
    val: np.ndarray        # float64[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rp[-1])

    def check(self) -> "CSR":
        assert self.rp.dtype == np.int32 and self.col.dtype == np.int32
        assert self.val.dtype == np.float64
        assert self.rp.shape == (self.n + 1,) and self.rp[0] == 0
        assert self.col.shape == (self.nnz,) and self.val.shape == (self.nnz,)
        return self


def _finish(n, ncols, rows, cols, vals, name, presorted=False) -> CSR:
    """Assemble COO triples (rows nondecreasing if presorted) into CSR."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    if not presorted:
        order = np.lexsort((cols, rows))
        rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n) if n > 0 else np.zeros(0, np.int64)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    assert rp[-1] < 2**31, "int32 index space exceeded"
    return CSR(n, ncols, rp.astype(np.int32), cols.astype(np.int32), vals, name).check()


# --------------------------------------------------------------------------
# Structured PDE matrices
# --------------------------------------------------------------------------

def laplacian_1d(n: int) -> CSR:
    """tridiag(-1, 2, -1), Dirichlet."""
    i = np.arange(n, dtype=np.int64)
    rows = np.concatenate([i[1:], i, i[:-1]])
    cols = np.concatenate([i[1:] - 1, i, i[:-1] + 1])
    vals = np.concatenate([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)])
    return _finish(n, n, rows, cols, vals, f"lap1d_{n}")


def _grid_stencil(dims, offsets, weights, name, nrows=None, values=None, rng=None):
    """Assemble a stencil on a row-major grid (last dimension fastest).

    ``offsets`` are integer grid offsets (tuples), ``weights`` the matching
    coefficients.  Neighbours outside the grid are dropped (Dirichlet).  When
    ``nrows`` is given only the first ``nrows`` grid points are kept (rows and
    columns), which turns any grid into an ``nrows x nrows`` matrix.
    ``values='normal'`` replaces the weights by N(0,1) draws from ``rng``.
    """
    dims = tuple(int(d) for d in dims)
    npts = int(np.prod(dims))
    n = npts if nrows is None else int(nrows)
    coords = np.unravel_index(np.arange(n, dtype=np.int64), dims)
    strides = [int(np.prod(dims[d + 1:])) for d in range(len(dims))]
    # offsets sorted by linear displacement so each row's columns come out sorted
    order = sorted(range(len(offsets)),
                   key=lambda t: sum(o * s for o, s in zip(offsets[t], strides)))
    base = np.arange(n, dtype=np.int64)
    noff = len(offsets)
    colmat = np.empty((n, noff), dtype=np.int64)
    okmat = np.empty((n, noff), dtype=bool)
    wvec = np.empty(noff)
    for j, t in enumerate(order):
        off = offsets[t]
        ok = np.ones(n, dtype=bool)
        lin = base.copy()
        for d, o in enumerate(off):
            c = coords[d] + o
            ok &= (c >= 0) & (c < dims[d])
            lin += o * strides[d]
        ok &= (lin >= 0) & (lin < n)
        colmat[:, j] = lin
        okmat[:, j] = ok
        wvec[j] = float(weights[t])
    # row-major flattening keeps rows in order and columns sorted inside rows
    mask = okmat.reshape(-1)
    cols = colmat.reshape(-1)[mask]
    rows = np.repeat(base, noff)[mask]
    vals = np.tile(wvec, n)[mask]
    if values == "normal":
        vals = rng.standard_normal(vals.shape[0])
    return _finish(n, n, rows, cols, vals, name, presorted=True)


def laplacian_2d(N: int) -> CSR:
    """5-point Dirichlet Laplacian on an N x N grid (centre 4, neighbours -1)."""
    offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
    w = [4.0, -1.0, -1.0, -1.0, -1.0]
    return _grid_stencil((N, N), offs, w, f"lap2d_{N}")


def laplacian_3d(N: int) -> CSR:
    """7-point Dirichlet Laplacian on an N^3 grid (centre 6, neighbours -1)."""
    offs = [(0, 0, 0)] + [tuple(s if d == a else 0 for d in range(3))
                          for a in range(3) for s in (-1, 1)]
    w = [6.0] + [-1.0] * 6
    return _grid_stencil((N, N, N), offs, w, f"lap3d_{N}")


def convection_diffusion_2d(N: int, peclet: float = 10.0) -> CSR:
    """-Lap(u) + Pe (u_x + u_y) on (0,1)^2, Dirichlet, first-order upwind.

    Mesh width h = 1/(N+1); the rows are scaled by h^2, giving centre
    4 + 2 Pe h, west and south -1 - Pe h, east and north -1 (global Peclet
    number ``peclet``).  Grid index = y * N + x, x fastest.
    """
    h = 1.0 / (N + 1)
    ph = peclet * h
    offs = [(0, 0), (-1, 0), (0, -1), (0, 1), (1, 0)]   # (dy, dx)
    w = [4.0 + 2.0 * ph, -1.0 - ph, -1.0 - ph, -1.0, -1.0]
    return _grid_stencil((N, N), offs, w, f"convdiff_{N}_pe{peclet:g}")


# stencil shapes for the banded family, by row length
def _stencil_offsets(r: int):
    if r == 5:
        return (2, [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)])
    if r == 9:
        return (2, [(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)])
    if r == 7:
        return (3, [(0, 0, 0)] + [tuple(s if d == a else 0 for d in range(3))
                                  for a in range(3) for s in (-1, 1)])
    if r == 13:   # 7-point plus the second neighbours along each axis
        return (3, [(0, 0, 0)] + [tuple(s if d == a else 0 for d in range(3))
                                  for a in range(3) for s in (-2, -1, 1, 2)])
    if r == 19:   # faces and edges of the 3x3x3 cube
        return (3, [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
                    if abs(a) + abs(b) + abs(c) <= 2])
    if r == 27:
        return (3, [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)])
    raise ValueError(f"no stencil with {r} points")


def banded_stencil(n: int, r: int, seed: int) -> CSR:
    """n x n stencil matrix with interior row length r, values N(0,1).

    The grid is the smallest near-cubic (or near-square) grid with >= n points;
    only the first n points are kept, so boundary rows are clipped.
    """
    dim, offs = _stencil_offsets(r)
    side = int(math.ceil(n ** (1.0 / dim)))
    while side ** dim < n:
        side += 1
    if dim == 2:
        dims = (int(math.ceil(n / side)), side)
    else:
        dims = (int(math.ceil(n / (side * side))), side, side)
    rng = np.random.default_rng(seed)
    return _grid_stencil(dims, offs, [1.0] * len(offs), f"banded{r}_{n}",
                         nrows=n, values="normal", rng=rng)


# --------------------------------------------------------------------------
# Random patterns
# --------------------------------------------------------------------------

def _random_sorted_columns(rng, lengths, ncols):
    """Distinct sorted column indices per row, uniform without replacement.

    Rows shorter than ncols/2 use sorted uniform order statistics built from
    normalised exponential gaps (no global sort needed), floored to integers;
    the rare coincident pair is merged, so a row can come out a little
    shorter than drawn.  Longer rows use an explicit random subset.
    """
    lengths = np.asarray(lengths, dtype=np.int64)
    n = lengths.shape[0]
    big = lengths > ncols // 2
    small_len = np.where(big, 0, lengths)
    seg = small_len + 1
    tot = int(seg.sum())
    e = rng.standard_exponential(tot)
    cs = np.cumsum(e)
    ends = np.cumsum(seg) - 1
    starts = ends - seg + 1
    base = np.zeros(n)
    base[1:] = cs[ends[:-1]]
    seg_id = np.repeat(np.arange(n, dtype=np.int64), seg)
    local = cs - base[seg_id]
    total = local[ends]
    pos = np.arange(tot, dtype=np.int64) - starts[seg_id]
    keep = pos < small_len[seg_id]                      # drop each row's last gap
    u = local[keep] / total[seg_id[keep]]
    rows = seg_id[keep]
    cols = np.minimum((u * ncols).astype(np.int64), ncols - 1)
    dup = np.zeros(cols.shape[0], dtype=bool)
    if cols.shape[0] > 1:
        dup[1:] = (cols[1:] == cols[:-1]) & (rows[1:] == rows[:-1])
    rows, cols = rows[~dup], cols[~dup]
    if big.any():
        br, bc = [], []
        for i in np.nonzero(big)[0]:
            c = np.sort(rng.choice(ncols, size=int(lengths[i]), replace=False))
            br.append(np.full(c.shape[0], i, dtype=np.int64))
            bc.append(c.astype(np.int64))
        rows = np.concatenate([rows] + br)
        cols = np.concatenate([cols] + bc)
        order = np.lexsort((cols, rows))
        rows, cols = rows[order], cols[order]
    return rows, cols


def zipf_lengths(rng, n, s, rmax):
    """Row lengths ~ Zipf(s) truncated to [1, rmax] (inverse-CDF sampling)."""
    k = np.arange(1, rmax + 1, dtype=np.float64)
    p = k ** (-s)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    u = rng.random(n)
    return np.searchsorted(cdf, u, side="right").clip(0, rmax - 1) + 1


def power_law_rows(n: int, s: float, seed: int, rmax: int = 10_000) -> CSR:
    """Row lengths ~ Zipf(s) in [1, min(rmax, n)], columns uniform, values N(0,1)."""
    rng = np.random.default_rng(seed)
    lengths = zipf_lengths(rng, n, s, min(rmax, n))
    rows, cols = _random_sorted_columns(rng, lengths, n)
    vals = rng.standard_normal(rows.shape[0])
    return _finish(n, n, rows, cols, vals, f"powerlaw{s:.3f}_{n}", presorted=True)


def uniform_random(n: int, seed: int, rmin: int = 4, rmax: int = 64) -> CSR:
    """Row lengths ~ U{rmin..rmax}, columns uniform without replacement, N(0,1)."""
    rng = np.random.default_rng(seed)
    lengths = rng.integers(rmin, rmax + 1, size=n)
    lengths = np.minimum(lengths, n)
    rows, cols = _random_sorted_columns(rng, lengths, n)
    vals = rng.standard_normal(rows.shape[0])
    return _finish(n, n, rows, cols, vals, f"uniform{rmin}-{rmax}_{n}", presorted=True)


def block_diagonal(n: int, seed: int, b: int = 8) -> CSR:
    """Dense b x b diagonal blocks (n rounded up to a multiple of b), N(0,1)."""
    n = int(math.ceil(n / b) * b)
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.int64)
    rows = np.repeat(i, b)
    cols = (np.repeat(i // b * b, b) + np.tile(np.arange(b), n))
    vals = rng.standard_normal(n * b)
    return _finish(n, n, rows, cols, vals, f"blockdiag{b}_{n}", presorted=True)


def graph_laplacian_chung_lu(n: int, seed: int, mean_degree: int = 16,
                             zipf_s: float = 2.0, wmax: int = 10_000,
                             shift: float = 1e-2) -> CSR:
    """Power-law graph Laplacian plus ``shift * I`` (SPD).

    Chung-Lu construction: vertex weights ~ Zipf(zipf_s) over [1, wmax];
    edge endpoints are drawn proportionally to weight until exactly
    ``mean_degree * n / 2`` distinct undirected non-loop edges exist.  Edges
    into a vertex whose degree already reached ``wmax`` are rejected (batch
    by batch, newest batch first).  Off-diagonal entries are -1 and the
    diagonal is degree + shift.
    """
    rng = np.random.default_rng(seed)
    target = mean_degree * n // 2
    w = zipf_lengths(rng, n, zipf_s, wmax).astype(np.float64)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    keys = np.zeros(0, dtype=np.int64)
    while keys.shape[0] < target:
        need = target - keys.shape[0]
        m = int(need * 1.25) + 1024
        u = np.searchsorted(cdf, rng.random(m), side="right").clip(0, n - 1)
        v = np.searchsorted(cdf, rng.random(m), side="right").clip(0, n - 1)
        ok = u != v
        a = np.minimum(u[ok], v[ok]).astype(np.int64)
        b = np.maximum(u[ok], v[ok]).astype(np.int64)
        new = a * n + b
        new = np.unique(new)                      # dedupe inside the batch
        new = new[~np.isin(new, keys)]            # drop edges already present
        rng.shuffle(new)
        new = new[:need]
        # degree cap: drop newest edges that push a vertex past wmax
        both = np.concatenate([keys, new])
        deg = np.bincount(both // n, minlength=n) + np.bincount(both % n, minlength=n)
        if deg.max() > wmax:
            over = deg > wmax
            bad = over[new // n] | over[new % n]
            new = new[~bad]
        keys = np.concatenate([keys, new])
    a, b = keys // n, keys % n
    deg = np.bincount(a, minlength=n) + np.bincount(b, minlength=n)
    rows = np.concatenate([a, b, np.arange(n, dtype=np.int64)])
    cols = np.concatenate([b, a, np.arange(n, dtype=np.int64)])
    vals = np.concatenate([-np.ones(2 * keys.shape[0]), deg.astype(np.float64) + shift])
    return _finish(n, n, rows, cols, vals, f"graphlap_{n}")


# --------------------------------------------------------------------------
# Small matrices for pins and edge cases
# --------------------------------------------------------------------------

def from_dense(D: np.ndarray, name: str = "dense") -> CSR:
    """Store every nonzero of a dense array (explicit zeros are dropped)."""
    D = np.asarray(D, dtype=np.float64)
    rows, cols = np.nonzero(D)
    return _finish(D.shape[0], D.shape[1], rows, cols, D[rows, cols], name, presorted=True)


def full_from_dense(D: np.ndarray, name: str = "full") -> CSR:
    """Store every entry of a dense array, zeros included."""
    D = np.asarray(D, dtype=np.float64)
    n, m = D.shape
    rows = np.repeat(np.arange(n), m)
    cols = np.tile(np.arange(m), n)
    return _finish(n, m, rows, cols, D.reshape(-1), name, presorted=True)


def spd_dense(n: int, eigs, seed: int) -> np.ndarray:
    """Q diag(eigs) Q^T with Q from the QR factor of a Gaussian matrix."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * np.asarray(eigs, dtype=np.float64)) @ Q.T


def random_integer(n: int, ncols: int, seed: int, density: float = 0.1,
                   lo: int = -8, hi: int = 8, empty_rows: float = 0.1,
                   long_rows: int = 0, long_len: int = 0) -> CSR:
    """Integer-valued random pattern (values in [lo, hi] without 0).

    A fraction ``empty_rows`` of the rows is left empty; ``long_rows`` rows get
    ``long_len`` entries so that row lengths are skewed.  Integer values keep
    every partial sum exact in floating point.
    """
    rng = np.random.default_rng(seed)
    lengths = rng.binomial(ncols, density, size=n).astype(np.int64)
    lengths[rng.random(n) < empty_rows] = 0
    if long_rows:
        idx = rng.choice(n, size=min(long_rows, n), replace=False)
        lengths[idx] = min(long_len, ncols)
    rows_l, cols_l = [], []
    for i in range(n):
        if lengths[i]:
            c = np.sort(rng.choice(ncols, size=int(lengths[i]), replace=False))
            rows_l.append(np.full(c.shape[0], i))
            cols_l.append(c)
    if rows_l:
        rows = np.concatenate(rows_l)
        cols = np.concatenate(cols_l)
    else:
        rows = np.zeros(0, np.int64)
        cols = np.zeros(0, np.int64)
    vals = rng.integers(1, hi + 1, size=rows.shape[0]) * rng.choice([-1, 1], size=rows.shape[0])
    vals = np.clip(vals, lo, hi).astype(np.float64)
    return _finish(n, ncols, rows, cols, vals, f"randint_{n}x{ncols}", presorted=True)


def column_runs(n: int, ncols: int, seed: int) -> CSR:
    """Rows made of runs of consecutive columns (run lengths 1..600, gaps
    1..5), row lengths drawn from {0, 1, 7, 8, 9, 63, 64, 65, 255, 256, 257,
    511, 512, 513, 700, 2000} so that runs and rows end at and across every
    power-of-two boundary; small integer values."""
    rng = np.random.default_rng(seed)
    lengths = np.array([0, 1, 7, 8, 9, 63, 64, 65, 255, 256, 257, 511, 512, 513, 700, 2000])
    rows, cols = [], []
    for i in range(n):
        r = int(min(rng.choice(lengths), ncols))
        c = int(rng.integers(0, max(1, ncols - 3 * r)))
        out = []
        while len(out) < r and c < ncols:
            run = int(rng.integers(1, 601))
            take = min(run, r - len(out), ncols - c)
            out.extend(range(c, c + take))
            c += take + int(rng.integers(1, 6))
        rows.extend([i] * len(out))
        cols.extend(out)
    vals = rng.integers(-9, 10, len(cols)).astype(np.float64)
    return _finish(n, ncols, rows, cols, vals, f"runs_{n}x{ncols}", presorted=True)


def diagonally_dominant(A: CSR, name: str | None = None) -> CSR:
    """Set a_ii = 1 + sum_{j != i} |a_ij| (inserting the diagonal if absent).

    Gives a strictly diagonally dominant (hence nonsingular) matrix for the
    nonsymmetric members of the serving pool.
    """
    assert A.n == A.ncols
    rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.rp.astype(np.int64)))
    cols = A.col.astype(np.int64)
    off = rows != cols
    rows, cols, vals = rows[off], cols[off], A.val[off]
    d = 1.0 + np.bincount(rows, weights=np.abs(vals), minlength=A.n)
    rows = np.concatenate([rows, np.arange(A.n)])
    cols = np.concatenate([cols, np.arange(A.n)])
    vals = np.concatenate([vals, d])
    return _finish(A.n, A.n, rows, cols, vals, name or A.name + "_dd")


def vector(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Uniform [lo, hi) vector (exact solutions x*, SpMV inputs)."""
    return np.random.default_rng(seed).uniform(lo, hi, size=n)
