"""Pins for the oracle SpMV: dense matvec, closed-form eigenpairs, invariants."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from synth import matrices as M


def sinvec(n, k):
    """sin(i k pi/(n+1)), i = 1..n, with the argument reduced exactly mod 2(n+1)."""
    i = np.arange(1, n + 1, dtype=np.int64)
    return np.sin(((i * k) % (2 * (n + 1))) * math.pi / (n + 1))


def dense(A):
    D = np.zeros((A.n, A.ncols))
    for i in range(A.n):
        for k in range(A.rp[i], A.rp[i + 1]):
            D[i, A.col[k]] = A.val[k]
    return D


@pytest.mark.parametrize("n,m,seed", [(1, 1, 0), (7, 5, 1), (64, 64, 2), (130, 77, 3),
                                      (257, 300, 4)])
def test_integer_matrix_bit_exact_vs_dense(orc, n, m, seed):
    A = M.random_integer(n, m, seed, density=0.2, long_rows=2, long_len=m)
    x = np.random.default_rng(seed).integers(-8, 9, size=m).astype(np.float64)
    y = orc.spmv(A, x)
    ref = dense(A) @ x             # every partial sum is an exact integer
    assert np.array_equal(y, ref)


def test_alpha_beta_exact_and_beta_zero_ignores_y(orc):
    A = M.random_integer(50, 40, 7, density=0.3)
    x = np.random.default_rng(1).integers(-8, 9, size=40).astype(np.float64)
    y0 = np.random.default_rng(2).integers(-8, 9, size=50).astype(np.float64)
    y = orc.spmv(A, x, alpha=-3.0, beta=2.0, y=y0)
    assert np.array_equal(y, -3.0 * (dense(A) @ x) + 2.0 * y0)
    ynan = np.full(50, np.nan)
    y = orc.spmv(A, x, alpha=1.0, beta=0.0, y=ynan)
    assert np.all(np.isfinite(y)) and np.array_equal(y, dense(A) @ x)


def test_empty_rows_and_empty_matrix(orc):
    A = M.from_dense(np.zeros((5, 3)))
    assert A.nnz == 0
    y = orc.spmv(A, np.ones(3), beta=0.5, y=np.full(5, 2.0))
    assert np.array_equal(y, np.full(5, 1.0))


@pytest.mark.parametrize("n", [8, 100, 1000])
def test_laplacian_1d_eigenvectors(orc, n):
    A = M.laplacian_1d(n)
    for k in (1, 2, n // 2, n):
        v = sinvec(n, k)
        lam = 2.0 - 2.0 * math.cos(k * math.pi / (n + 1))
        assert np.max(np.abs(orc.spmv(A, v) - lam * v)) <= 1e-13 * 4 * np.max(np.abs(v))


def test_laplacian_2d_eigenvectors_and_condition(orc):
    N = 64
    A = M.laplacian_2d(N)
    for j, k in [(1, 1), (3, 7), (N, N), (10, 50)]:
        v = np.outer(sinvec(N, j), sinvec(N, k)).ravel()
        lam = 4 - 2 * math.cos(j * math.pi / (N + 1)) - 2 * math.cos(k * math.pi / (N + 1))
        assert np.max(np.abs(orc.spmv(A, v) - lam * v)) <= 1e-13 * 8
    lmin = 4 - 4 * math.cos(math.pi / (N + 1))
    lmax = 4 + 4 * math.cos(math.pi / (N + 1))
    assert abs(lmax / lmin - 1711.66) < 0.01


def test_laplacian_2d_row_sums(orc):
    N = 16
    A = M.laplacian_2d(N)
    s = orc.spmv(A, np.ones(A.n)).reshape(N, N)
    expect = np.zeros((N, N))
    expect[0, :] += 1
    expect[-1, :] += 1
    expect[:, 0] += 1
    expect[:, -1] += 1
    assert np.array_equal(s, expect)       # 0 interior, 1 edges, 2 corners


def test_convection_diffusion_interior_rows_sum_to_zero(orc):
    N = 32
    A = M.convection_diffusion_2d(N, 10.0)
    s = orc.spmv(A, np.ones(A.n)).reshape(N, N)
    assert np.max(np.abs(s[1:-1, 1:-1])) <= 1e-14
    # boundary rows keep the missing neighbour's weight
    h = 1.0 / (N + 1)
    assert abs(s[0, 1] - (1.0 + 10.0 * h)) < 1e-14      # south neighbour missing
    assert abs(s[1, -1] - 1.0) < 1e-14                   # east neighbour missing


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_scipy_on_gaussian_values(orc, seed):
    A = M.uniform_random(3000, seed)
    x = M.vector(3000, seed + 10)
    y0 = M.vector(3000, seed + 20)
    S = sp.csr_matrix((A.val, A.col, A.rp), shape=(A.n, A.ncols))
    y = orc.spmv(A, x, alpha=0.7, beta=-1.3, y=y0)
    ref = 0.7 * (S @ x) - 1.3 * y0
    normA = np.max(np.abs(S).sum(axis=1))
    assert np.max(np.abs(y - ref)) <= 1e-13 * (0.7 * normA * np.max(np.abs(x)) + 1.3 * np.max(np.abs(y0)))


def test_relres(orc):
    A = M.laplacian_1d(20)
    x = M.vector(20, 3)
    b = orc.spmv(A, x)
    assert orc.relres(A, b, x) == 0.0
    assert abs(orc.relres(A, b, np.zeros(20)) - 1.0) < 1e-15
