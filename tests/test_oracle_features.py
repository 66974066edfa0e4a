"""Pins for the oracle features (feature table): closed forms and brute force."""
import math

import numpy as np
import pytest

from synth import matrices as M


def lap2d_closed_form(N):
    """Integer accumulators of the N x N 5-point Laplacian by counting row types."""
    interior, edge_tb, edge_lr, corner = (N - 2) ** 2, 2 * (N - 2), 2 * (N - 2), 4
    n = N * N
    nnz = 5 * interior + 4 * (edge_tb + edge_lr) + 3 * corner
    sum_r2 = 25 * interior + 16 * (edge_tb + edge_lr) + 9 * corner
    # span c_last - c_first: 2N if both vertical neighbours, N+1 or N+... per row type
    span = 0
    for a in range(N):
        for b in range(N):
            i = a * N + b
            first = i - N if a > 0 else (i - 1 if b > 0 else i)
            last = i + N if a < N - 1 else (i + 1 if b < N - 1 else i)
            span += last - first
    # longest run: i-1, i, i+1 consecutive unless at a left/right edge
    cl = 3 * (interior + edge_tb) + 2 * (edge_lr + corner)
    return dict(n=n, nnz=nnz, sum_r2=sum_r2, span=span, cl=cl, max=5, min=3, ndiag=5)


def test_lap2d_64_worked_example(orc):
    A = M.laplacian_2d(64)
    ints, der, f = orc.features(A)
    c = lap2d_closed_form(64)
    assert ints[0] == 4096 and ints[1] == 4096 and ints[2] == c["nnz"] == 20224
    assert ints[3] == 20224 and ints[4] == c["sum_r2"] == 100104
    assert ints[5] == 5 and ints[6] == 3
    assert ints[7] == c["span"] == 516222
    assert ints[8] == c["cl"] == 12160
    assert ints[9] == 5 and ints[10] == 4096
    assert ints[27] == 1
    # histogram: lengths 3 -> bin 2 ([2,4)), 4 and 5 -> bin 3 ([4,8))
    assert ints[11 + 2] == 4 and ints[11 + 3] == 4092 and ints[11:27].sum() == 4096
    n = 4096
    mean = 20224 / 4096
    assert der[0] == 20224 / (4096.0 * 4096.0) == 0.0012054443359375
    assert der[1] == mean == 4.9375
    sd_direct = math.sqrt(sum((mean - r) ** 2 for r in [5] * 62 ** 2 + [4] * 248 + [3] * 4) / n)
    assert abs(der[2] - sd_direct) <= 1e-15 and der[2] == 0.2460627460628691
    assert der[3] == der[2] / mean
    assert der[4] == 5 - mean == 0.0625
    assert der[5] == 516222 / 4096 == 126.03076171875
    assert der[6] == 12160 / 4096 == 2.96875
    assert der[7] == 4096 * 5 / 20224 == der[8]
    assert list(f) == [4096, 4096, 20224, der[0], der[1], der[2], der[3], 5, 3, der[4],
                       der[5], der[6], der[7], 5, der[8]]


def test_lap1d_8(orc):
    ints, der, _ = orc.features(M.laplacian_1d(8))
    assert ints[2] == 22 and ints[5] == 3 and ints[6] == 2 and ints[9] == 3
    assert der[1] == 2.75 and abs(der[2] - math.sqrt(0.1875)) < 1e-16
    assert der[5] == 14 / 8 == 1.75 and der[6] == 2.75
    assert der[7] == der[8] == 24 / 22


def test_block_diagonal_8(orc):
    ints, der, _ = orc.features(M.block_diagonal(64, 1))
    assert ints[5] == ints[6] == 8 and der[1] == 8.0 and der[2] == 0.0
    assert ints[9] == 15 and der[6] == 8.0 and der[5] == 7.0
    assert der[7] == 1.0 and der[8] == 64 * 15 / 512


def brute_force(D_pattern, D_vals):
    """Features straight from the dense pattern, by the table's formulas."""
    n, m = D_pattern.shape
    r = D_pattern.sum(axis=1).astype(int)
    nnz = int(r.sum())
    spans, cls, hist = [], [], [0] * 16
    for i in range(n):
        cols = [j for j in range(m) if D_pattern[i, j]]
        spans.append(cols[-1] - cols[0] if cols else 0)
        best, run = 0, 0
        for t, j in enumerate(cols):
            run = run + 1 if t > 0 and j == cols[t - 1] + 1 else 1
            best = max(best, run)
        cls.append(best)
        hist[0 if r[i] == 0 else min(15, int(r[i]).bit_length())] += 1
    diags = {j - i for i in range(n) for j in range(m) if D_pattern[i, j]}
    mean = nnz / n
    sd = math.sqrt(sum((mean - ri) ** 2 for ri in r) / n)
    sym = int(n == m and np.array_equal(D_pattern, D_pattern.T)
              and np.array_equal(D_vals, D_vals.T))
    return dict(nnz=nnz, sum_r2=int((r * r).sum()), max=int(r.max()), min=int(r.min()),
                span=sum(spans), cl=sum(cls), ndiag=len(diags),
                diag=int(sum(D_pattern[i, i] for i in range(min(n, m)))), hist=hist, sym=sym,
                density=nnz / (n * m), mean=mean, sd=sd, cov=sd / mean if mean else 0.0,
                maxavg=r.max() - mean, distavg=sum(spans) / n, clusteravg=sum(cls) / n,
                fill=n * r.max() / nnz if nnz else 0.0,
                diagfill=n * len(diags) / nnz if nnz else 0.0)


@pytest.mark.parametrize("n,m,seed,dens", [(1, 1, 0, 1.0), (9, 13, 1, 0.3), (40, 40, 2, 0.15),
                                           (33, 20, 3, 0.5), (50, 70, 4, 0.05)])
def test_brute_force_tiny(orc, n, m, seed, dens):
    A = M.random_integer(n, m, seed, density=dens, long_rows=1, long_len=m)
    P = np.zeros((n, m), dtype=bool)
    V = np.zeros((n, m))
    for i in range(n):
        for k in range(A.rp[i], A.rp[i + 1]):
            P[i, A.col[k]] = True
            V[i, A.col[k]] = A.val[k]
    bf = brute_force(P, V)
    ints, der, _ = orc.features(A)
    assert ints[2] == bf["nnz"] == ints[3]
    assert ints[4] == bf["sum_r2"] and ints[5] == bf["max"] and ints[6] == bf["min"]
    assert ints[7] == bf["span"] and ints[8] == bf["cl"] and ints[9] == bf["ndiag"]
    assert ints[10] == bf["diag"] and list(ints[11:27]) == bf["hist"] and ints[27] == bf["sym"]
    for t, key in enumerate(["density", "mean", "sd", "cov", "maxavg", "distavg",
                             "clusteravg", "fill", "diagfill"]):
        assert abs(der[t] - bf[key]) <= 1e-13 * max(1.0, abs(bf[key])), key


def test_symmetry_flag(orc):
    A = M.random_integer(30, 30, 5, density=0.2)
    P = np.zeros((30, 30))
    for i in range(30):
        for k in range(A.rp[i], A.rp[i + 1]):
            P[i, A.col[k]] = A.val[k]
    S = P + P.T
    assert orc.features(M.from_dense(S))[0][27] == 1
    S2 = S.copy()
    i, j = np.argwhere(np.triu(S, 1) != 0)[0]
    S2[i, j] += 1.0
    assert orc.features(M.from_dense(S2))[0][27] == 0
    assert orc.features(M.convection_diffusion_2d(8))[0][27] == 0
    assert orc.features(M.random_integer(4, 5, 1))[0][27] == 0       # not square


def test_empty_and_degenerate(orc):
    ints, der, _ = orc.features(M.from_dense(np.zeros((4, 4))))
    assert ints[2] == 0 and ints[11] == 4 and ints[6] == 0 and ints[9] == 0
    assert list(der) == [0.0] * 9
    ints, der, _ = orc.features(M.from_dense(np.eye(1)))
    assert ints[8] == 1 and der[7] == 1.0


def test_invalid_csr_rejected(orc):
    A = M.laplacian_1d(6)
    bad = M.CSR(A.n, A.ncols, A.rp.copy(), A.col.copy(), A.val.copy())
    bad.col[3], bad.col[4] = bad.col[4], bad.col[3]                 # unsorted row
    assert orc.validate(bad) == orc.INVALID
    bad = M.CSR(A.n, A.ncols, A.rp.copy(), A.col.copy(), A.val.copy())
    bad.col[0] = 6                                                  # out of range
    assert orc.validate(bad) == orc.INVALID
    assert orc.validate(A) == orc.OK
