"""Pins for the oracle's DIA and HYB conversions (the DIA and HYB formats of
the configuration space, Section III-B-2): closed-form layouts of stencil
matrices, hand-worked HYB widths at the rule's boundary, and brute-force
round trips on small random patterns."""
import numpy as np
import pytest

from synth import matrices as M


def dense_csr(A):
    D = np.zeros((A.n, A.ncols))
    for i in range(A.n):
        D[i, A.col[A.rp[i]:A.rp[i + 1]]] = A.val[A.rp[i]:A.rp[i + 1]]
    return D


def csr_with_lengths(lengths, ncols=None):
    """Row i holds columns 0..r_i-1 with value 100*i + k + 1 (distinct, nonzero)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    n = lengths.shape[0]
    ncols = int(lengths.max()) if ncols is None else ncols
    rows = np.repeat(np.arange(n), lengths)
    cols = np.concatenate([np.arange(r) for r in lengths]) if n else np.zeros(0, np.int64)
    vals = 100.0 * rows + cols + 1.0
    return M._finish(n, max(ncols, 1), rows, cols, vals, "lengths", presorted=True)


def test_dia_tridiagonal_closed_form(orc):
    n = 100
    A = M.laplacian_1d(n)
    st, nd, pitch, off, dv = orc.to_dia(A)
    assert st == orc.OK and nd == 3 and pitch == 128
    assert list(off) == [-1, 0, 1]
    sub, main, sup = (dv[d * pitch:(d + 1) * pitch] for d in range(3))
    assert sub[0] == 0.0 and np.all(sub[1:n] == -1.0)
    assert np.all(main[:n] == 2.0)
    assert np.all(sup[:n - 1] == -1.0) and sup[n - 1] == 0.0
    for d in (sub, main, sup):             # rows n..pitch-1 are +0.0 padding
        assert np.all(d[n:] == 0.0) and not np.any(np.signbit(d[n:]))


def test_dia_2d_laplacian_offsets(orc):
    N = 12
    A = M.laplacian_2d(N)
    st, nd, pitch, off, dv = orc.to_dia(A)
    assert st == orc.OK and list(off) == [-N, -1, 0, 1, N]
    # the +-1 diagonals break at the grid-line ends: row i = a*N (a >= 1) has
    # no west neighbour, so its slot on offset -1 is padding
    west = dv[1 * pitch:2 * pitch]
    for a in range(1, N):
        assert west[a * N] == 0.0
        assert west[a * N + 1] == -1.0


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_dia_round_trip_random(orc, seed):
    A = M.random_integer(90, 70, seed, density=0.04, empty_rows=0.2)
    st, nd, pitch, off, dv = orc.to_dia(A)
    rows = np.repeat(np.arange(A.n), np.diff(A.rp))
    expect = np.unique(A.col.astype(np.int64) - rows)
    assert nd == expect.shape[0] and np.array_equal(off, expect)
    if st != orc.OK:
        assert nd * pitch > 8 * A.nnz
        return
    D = np.zeros((A.n, A.ncols))
    stored = set(zip(rows.tolist(), A.col.tolist()))
    for d, o in enumerate(off):
        for i in range(pitch):
            v = dv[d * pitch + i]
            j = i + o
            if i < A.n and 0 <= j < A.ncols and (i, j) in stored:
                D[i, j] = v
            else:
                assert v == 0.0 and not np.signbit(v)
    assert np.array_equal(D, dense_csr(A))


def test_dia_keeps_stored_zeros_bit_for_bit_and_matches_ndiag_feature(orc):
    A = M.laplacian_1d(64)
    A.val = A.val.copy()
    A.val[A.rp[5]] = -0.0                    # row 5's sub-diagonal entry: stored -0.0
    A.val[A.rp[7] + 1] = 0.0                 # row 7's main-diagonal entry: stored +0.0
    st, nd, pitch, off, dv = orc.to_dia(A)
    assert st == orc.OK and list(off) == [-1, 0, 1]
    assert dv[0 * pitch + 5] == 0.0 and np.signbit(dv[0 * pitch + 5])
    assert dv[1 * pitch + 7] == 0.0 and not np.signbit(dv[1 * pitch + 7])
    assert dv[0 * pitch + 6] == -1.0 and dv[2 * pitch + 7] == -1.0
    ints = orc.features(M.block_diagonal(64, 1))[0]
    st, nd, _, _ = orc.dia_shape(M.block_diagonal(64, 1))
    assert nd == ints[9] == 15              # 8x8 blocks: offsets -7..7


def test_dia_fill_limit_boundary(orc):
    # n = 64 (pitch 64): 8 diagonals and 64 entries sit exactly on the limit
    # ndiag * pitch = 8 * nnz; one more entry on a new diagonal crosses it
    rows = list(range(57)) + [0] * 7
    cols = list(range(57)) + list(range(1, 8))
    vals = [1.0] * 64
    A = M._finish(64, 64, rows, cols, vals, "edge")
    st, nd, pitch, _ = orc.dia_shape(A)
    assert (st, nd, pitch, A.nnz) == (orc.OK, 8, 64, 64)
    B = M._finish(64, 64, rows + [0], cols + [8], vals + [1.0], "edge+1")
    st, nd, pitch, _ = orc.dia_shape(B)
    assert (st, nd, B.nnz) == (orc.UNSUPPORTED, 9, 65)


def test_dia_refused_for_random_pattern(orc):
    A = M.uniform_random(4000, 3)
    st, nd, pitch, off = orc.dia_shape(A)
    assert st == orc.UNSUPPORTED and nd * pitch > 8 * A.nnz


@pytest.mark.parametrize("lengths,K", [
    ([0, 1, 2, 3, 4, 5], 4),                 # 3 * #{r >= 4} = 6 >= 6, #{r >= 5} = 1
    ([7] * 10, 7),                           # constant rows: HYB = ELL
    ([1] * 20 + [10] * 10, 10),              # exactly a third of the rows are long
    ([1] * 21 + [10] * 9, 1),                # one long row fewer: K drops to 1
    ([0] * 5, 0),                            # empty rows
])
def test_hyb_width_worked_examples(orc, lengths, K):
    A = csr_with_lengths(lengths)
    assert orc.hyb_width(A) == K
    K2, pitch, ec, ev, tr = orc.to_hyb(A)
    assert K2 == K
    assert list(tr) == [i for i, r in enumerate(lengths) if r > K]


@pytest.mark.parametrize("seed", [4, 5])
def test_hyb_round_trip(orc, seed):
    A = M.random_integer(120, 80, seed, density=0.05, empty_rows=0.1, long_rows=6, long_len=60)
    K, pitch, ec, ev, tr = orc.to_hyb(A)
    r = np.diff(A.rp)
    assert 3 * np.sum(r >= K) >= A.n and 3 * np.sum(r >= K + 1) < A.n
    assert np.array_equal(tr, np.nonzero(r > K)[0])
    E = np.zeros((A.n, A.ncols))
    for s in range(K):
        for i in range(pitch):
            c, v = ec[s * pitch + i], ev[s * pitch + i]
            if i < A.n and s < r[i]:
                assert c == A.col[A.rp[i] + s] and v == A.val[A.rp[i] + s]
                E[i, c] = v
            else:
                assert c == -1 and v == 0.0 and not np.signbit(v)
    for i in tr:                              # the remainder stays in the CSR arrays
        for k in range(A.rp[i] + K, A.rp[i + 1]):
            E[i, A.col[k]] = A.val[k]
    assert np.array_equal(E, dense_csr(A))
