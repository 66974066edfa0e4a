"""Pins for the oracle conversions (ELL, COO) and decision-tree cascade."""
import numpy as np
import pytest

from synth import matrices as M


def dense_csr(A):
    D = np.zeros((A.n, A.ncols))
    for i in range(A.n):
        D[i, A.col[A.rp[i]:A.rp[i + 1]]] = A.val[A.rp[i]:A.rp[i + 1]]
    return D


@pytest.mark.parametrize("maker", [lambda: M.laplacian_2d(10), lambda: M.block_diagonal(70, 3),
                                   lambda: M.random_integer(100, 90, 4, density=0.05),
                                   lambda: M.banded_stencil(1000, 27, 5)])
def test_ell_round_trip_and_layout(orc, maker):
    A = maker()
    st, K, pitch, ec, ev = orc.to_ell(A)
    assert st == orc.OK
    r = np.diff(A.rp)
    assert K == r.max() and pitch % 64 == 0 and pitch >= A.n > pitch - 64
    E = np.zeros((A.n, A.ncols))
    for s in range(K):
        for i in range(pitch):
            c = ec[s * pitch + i]
            if i >= A.n or s >= r[i]:
                assert c == -1 and ev[s * pitch + i] == 0.0
                assert not np.signbit(ev[s * pitch + i])
            else:
                E[i, c] = ev[s * pitch + i]
    assert np.array_equal(E, dense_csr(A))


def test_ell_refused_for_skewed_rows(orc):
    A = M.power_law_rows(20000, 1.5, 1)
    st, K, pitch, _, _ = orc.to_ell(A)
    assert st == orc.UNSUPPORTED and K * pitch > 8 * A.nnz


def test_coo_rows_round_trip(orc):
    A = M.random_integer(200, 150, 6, density=0.05, empty_rows=0.3)
    row = orc.to_coo_rows(A)
    assert np.all(np.diff(row) >= 0)
    rp = np.zeros(A.n + 1, dtype=np.int64)
    np.cumsum(np.bincount(row, minlength=A.n), out=rp[1:])
    assert np.array_equal(rp, A.rp)


def tree(feature, threshold, left, right, cls):
    return dict(feature=feature, threshold=threshold, left=left, right=right, cls=cls)


def test_hand_built_tree_and_float_cast(orc):
    # root: feature 4 (mean) <= 5.5 -> leaf 1, else leaf 2
    t = tree([4, -1, -1], [5.5, 0, 0], [1, -1, -1], [2, -1, -1], [-1, 7, 9])
    f = np.zeros(15)
    f[4] = 5.5
    assert orc.tree_eval(t, f) == 7
    f[4] = 5.501
    assert orc.tree_eval(t, f) == 9
    # a value above the threshold in double but equal to it after the float cast
    thr = float(np.float32(0.1))
    t2 = tree([3, -1, -1], [thr, 0, 0], [1, -1, -1], [2, -1, -1], [-1, 1, 2])
    f[3] = np.nextafter(thr, 1.0)
    assert f[3] > thr and float(np.float32(f[3])) == thr
    assert orc.tree_eval(t2, f) == 1


def sk_to_tree(clf):
    tr = clf.tree_
    cls = np.where(tr.children_left < 0, clf.classes_[np.argmax(tr.value[:, 0, :], axis=1)], -1)
    return tree(np.where(tr.children_left < 0, -1, tr.feature).astype(np.int32),
                tr.threshold.astype(np.float64), tr.children_left.astype(np.int32),
                tr.children_right.astype(np.int32), cls.astype(np.int32))


def test_matches_sklearn_predict(orc):
    from sklearn.tree import DecisionTreeClassifier
    rng = np.random.default_rng(0)
    X = np.exp(rng.normal(0, 3, size=(400, 15)))
    y = ((X[:, 4] > 3) * 1 + (X[:, 10] > X[:, 2] / 100) * 2 + (X[:, 0] > 50)) % 5
    clf = DecisionTreeClassifier(max_depth=7, random_state=0).fit(X, y)
    t = sk_to_tree(clf)
    Xt = np.exp(rng.normal(0, 3, size=(2000, 15)))
    Xt[:50] = X[:50]
    pred = clf.predict(Xt)
    mine = [orc.tree_eval(t, x) for x in Xt]
    assert np.array_equal(pred, mine)


def test_cascade_gating(orc):
    def const(c):
        return tree([-1], [0.0], [-1], [-1], [c])
    f = np.zeros(15)
    assert orc.cascade([const(1), const(1), const(3)], f) == [1, -1, -1]
    assert orc.cascade([const(2), const(1), const(3)], f) == [2, -1, -1]
    assert orc.cascade([const(0), const(0), const(3)], f) == [0, 0, -1]
    assert orc.cascade([const(0), const(2), const(3)], f) == [0, 2, -1]
    assert orc.cascade([const(0), const(1), const(3)], f) == [0, 1, 3]
