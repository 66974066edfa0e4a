"""Offline trainer (CPU): labels follow the stated rule, and an exported model
evaluates like scikit-learn's predict under the oracle's tree walk."""
import math

import numpy as np

from helpers import parse_model
from paper_2411_10143_amd import train


def test_labels_rule_and_ties():
    inf = math.inf
    # fastest overall is CSR-vector with 8 lanes (id 3)
    t = [9, 8, 7, 1.0, 2, 3, 4, 5, 6, 7, 8]
    assert train.labels(t) == (0, 1, 3)
    # ELL fastest overall; CSR algorithm and lanes labels still defined
    t = [9, 8, 7, 3, 2.5, 3, 4, 2.0, 6, 1.0, 8]
    assert train.labels(t) == (1, 0, 4)
    # COO fastest, merge fastest CSR algorithm, ELL refused (inf)
    t = [9, 8, 7, 6, 5, 4, 4, 5, 3.0, inf, 1.0]
    assert train.labels(t) == (2, 2, 5)
    # ties go to the lower configuration index
    t = [2.0, 2.0, 3, 3, 3, 3, 3, 2.0, 2.0, 2.0, 2.0]
    assert train.labels(t) == (0, 1, 0)
    # CSR-panel (id 11) fastest: a CSR format label and algorithm class 3
    t = [9, 8, 7, 6, 5, 4, 4, 5, 3.0, 8, 2.0, 1.0]
    assert train.labels(t) == (0, 3, 5)
    # DIA (id 12) and HYB (id 13) fastest: format classes 3 and 4
    t = [9, 8, 7, 6, 5, 4, 4, 5, 3.0, 8, 2.0, 1.5, 1.0, 1.2]
    assert train.labels(t) == (3, 3, 5)
    t = [9, 8, 7, 6, 5, 4, 4, 5, 3.0, 8, 2.0, 1.5, inf, 1.0]
    assert train.labels(t) == (4, 3, 5)


def test_export_round_trip_matches_sklearn(orc, tmp_path):
    rng = np.random.default_rng(0)
    X = np.exp(rng.normal(0, 2, size=(300, 15)))
    T = rng.uniform(1, 10, size=(300, 14))
    T[X[:, 4] > 3, 9] = 0.5          # make ELL win on part of the data
    T[X[:, 6] > 5, 8] = 0.4          # merge on another part
    T[X[:, 2] > 20, 12] = 0.3        # DIA and HYB on others
    T[X[:, 9] < 0.05, 13] = 0.2
    trees, Y = train.fit_trees(X, T, max_depth=6)
    path = tmp_path / "model.txt"
    train.export(trees, str(path))
    parsed = parse_model(str(path))
    Xt = np.exp(rng.normal(0, 2, size=(500, 15)))
    for x in Xt:
        stages = orc.cascade(parsed, x)
        cid = train.cascade_predict(trees, x)
        if stages[0] != 0:
            assert cid == {1: 9, 2: 10, 3: 12, 4: 13}[stages[0]]
        elif stages[1] == 0:
            assert cid == 7
        elif stages[1] == 2:
            assert cid == 8
        elif stages[1] == 3:
            assert cid == 11
        else:
            assert cid == stages[2]


def test_shipped_model_is_well_formed():
    from helpers import MODEL
    trees = parse_model(MODEL)
    for t in trees:
        n = len(t["feature"])
        for i in range(n):
            if t["feature"][i] >= 0:
                assert 0 <= t["feature"][i] < 15
                assert i < t["left"][i] < n and i < t["right"][i] < n
    assert {c for c in trees[0]["cls"] if c >= 0} <= {0, 1, 2, 3, 4}
    assert {c for c in trees[1]["cls"] if c >= 0} <= {0, 1, 2, 3}
    assert {c for c in trees[2]["cls"] if c >= 0} <= set(range(7))


def test_start_tree_export_matches_sklearn_and_minimises_leaf_slowdown(orc, tmp_path):
    """The start tree exported as a node table picks, under the oracle's tree
    walk, what the fitted regressor's argmin picks; on its own training rows
    each leaf's pick has the smallest geometric-mean slowdown of the nine."""
    from helpers import parse_start_tree
    rng = np.random.default_rng(1)
    X = np.exp(rng.normal(0, 2, size=(400, 15)))
    T = rng.uniform(1, 10, size=(400, 14))
    T[X[:, 2] > 5, 8] = 0.5             # merge wins for large nnz
    T[X[:, 4] < 0.3, 7] = 0.4           # scalar for short rows
    T[X[:, 0] > 20, 3] = 0.3
    trees, _ = train.fit_trees(X, T, max_depth=3)
    reg = train.fit_start(X, T, max_depth=4, min_leaf=3)
    path = tmp_path / "model.txt"
    train.export(trees + [reg], str(path))
    start = parse_start_tree(str(path))
    assert max(start["feature"]) < train.KNOWN
    want = train.start_predict(reg, X)
    got = np.array([orc.tree_eval(start, x) for x in X])
    assert np.array_equal(got, want)
    leaf = reg.apply(X[:, :train.KNOWN].astype(np.float32))
    slow = np.log(T[:, :train.NO_COPY] / T[:, :train.NO_COPY].min(axis=1, keepdims=True))
    for l in np.unique(leaf):
        rows = leaf == l
        assert slow[rows].mean(axis=0).argmin() == got[rows][0]
        assert np.all(got[rows] == got[rows][0])
