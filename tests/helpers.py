"""Shared test helpers: device upload, oracle-side bounds, model parsing."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MODEL = os.path.join(ROOT, "paper_2411_10143_amd", "cascade_model.txt")


def say(*a):
    """Name the case before a GPU step (flushed so it survives a crash)."""
    print(*a, flush=True)
    sys.stdout.flush()


def upload(A):
    import torch
    return (torch.from_numpy(A.rp).cuda(), torch.from_numpy(A.col).cuda(),
            torch.from_numpy(A.val).cuda())


def abs_csr(A):
    from synth.matrices import CSR
    return CSR(A.n, A.ncols, A.rp, A.col, np.abs(A.val))


def spmv_bound(orc, A, x, alpha, beta, y0, u, k_extra=2):
    """Per-row bound (r_i + k_extra) * u * (|alpha| sum_j |a_ij x_j| + |beta y0_i|)."""
    s = orc.spmv(abs_csr(A), np.abs(x))
    r = np.diff(A.rp.astype(np.int64)).astype(np.float64)
    mag = abs(alpha) * s + (abs(beta) * np.abs(y0) if beta != 0 else 0.0)
    return (r + k_extra) * u * mag + 1e-300


def parse_model(path=MODEL):
    """Read the cascade model text into three oracle tree dicts."""
    trees, cur = {}, None
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        parts = line.split()
        if parts[0] == "tree":
            cur = parts[1]
            trees[cur] = dict(feature=[], threshold=[], left=[], right=[], cls=[])
            continue
        t = trees[cur]
        t["feature"].append(int(parts[0]))
        t["threshold"].append(float.fromhex(parts[1]))
        t["left"].append(int(parts[2]))
        t["right"].append(int(parts[3]))
        t["cls"].append(int(parts[4]))
    return [trees["format"], trees["algorithm"], trees["lanes"]]


def parse_start_tree(path=MODEL):
    """The model's optional start tree (None if it has none)."""
    trees, cur = {}, None
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        parts = line.split()
        if parts[0] == "tree":
            cur = parts[1]
            trees[cur] = dict(feature=[], threshold=[], left=[], right=[], cls=[])
            continue
        for k, v in zip(("feature", "threshold", "left", "right", "cls"), parts):
            trees[cur][k].append(float.fromhex(v) if k == "threshold" else int(v))
    return trees.get("start")


def write_model(path, trees):
    names = ["format", "algorithm", "lanes", "start"][:len(trees)]
    with open(path, "w") as f:
        f.write("# test model\n")
        for name, t in zip(names, trees):
            f.write(f"tree {name} {len(t['feature'])}\n")
            for i in range(len(t["feature"])):
                f.write(f"{t['feature'][i]} {float(t['threshold'][i]).hex()} {t['left'][i]} "
                        f"{t['right'][i]} {t['cls'][i]}\n")


def sk_tree(clf):
    tr = clf.tree_
    leaf = tr.children_left < 0
    cls = np.where(leaf, clf.classes_[np.argmax(tr.value[:, 0, :], axis=1)], -1)
    return dict(feature=np.where(leaf, -1, tr.feature).astype(int).tolist(),
                threshold=[float(v) for v in tr.threshold],
                left=tr.children_left.astype(int).tolist(),
                right=tr.children_right.astype(int).tolist(),
                cls=cls.astype(int).tolist())
