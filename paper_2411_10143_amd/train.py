"""Offline phase of the method (Section III-B): time every SpMV configuration
on a corpus of matrices, label each matrix per cascade stage, fit one
decision tree per stage and export the trees as the library's model file.

  collect : features (GPU kernels) + mean time of every configuration (the
            library's event-timed loop of back-to-back products) per matrix
  label   : stage 1 = format of the fastest configuration overall (CSR,
            ELL, COO, DIA or HYB);
            stage 2 = fastest CSR algorithm (vector at its best lane count,
            scalar, merge-path); stage 3 = fastest lane count.  Ties go to
            the lower configuration index.  With a perfect classifier the
            cascade therefore reaches the fastest configuration.
  fit     : a CART tree per stage (scikit-learn), exported as node tables;
            plus a "start" tree over the five inputs known without a pass
            over the entries (nrows, ncols, nnz, density, mean) that picks
            the configuration a solve starts from among those that need no
            copy of the matrix (ids 0..8): a regression tree on the log
            slowdowns log(t_c / min_{c<9} t) of all nine, whose leaf names
            the configuration with the smallest mean log slowdown over the
            leaf's matrices (the geometric-mean-optimal pick for the leaf;
            a classifier on the argmin labels instead ignores how much a
            wrong pick costs).

The corpus is synthetic (stencil, power-law, block-diagonal and uniform-random
families, disjoint seeds from the 48 held-out evaluation matrices, plus
Chung-Lu graph Laplacians, whose hub columns none of those families has),
timed on this GPU.

  python -m paper_2411_10143_amd.train collect --out data.csv [--count 200]
  python -m paper_2411_10143_amd.train retime --data data.csv --out new.csv --configs 11
  python -m paper_2411_10143_amd.train fit --data data.csv --model cascade_model.txt
"""
from __future__ import annotations

import argparse
import csv
import math
import os
import sys
import time

import numpy as np

FEATURES = ["nrows", "ncols", "nnz", "density", "mean", "sd", "cov", "max", "min", "maxavg",
            "distavg", "clusteravg", "fill", "ndiag", "diagfill"]
CONFIGS = 14
CSR_IDS = (0, 1, 2, 3, 4, 5, 6, 7, 8, 11)   # configurations stored in CSR (incl. CSR-panel)
FORMAT_OF = {9: 1, 10: 2, 12: 3, 13: 4}     # ELL, COO, DIA, HYB; every other id is CSR
KNOWN = 5                                   # inputs 0..4 need no pass over the entries
NO_COPY = 9                                 # ids 0..8 run on the CSR arrays as given


def reps_for(us_probe: float, budget_us: float = 4000.0, lo: int = 20, hi: int = 200) -> int:
    return int(min(hi, max(lo, budget_us / max(us_probe, 1e-3))))


def time_all_configs(ck, Mx, x, y, warmup=10, reps=None):
    """Mean us per product for each of the 14 configurations (inf if refused)."""
    out = []
    for cid in range(CONFIGS):
        cfg = ck.config_from_id(cid)
        try:
            ck.spmv_convert(Mx.handle, cfg)
        except ck.CkError as e:
            if e.status != ck.CK_E_UNSUPPORTED:
                raise
            out.append(math.inf)
            continue
        r = reps
        if r is None:
            probe = ck.time_spmv(Mx.handle, cfg, x, y, warmup=warmup, reps=5)
            r = reps_for(probe)
        out.append(ck.time_spmv(Mx.handle, cfg, x, y, warmup=2, reps=r))
    return out


def _first_within(t, tie):
    """Index of the first time within a factor (1 + tie) of the smallest."""
    t = np.asarray(t, dtype=np.float64)
    return int(np.nonzero(t <= t.min() * (1.0 + tie))[0][0])


def labels(times, tie=0.0):
    """(format, algorithm, log2 lanes) labels from the configuration times
    (ids: 0-6 CSR-vector lanes 1..64, 7 scalar, 8 merge, 9 ELL, 10 COO,
    11 CSR-panel, 12 DIA, 13 HYB; a time of inf marks a refused conversion).
    Times within a factor (1 + tie) of the fastest count as ties, and ties go
    to the lower configuration index (so HYB without a remainder, which runs
    the ELL kernel, is labelled ELL)."""
    t = np.full(CONFIGS, np.inf)
    t[:len(times)] = np.asarray(times, dtype=np.float64)
    best = _first_within(t, tie)
    fmt = FORMAT_OF.get(best, 0)
    lanes = _first_within(t[:7], tie)
    # candidates in configuration-index order: vector at its best lanes (id
    # 0..6), scalar (7), merge (8), panel (11)
    cand = [(t[int(np.argmin(t[:7]))], 1), (t[7], 0), (t[8], 2), (t[11], 3)]
    alg = cand[_first_within([c[0] for c in cand], tie)][1]
    return fmt, alg, lanes


def default_id(n, nnz):
    """Configuration id of the library's default: CSR-vector with
    clamp(2^floor(log2(max(1, nnz/n))), 2, 64) lanes."""
    q = max(1, nnz // n) if n > 0 else 1
    return min(max(int(q).bit_length() - 1, 1), 6)


def collect(out_csv, count=600, seed=9000, reps=None):
    import torch

    import paper_2411_10143_amd as ck
    from synth import workloads as W

    specs = W.training_specs(count=count, seed=seed)
    new = not os.path.exists(out_csv)
    done = set()
    if not new:
        with open(out_csv) as f:
            done = {row["name"] for row in csv.DictReader(f)}
    f = open(out_csv, "a", newline="")
    w = csv.writer(f)
    if new:
        w.writerow(["name", "family", "n", "nnz"] + FEATURES + [f"t{c}" for c in range(CONFIGS)])
    t0 = time.time()
    for i, spec in enumerate(specs):
        name, fam, k, n, s = spec
        if name in done:
            continue
        A = W.family_matrix(fam, k, n, s)
        Mx = ck.Matrix.from_csr(A)
        F = ck.spmv_features(Mx.handle)
        x = torch.from_numpy(np.random.default_rng(s).uniform(-1, 1, A.ncols)).cuda()
        y = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        times = time_all_configs(ck, Mx, x, y, reps=reps)
        Mx.close()
        del x, y
        w.writerow([name, fam, A.n, A.nnz] + [repr(v) for v in F.model_inputs()] +
                   [repr(v) for v in times])
        f.flush()
        best = int(np.argmin(times))
        print(f"[{i + 1}/{len(specs)}] {name} nnz={A.nnz} best={ck.CONFIG_NAMES[best]} "
              f"{min(times):.2f}us elapsed={time.time() - t0:.0f}s", flush=True)
    f.close()


def _gen_to_file(args):
    """Worker: draw one training matrix and save it (npz) for the timing process."""
    spec, path = args
    from synth import workloads as W
    name, fam, k, n, s = spec
    A = W.family_matrix(fam, k, n, s)
    np.savez(path, n=A.n, ncols=A.ncols, rp=A.rp, col=A.col, val=A.val)
    return path


def retime(in_csv, out_csv, configs, count=600, seed=9000, reps=None, jobs=8, tmpdir="/tmp"):
    """Re-time the given configuration ids of every matrix already in in_csv
    (after a kernel changed) and write the updated rows to out_csv; the
    matrices are drawn again by `jobs` worker processes."""
    import multiprocessing as mp
    import tempfile

    import torch

    import paper_2411_10143_amd as ck
    from synth import workloads as W
    from synth.matrices import CSR

    with open(in_csv) as f:
        rows = list(csv.DictReader(f))
    byname = {r["name"]: r for r in rows}
    specs = [sp for sp in W.training_specs(count=count, seed=seed) if sp[0] in byname]
    d = tempfile.mkdtemp(dir=tmpdir)
    work = [(sp, os.path.join(d, f"m{i}.npz")) for i, sp in enumerate(specs)]
    t0 = time.time()
    with mp.get_context("spawn").Pool(jobs) as pool:
        for i, path in enumerate(pool.imap(_gen_to_file, work)):
            name, fam, k, n, s = specs[i]
            z = np.load(path)
            A = CSR(int(z["n"]), int(z["ncols"]), z["rp"], z["col"], z["val"], name)
            os.remove(path)
            Mx = ck.Matrix.from_csr(A)
            x = torch.from_numpy(np.random.default_rng(s).uniform(-1, 1, A.ncols)).cuda()
            y = torch.zeros(A.n, dtype=torch.float64, device="cuda")
            for cid in configs:
                cfg = ck.config_from_id(cid)
                try:
                    ck.spmv_convert(Mx.handle, cfg)
                except ck.CkError as e:
                    if e.status != ck.CK_E_UNSUPPORTED:
                        raise
                    byname[name][f"t{cid}"] = repr(math.inf)
                    continue
                r = reps
                if r is None:
                    r = reps_for(ck.time_spmv(Mx.handle, cfg, x, y, warmup=10, reps=5))
                old = float(byname[name][f"t{cid}"])
                new = ck.time_spmv(Mx.handle, cfg, x, y, warmup=2, reps=r)
                byname[name][f"t{cid}"] = repr(new)
                print(f"[{i + 1}/{len(specs)}] {name} {ck.CONFIG_NAMES[cid]} {old:.2f} -> "
                      f"{new:.2f} us elapsed={time.time() - t0:.0f}s", flush=True)
            Mx.close()
            del x, y
    os.rmdir(d)
    with open(out_csv, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0].keys()))
        w.writeheader()
        for r in rows:
            w.writerow(r)


def load(path):
    X, T, names = [], [], []
    with open(path) as f:
        for row in csv.DictReader(f):
            X.append([float(row[k]) for k in FEATURES])
            # files written before a configuration existed lack its column
            T.append([float(row[f"t{c}"]) if f"t{c}" in row else math.inf
                      for c in range(CONFIGS)])
            names.append(row["name"])
    return np.array(X), np.array(T), names


def fit_trees(X, T, max_depth=8, min_leaf=2, seed=0, tie=0.0):
    """Three classifiers; stage-2/3 trees are trained on every matrix (the
    labels are defined for all of them), as the cascade may reach them."""
    from sklearn.tree import DecisionTreeClassifier
    Y = np.array([labels(t, tie) for t in T])
    # inputs as the library evaluates them: rounded to float32
    X32 = X.astype(np.float32)
    trees = []
    for stage in range(3):
        clf = DecisionTreeClassifier(max_depth=max_depth, min_samples_leaf=min_leaf,
                                     random_state=seed)
        clf.fit(X32, Y[:, stage])
        trees.append(clf)
    return trees, Y


def fit_start(X, T, max_depth=8, min_leaf=3, seed=0):
    from sklearn.tree import DecisionTreeRegressor
    t = np.asarray(T, dtype=np.float64)[:, :NO_COPY]
    slow = np.log(t / t.min(axis=1, keepdims=True))
    reg = DecisionTreeRegressor(max_depth=max_depth, min_samples_leaf=min_leaf,
                                random_state=seed)
    reg.fit(X[:, :KNOWN].astype(np.float32), slow)
    return reg


def start_predict(reg, X):
    """Configuration ids (0..8) the start tree picks for feature rows."""
    return np.argmin(reg.predict(np.asarray(X)[:, :KNOWN].astype(np.float32)), axis=1)


def export(trees, path, note=""):
    names = ["format", "algorithm", "lanes", "start"][:len(trees)]
    with open(path, "w") as f:
        f.write("# caskrylov cascade model: CART trees fitted on MI355X SpMV timings\n")
        if note:
            f.write(f"# {note}\n")
        f.write("# node: feature threshold(hex) left right class; features in feature-table "
                "order:\n# " + " ".join(f"{i} {n}" for i, n in enumerate(FEATURES)) + "\n")
        for name, clf in zip(names, trees):
            tr = clf.tree_
            f.write(f"tree {name} {tr.node_count}\n")
            for t in range(tr.node_count):
                leaf = tr.children_left[t] < 0
                if not leaf:
                    cls = -1
                elif hasattr(clf, "classes_"):       # classifier: majority class
                    cls = int(clf.classes_[int(np.argmax(tr.value[t, 0, :]))])
                else:                                # start tree: smallest mean log slowdown
                    cls = int(np.argmin(tr.value[t, :, 0]))
                feat = -1 if leaf else int(tr.feature[t])
                thr = 0.0 if leaf else float(tr.threshold[t])
                f.write(f"{feat} {thr.hex()} {int(tr.children_left[t])} "
                        f"{int(tr.children_right[t])} {cls}\n")


def cascade_predict(trees, x):
    """Configuration id the cascade picks for one feature row (sklearn side)."""
    x = np.asarray(x, dtype=np.float32)[None, :]
    fmt = int(trees[0].predict(x)[0])
    if fmt != 0:
        return {1: 9, 2: 10, 3: 12, 4: 13}[fmt]
    alg = int(trees[1].predict(x)[0])
    if alg == 0:
        return 7
    if alg == 2:
        return 8
    if alg == 3:
        return 11
    return int(trees[2].predict(x)[0])


def main(argv=None):
    p = argparse.ArgumentParser()
    sub = p.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--out", required=True)
    c.add_argument("--count", type=int, default=600)
    c.add_argument("--seed", type=int, default=9000)
    c.add_argument("--reps", type=int, default=None)
    r = sub.add_parser("retime")
    r.add_argument("--data", required=True)
    r.add_argument("--out", required=True)
    r.add_argument("--configs", type=int, nargs="+", required=True)
    r.add_argument("--count", type=int, default=600)
    r.add_argument("--seed", type=int, default=9000)
    r.add_argument("--reps", type=int, default=None)
    r.add_argument("--jobs", type=int, default=8)
    fa = sub.add_parser("fit")
    fa.add_argument("--data", required=True, nargs="+")
    fa.add_argument("--model", required=True)
    fa.add_argument("--max-depth", type=int, default=5)
    fa.add_argument("--min-leaf", type=int, default=1)
    fa.add_argument("--start-depth", type=int, default=8)
    fa.add_argument("--start-min-leaf", type=int, default=3)
    fa.add_argument("--tie", type=float, default=0.02,
                    help="times within this fraction of the fastest count as ties")
    a = p.parse_args(argv)
    if a.cmd == "collect":
        collect(a.out, a.count, a.seed, a.reps)
    elif a.cmd == "retime":
        retime(a.data, a.out, a.configs, a.count, a.seed, a.reps, a.jobs)
    else:
        Xs, Ts = [], []
        for d in a.data:
            X, T, _ = load(d)
            Xs.append(X)
            Ts.append(T)
        X, T = np.concatenate(Xs), np.concatenate(Ts)
        trees, Y = fit_trees(X, T, a.max_depth, a.min_leaf, tie=a.tie)
        start = fit_start(X, T, a.start_depth, a.start_min_leaf)
        picks = np.array([cascade_predict(trees, x) for x in X])
        rows = np.arange(len(T))
        slow = T[rows, picks] / T.min(axis=1)
        s_pick = start_predict(start, X)
        d_pick = np.array([default_id(int(x[0]), int(x[2])) for x in X])
        gm = lambda r: math.exp(np.mean(np.log(r)))
        best9 = T[:, :NO_COPY].min(axis=1)
        note = (f"{len(X)} training matrices; training-set geomean t_pred/t_best = "
                f"{gm(slow):.4f}; start tree vs the best of ids 0..8 {gm(T[rows, s_pick] / best9):.4f} "
                f"(default rule {gm(T[rows, d_pick] / best9):.4f})")
        export(trees + [start], a.model, note)
        print(note)


if __name__ == "__main__":
    sys.exit(main())
