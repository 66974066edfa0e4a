"""The C-ABI library loads without a GPU and exports every declared symbol."""
import ctypes
import glob
import os
import re

from helpers import ROOT

LIB = os.path.join(ROOT, "paper_2411_10143_amd", "libcaskrylov.so")


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w]*\s*\**\s+\**(\w+)\s*\(", text,
                             flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


def ensure_built():
    if not os.path.exists(LIB):
        from paper_2411_10143_amd import build
        build.build()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["spmv_create", "spmv_features", "spmv_select", "spmv_convert", "spmv_apply",
              "cg_solve", "gmres_solve", "spmv_destroy", "ck_last_error"]:
        assert n in names, n


def test_library_exports_every_declared_symbol():
    ensure_built()
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_host_only_calls_work_without_gpu():
    ensure_built()
    import paper_2411_10143_amd as ck
    for i in range(ck.NUM_CONFIGS):
        c = ck.config_from_id(i)
        assert ck.config_id(c) == i
        assert ck.kernel_name(c).startswith("spmv_")
    try:
        ck.config_from_id(ck.NUM_CONFIGS)
        raise AssertionError("expected an error")
    except ck.CkError as e:
        assert e.status == ck.CK_E_INVALID
    f = ck.Features()
    f.nrows, f.ncols, f.nnz = 100, 100, 500
    c = ck.spmv_select(f)
    assert c.format in (0, 1, 2, 3, 4) and 1 <= c.stages_done <= 3


def test_library_cascade_equals_oracle_on_training_features(orc):
    """The library's host-side cascade (spmv_select / ck_select_stages /
    ck_eval_stage) against the oracle's tree walk over the shipped model, on
    the 600 feature rows of the shipped training timings (every format class
    the model can output)."""
    ensure_built()
    import csv
    import paper_2411_10143_amd as ck
    from helpers import MODEL, parse_model
    from paper_2411_10143_amd import train
    trees = parse_model(MODEL)
    path = os.path.join(ROOT, "paper_2411_10143_amd", "training", "mi355x_spmv_timings.csv")
    seen = set()
    for row in csv.DictReader(open(path)):
        f15 = [float(row[k]) for k in train.FEATURES]
        F = ck.Features.from_model_inputs(f15)
        want = orc.cascade(trees, f15)
        assert ck.select_stages(F) == want, row["name"]
        assert [ck.eval_stage(F, t) for t in range(3)] == \
            [orc.tree_eval(trees[t], f15) for t in range(3)]
        c = ck.spmv_select(F)
        assert c.format == want[0] and c.stages_done == sum(1 for v in want if v >= 0)
        seen.add(want[0])
    assert {0, 1, 3} <= seen, seen


def test_start_config_equals_oracle_tree_walk(orc):
    """The known-inputs start tree (ck_start_config): the library, deriving
    density and mean from (nrows, ncols, nnz) itself, against the oracle's
    walk of the shipped start tree over the stored feature rows; every pick
    is a configuration that needs no copy of the matrix."""
    ensure_built()
    import csv
    import paper_2411_10143_amd as ck
    from helpers import MODEL, parse_start_tree
    from paper_2411_10143_amd import train
    start = parse_start_tree(MODEL)
    assert start is not None and max(f for f in start["feature"]) < train.KNOWN
    path = os.path.join(ROOT, "paper_2411_10143_amd", "training", "mi355x_spmv_timings.csv")
    seen = set()
    for row in csv.DictReader(open(path)):
        f15 = [float(row[k]) for k in train.FEATURES]
        want = orc.tree_eval(start, f15)
        c, from_tree = ck.start_config(int(f15[0]), int(f15[1]), int(f15[2]))
        assert from_tree and ck.config_id(c) == want, row["name"]
        assert 0 <= want < train.NO_COPY
        seen.add(want)
    assert len(seen) >= 3, seen
    c, from_tree = ck.start_config(0, 0, 0)
    assert not from_tree


def test_start_tree_optional_and_checked(tmp_path):
    ensure_built()
    import paper_2411_10143_amd as ck
    from helpers import MODEL, parse_model, write_model
    from paper_2411_10143_amd import train
    trees = parse_model(MODEL)
    plain = str(tmp_path / "three.txt")
    write_model(plain, trees)
    for n, nnz in [(1000, 9000), (1000, 0), (1000, 1999), (1000, 2000), (7, 7 * 64),
                   (5, 5 * 1000), (3, 2), (1 << 20, 17 << 20)]:
        c, from_tree = ck.start_config(n, n, nnz, model_path=plain)   # the default rule
        assert not from_tree and ck.config_id(c) == train.default_id(n, nnz), (n, nnz)
    leaf = dict(feature=[-1], threshold=[0.0], left=[-1], right=[-1], cls=[8])
    ok = str(tmp_path / "leaf.txt")
    write_model(ok, trees + [leaf])
    c, from_tree = ck.start_config(1000, 1000, 9000, model_path=ok)
    assert from_tree and ck.config_id(c) == 8
    for bad_tree in (dict(feature=[5, -1, -1], threshold=[1.0, 0.0, 0.0], left=[1, -1, -1],
                          right=[2, -1, -1], cls=[-1, 0, 1]),     # a gathered input
                     dict(leaf, cls=[9])):                        # ELL needs a copy
        bad = str(tmp_path / "bad.txt")
        write_model(bad, trees + [bad_tree])
        try:
            ck.start_config(1000, 1000, 9000, model_path=bad)
            raise AssertionError("expected a malformed-model error")
        except ck.CkError as e:
            assert e.status == ck.CK_E_INVALID


def test_overhead_gate_rule_on_host():
    """The overhead-aware conversion rule: exact geometric extrapolation, the
    no-decay and converged cases, cost ordering, and the 0.25 * R >= cost
    threshold."""
    ensure_built()
    import math
    import paper_2411_10143_amd as ck
    F = ck.Features.from_model_inputs([1e6, 1e6, 7e6, 7e-6, 7.0, 0.0, 0.0, 7, 7, 0.0, 2e4,
                                       3.0, 1.0, 7, 7e-6])
    dia = ck.config_from_id(ck.ID_DIA)
    q = 0.5
    rem, cost, _ = ck.overhead_gate(F, dia, 2, q ** 2, 6, q ** 6, q ** 30)
    assert abs(rem - 2 * 24.0) < 1e-9          # twice the geometric extrapolation
    assert ck.overhead_gate(F, dia, 2, 0.1, 6, 0.2, 1e-10)[0] == 1e9      # residual grew
    assert ck.overhead_gate(F, dia, 2, 0.1, 6, 1e-11, 1e-10)[0] == 0.0    # already converged
    coo = ck.overhead_gate(F, ck.config_from_id(10), 2, 0.5, 6, 0.1, 1e-10)[1]
    ell = ck.overhead_gate(F, ck.config_from_id(ck.ID_ELL), 2, 0.5, 6, 0.1, 1e-10)[1]
    assert 2.0 < coo < ell < cost
    # threshold: convert iff 0.25 * remaining >= cost
    for want_rem in (cost * 4 * 0.9, cost * 4 * 1.1):
        t1 = 10
        r1 = 1e-3
        r0 = r1 * math.exp(-2 * 10 * math.log(1e-10 / r1) / want_rem)   # from t0 = 0
        rem, c2, go = ck.overhead_gate(F, dia, 0, r0, t1, r1, 1e-10)
        assert abs(rem - want_rem) < 1e-6 * want_rem and c2 == cost
        assert go == (0.25 * rem >= cost)
