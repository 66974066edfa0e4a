"""GPU parity of the SpMV family, features, conversions and the cascade,
through the C ABI, against the CPU oracle on the same seeded inputs."""
import numpy as np
import pytest

from helpers import MODEL, parse_model, say, sk_tree, spmv_bound, upload, write_model
from synth import matrices as M

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def ck():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_10143_amd as ck
    ck.lib()
    return ck


CASES = {
    "int_ragged": lambda: M.random_integer(3001, 2800, 1, density=0.004, empty_rows=0.2,
                                           long_rows=3, long_len=2500),
    "int_wide": lambda: M.random_integer(700, 9000, 2, density=0.01, empty_rows=0.0),
    # four rows of 20,000 entries: each spans about ten merge-path workgroups
    # and every wave of them (the carry runs across waves and workgroups)
    "int_hub": lambda: M.random_integer(2000, 40000, 9, density=0.0005, empty_rows=0.1,
                                        long_rows=4, long_len=20000),
    "powerlaw": lambda: M.power_law_rows(20011, 1.6, 3),
    "banded27": lambda: M.banded_stencil(30011, 27, 4),
    "banded9": lambda: M.banded_stencil(5003, 9, 5),
    "banded13": lambda: M.banded_stencil(7001, 13, 6),
    "banded19": lambda: M.banded_stencil(9001, 19, 7),
    "blockdiag": lambda: M.block_diagonal(10007, 5),
    "uniform": lambda: M.uniform_random(50003, 6),
    "lap1d": lambda: M.laplacian_1d(5003),
    "lap2d_64": lambda: M.laplacian_2d(64),
    "lap3d_12": lambda: M.laplacian_3d(12),
    "convdiff": lambda: M.convection_diffusion_2d(100, 10.0),
    "empty": lambda: M.from_dense(np.zeros((5, 7))),
    "one_by_one": lambda: M.from_dense(np.array([[3.0]])),
    "single_row": lambda: M.from_dense(np.arange(1.0, 200.0)[None, :]),
    "single_col": lambda: M.from_dense(np.arange(1.0, 300.0)[:, None]),
    "column_runs": lambda: M.column_runs(1500, 6000, 8),
}

_cache = {}


def case(name):
    if name not in _cache:
        _cache[name] = CASES[name]()
    return _cache[name]


def is_int(A):
    return np.all(A.val == np.round(A.val))


@pytest.mark.parametrize("name", list(CASES))
def test_spmv_all_configs_fp64(ck, orc, name):
    import torch
    A = case(name)
    rng = np.random.default_rng(7)
    integer = is_int(A)
    x = rng.integers(-8, 9, A.ncols).astype(float) if integer else rng.uniform(-1, 1, A.ncols)
    y0 = rng.integers(-8, 9, A.n).astype(float) if integer else rng.uniform(-1, 1, A.n)
    Mx = ck.Matrix.from_csr(A)
    dx = torch.from_numpy(x).cuda()
    refused = {ck.ID_ELL: orc.ell_shape(A)[0] != orc.OK,
               ck.ID_DIA: orc.dia_shape(A)[0] != orc.OK}
    for cid in range(ck.NUM_CONFIGS):
        cfg = ck.config_from_id(cid)
        say(f"spmv {name} n={A.n} nnz={A.nnz} config={ck.CONFIG_NAMES[cid]}")
        if refused.get(cid, False):
            with pytest.raises(ck.CkError) as e:
                ck.spmv_convert(Mx.handle, cfg)
            assert e.value.status == ck.CK_E_UNSUPPORTED
            continue
        ck.spmv_convert(Mx.handle, cfg)
        for alpha, beta in [(1.0, 0.0), (-0.5, 2.0)]:
            dy = torch.from_numpy(y0).cuda() if beta else torch.full((A.n,), float("nan"),
                                                                      dtype=torch.float64,
                                                                      device="cuda")
            ck.spmv_apply(Mx.handle, dx, dy, alpha, beta, cfg)
            got = dy.cpu().numpy()
            ref = orc.spmv(A, x, alpha, beta, y0)
            if integer:
                assert np.array_equal(got, ref), (name, cid, alpha, beta)
            else:
                # HYB rounds the ELL part and the remainder separately (two
                # more roundings than one sequential row sum)
                bound = spmv_bound(orc, A, x, alpha, beta, y0, U64,
                                   k_extra=4 if cid == 13 else 2)
                assert np.all(np.abs(got - ref) <= bound), (name, cid, alpha, beta)
                normA = np.max(orc.spmv(M.CSR(A.n, A.ncols, A.rp, A.col, np.abs(A.val)),
                                        np.ones(A.ncols)), initial=0.0)
                err = np.max(np.abs(got - ref), initial=0.0)
                assert err <= 1e-13 * (abs(alpha) * normA * np.max(np.abs(x), initial=0.0)
                                       + abs(beta) * np.max(np.abs(y0), initial=0.0)) + 1e-300
        # determinism: same inputs, same bits
        d1 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        d2 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        ck.spmv_apply(Mx.handle, dx, d1, 1.0, 0.0, cfg)
        ck.spmv_apply(Mx.handle, dx, d2, 1.0, 0.0, cfg)
        assert torch.equal(d1, d2)
    Mx.close()


@pytest.mark.parametrize("name", ["int_ragged", "int_hub", "powerlaw", "banded27", "uniform",
                                  "empty", "single_row", "lap1d", "lap2d_64", "lap3d_12", "banded9",
                                  "banded13", "banded19", "blockdiag"])
def test_spmv_all_configs_fp32(ck, orc, name):
    import torch
    A = case(name)
    rng = np.random.default_rng(8)
    integer = is_int(A)
    x = rng.integers(-8, 9, A.ncols).astype(float) if integer else rng.uniform(-1, 1, A.ncols)
    y0 = rng.integers(-8, 9, A.n).astype(float) if integer else rng.uniform(-1, 1, A.n)
    x32, y32 = x.astype(np.float32), y0.astype(np.float32)
    A32 = M.CSR(A.n, A.ncols, A.rp, A.col, A.val.astype(np.float32).astype(np.float64))
    Mx = ck.Matrix.from_csr(A, keep_fp32=True)
    dx = torch.from_numpy(x32).cuda()
    for cid in range(ck.NUM_CONFIGS):
        cfg = ck.config_from_id(cid)
        say(f"spmv32 {name} config={ck.CONFIG_NAMES[cid]}")
        try:
            ck.spmv_convert(Mx.handle, cfg)
        except ck.CkError as e:
            assert cid in (ck.ID_ELL, ck.ID_DIA) and e.status == ck.CK_E_UNSUPPORTED
            assert (orc.ell_shape(A) if cid == ck.ID_ELL else orc.dia_shape(A))[0] != orc.OK
            continue
        dy = torch.from_numpy(y32).cuda()
        ck.spmv_apply_f32(Mx.handle, dx, dy, -0.5, 2.0, cfg)
        got = dy.cpu().numpy().astype(np.float64)
        ref = orc.spmv(A32, x32.astype(np.float64), -0.5, 2.0, y32.astype(np.float64))
        if integer:
            assert np.array_equal(got, ref)
        else:
            bound = spmv_bound(orc, A32, x32.astype(np.float64), -0.5, 2.0,
                               y32.astype(np.float64), U32, k_extra=5 if cid == 13 else 3)
            assert np.all(np.abs(got - ref) <= bound), (name, cid)
    Mx.close()


@pytest.mark.parametrize("name", list(CASES))
def test_dia_and_hyb_layouts_bit_exact(ck, orc, name):
    """DIA offsets and values, HYB width, ELL part and long-row list equal the
    oracle's conversions bit for bit (values compared as raw bits, so the sign
    of a zero counts)."""
    A = case(name)
    say(f"dia/hyb layout {name} n={A.n} nnz={A.nnz}")
    Mx = ck.Matrix.from_csr(A)
    st, nd, pitch, off, dv = orc.to_dia(A)
    if st != orc.OK:
        with pytest.raises(ck.CkError) as e:
            ck.spmv_convert(Mx.handle, ck.config_from_id(ck.ID_DIA))
        assert e.value.status == ck.CK_E_UNSUPPORTED
    else:
        ck.spmv_convert(Mx.handle, ck.config_from_id(ck.ID_DIA))
        gnd, gpitch, goff, gdv = ck.export_dia(Mx.handle)
        assert (gnd, gpitch) == (nd, pitch)
        assert np.array_equal(goff.cpu().numpy(), off)
        assert np.array_equal(gdv.cpu().numpy().view(np.uint64), dv.view(np.uint64))
    K, pitch, ec, ev, tr = orc.to_hyb(A)
    ck.spmv_convert(Mx.handle, ck.config_from_id(13))
    gK, gpitch, lanes, gec, gev, gtr = ck.export_hyb(Mx.handle)
    assert (gK, gpitch) == (K, pitch)
    assert np.array_equal(gec.cpu().numpy(), ec)
    assert np.array_equal(gev.cpu().numpy().view(np.uint64), ev.view(np.uint64))
    assert np.array_equal(gtr.cpu().numpy(), tr)
    r = np.diff(A.rp.astype(np.int64))
    tail = int(np.sum(r[tr] - K)) if tr.shape[0] else 0
    mean = tail // tr.shape[0] if tr.shape[0] else 0
    expect_lanes = 1
    while expect_lanes * 2 <= mean and expect_lanes < 64:
        expect_lanes *= 2
    assert lanes == expect_lanes
    Mx.close()


@pytest.mark.parametrize("name", ["int_ragged", "int_wide", "int_hub", "powerlaw", "banded27", "blockdiag",
                                  "uniform", "lap2d_64", "convdiff", "empty", "one_by_one",
                                  "single_row", "single_col", "column_runs"])
def test_features_bit_exact(ck, orc, name):
    A = case(name)
    say(f"features {name}")
    Mx = ck.Matrix.from_csr(A)
    F = ck.spmv_features(Mx.handle)
    ints, der, f15 = orc.features(A)
    assert F.ints() == [int(v) for v in ints], name
    got = np.array(F.derived())
    assert np.array_equal(got.view(np.int64), der.view(np.int64)), (name, got, der)
    assert np.array_equal(np.array(F.model_inputs()), f15)
    Mx.close()


@pytest.mark.parametrize("name", ["powerlaw", "uniform", "lap2d_64", "empty"])
def test_features_without_symmetry(ck, orc, name):
    A = case(name)
    say(f"features without symmetry {name}")
    Mx = ck.Matrix.from_csr(A)
    full = ck.spmv_features(Mx.handle)
    part = ck.spmv_features(Mx.handle, symmetry=False)
    assert part.is_symmetric == -1
    assert part.ints()[:27] == full.ints()[:27]
    assert np.array_equal(np.array(part.model_inputs()), np.array(full.model_inputs()))
    assert ck.spmv_select(part).__repr__() == ck.spmv_select(full).__repr__()
    Mx.close()


def _hub_asymmetric(A):
    """The graph Laplacian with one off-diagonal value of its longest row
    changed: the pattern stays symmetric, the values do not."""
    from synth.matrices import CSR
    r = np.diff(A.rp)
    i = int(np.argmax(r))
    val = A.val.copy()
    ks = [k for k in range(A.rp[i], A.rp[i + 1]) if A.col[k] != i]
    val[ks[len(ks) // 2]] += 0.5
    return CSR(A.n, A.ncols, A.rp, A.col, val, A.name + "_asym")


def test_symmetric_flag(ck, orc):
    hub = M.graph_laplacian_chung_lu(20000, 12, wmax=4000)     # rows well over 512 entries
    assert np.diff(hub.rp).max() > 512
    for A in [M.laplacian_2d(30), M.graph_laplacian_chung_lu(5000, 11, wmax=500),
              M.convection_diffusion_2d(30), M.diagonally_dominant(M.uniform_random(3000, 2)),
              hub, _hub_asymmetric(hub)]:
        say(f"symmetry {A.name}")
        Mx = ck.Matrix.from_csr(A)
        F = ck.spmv_features(Mx.handle)
        ints = orc.features(A)[0]
        assert F.is_symmetric == ints[27], A.name
        assert F.ints() == [int(v) for v in ints], A.name
        Mx.close()


@pytest.mark.parametrize("name", ["int_ragged", "banded27", "blockdiag", "lap2d_64", "convdiff",
                                  "single_col", "one_by_one"])
def test_ell_conversion_bit_exact(ck, orc, name):
    A = case(name)
    say(f"ell {name}")
    st, K, pitch, ec, ev = orc.to_ell(A)
    Mx = ck.Matrix.from_csr(A)
    if st != orc.OK:
        with pytest.raises(ck.CkError):
            ck.spmv_convert(Mx.handle, ck.config_from_id(9))
        return
    ck.spmv_convert(Mx.handle, ck.config_from_id(9))
    gK, gp, gc, gv = ck.export_ell(Mx.handle)
    assert (gK, gp) == (K, pitch)
    assert np.array_equal(gc.cpu().numpy(), ec)
    assert np.array_equal(gv.cpu().numpy().view(np.int64), ev.view(np.int64))   # +0.0 padding
    Mx.close()


def test_ell_refused_like_oracle(ck, orc):
    A = case("powerlaw")
    assert orc.ell_shape(A)[0] == orc.UNSUPPORTED
    Mx = ck.Matrix.from_csr(A)
    with pytest.raises(ck.CkError) as e:
        ck.spmv_convert(Mx.handle, ck.config_from_id(9))
    assert e.value.status == ck.CK_E_UNSUPPORTED
    Mx.close()


@pytest.mark.parametrize("name", ["int_ragged", "powerlaw", "uniform", "empty", "single_col"])
def test_coo_conversion_bit_exact(ck, orc, name):
    A = case(name)
    say(f"coo {name}")
    Mx = ck.Matrix.from_csr(A)
    ck.spmv_convert(Mx.handle, ck.config_from_id(10))
    got = ck.export_coo_rows(Mx.handle, A.nnz).cpu().numpy()
    assert np.array_equal(got, orc.to_coo_rows(A))
    Mx.close()


def test_cascade_decisions_match_oracle(ck, orc, tmp_path):
    """Same features + same model -> same decisions (shipped model and a
    freshly fitted sklearn model)."""
    from sklearn.tree import DecisionTreeClassifier
    mats = [case(n) for n in ["int_ragged", "powerlaw", "banded27", "blockdiag", "uniform",
                              "lap2d_64", "convdiff"]]
    feats = []
    for A in mats:
        Mx = ck.Matrix.from_csr(A)
        feats.append(ck.spmv_features(Mx.handle))
        Mx.close()
    trees = parse_model(MODEL)
    for F, A in zip(feats, mats):
        _, _, f15 = orc.features(A)
        assert ck.select_stages(F) == orc.cascade(trees, f15)
    # a model fitted here on oracle features with arbitrary labels
    X = np.array([orc.features(A)[2] for A in mats] * 3)
    X = X * np.repeat([1.0, 0.5, 2.0], len(mats))[:, None]
    y1 = np.arange(len(X)) % 3
    y2 = (np.arange(len(X)) // 2) % 3
    y3 = np.arange(len(X)) % 7
    fitted = [sk_tree(DecisionTreeClassifier(random_state=0).fit(X, y)) for y in (y1, y2, y3)]
    path = str(tmp_path / "m.txt")
    write_model(path, fitted)
    for F, A in zip(feats, mats):
        _, _, f15 = orc.features(A)
        assert ck.select_stages(F, path) == orc.cascade(fitted, f15)


def test_merge_with_and_without_cached_partition(ck, orc):
    """CSR-merge gives the same bits whether its workgroups read the matrix's
    cached partition (after conversion) or search their bounds themselves."""
    import torch
    for name in ["int_ragged", "powerlaw", "uniform", "single_row"]:
        A = case(name)
        say(f"merge partition {name}")
        x = np.random.default_rng(3).uniform(-1, 1, A.ncols)
        dx = torch.from_numpy(x).cuda()
        cfg = ck.config_from_id(8)
        Mx = ck.Matrix.from_csr(A)
        y1 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        ck.spmv_apply(Mx.handle, dx, y1, 1.0, 0.0, cfg)        # no conversion yet: searches
        ck.spmv_convert(Mx.handle, cfg)
        y2 = torch.zeros_like(y1)
        ck.spmv_apply(Mx.handle, dx, y2, 1.0, 0.0, cfg)        # cached partition
        assert torch.equal(y1, y2), name
        ref = orc.spmv(A, x)
        assert np.all(np.abs(y2.cpu().numpy() - ref) <= spmv_bound(orc, A, x, 1.0, 0.0, None, U64))
        Mx.close()


def test_dot_deterministic_and_accurate(ck):
    import torch
    for n in [0, 1, 1000, 1 << 20, 3_000_001]:
        say(f"dot n={n}")
        rng = np.random.default_rng(n)
        x, y = rng.standard_normal(n), rng.standard_normal(n)
        dx, dy = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
        o1 = torch.zeros(1, dtype=torch.float64, device="cuda")
        o2 = torch.zeros(1, dtype=torch.float64, device="cuda")
        ck.dot(dx, dy, o1)
        ck.dot(dx, dy, o2)
        assert torch.equal(o1, o2)
        ref = float(np.dot(x, y))
        assert abs(o1.item() - ref) <= 1e-14 * max(1.0, float(np.dot(np.abs(x), np.abs(y))))


def test_invalid_csr_rejected(ck):
    import torch
    A = M.laplacian_1d(10)
    rp, col, val = upload(A)
    bad = col.clone()
    bad[3], bad[4] = col[4], col[3]
    with pytest.raises(ck.CkError) as e:
        ck.spmv_create(rp, bad, val)
    assert e.value.status == ck.CK_E_INVALID
    bad = col.clone()
    bad[0] = 10
    with pytest.raises(ck.CkError):
        ck.spmv_create(rp, bad, val)
    badrp = rp.clone()
    badrp[5] = rp[7]                      # row pointers not monotone
    with pytest.raises(ck.CkError):
        ck.spmv_create(badrp, col, val)
    # rows longer than 512 entries are checked by their own pass: a repeated,
    # an out-of-order and an out-of-range column deep inside a 2000-entry row
    D = np.zeros((3, 4000))
    D[1, ::2] = 1.0
    D[0, 7] = D[2, 3999] = 2.0
    L = M.from_dense(D)
    assert np.diff(L.rp).max() == 2000
    rp, col, val = upload(L)
    ck.Matrix(rp, col, val, ncols=L.ncols).close()   # the valid one is accepted
    k = int(L.rp[1]) + 1500
    for what in ("repeat", "swap", "range"):
        bad = col.clone()
        if what == "repeat":
            bad[k] = col[k - 1]
        elif what == "swap":
            bad[k], bad[k + 1] = col[k + 1], col[k]
        else:
            bad[k + 400] = 4000
        say(f"invalid long row: {what}")
        with pytest.raises(ck.CkError) as e:
            ck.spmv_create(rp, bad, val, ncols=L.ncols)
        assert e.value.status == ck.CK_E_INVALID, what
    # row pointers that go up and down: every other row has valid bounds and
    # 1000 entries, so more rows look long than 1000 entries can hold (the
    # long-row list is sized for disjoint rows and must not overflow)
    import torch
    n = 64
    rpl = torch.tensor([0 if t % 2 == 0 else 1000 for t in range(n)] + [1000],
                       dtype=torch.int32, device="cuda")
    coll = torch.arange(1000, dtype=torch.int32, device="cuda")
    vall = torch.ones(1000, dtype=torch.float64, device="cuda")
    say("invalid: overlapping long rows")
    with pytest.raises(ck.CkError) as e:
        ck.spmv_create(rpl, coll, vall, ncols=1000)
    assert e.value.status == ck.CK_E_INVALID


@pytest.mark.parametrize("cid", [8, 9, 10, 11, 12, 13])
def test_converted_copy_serves_another_stream_at_once(ck, orc, cid):
    """spmv_convert returns when the copy is built, so a product on a
    different stream right after it (no synchronisation in between) reads a
    complete copy; the request loop relies on this when its scheduler
    converts and a worker stream solves."""
    import torch
    A = M.uniform_random(200003, 31, 4, 40) if cid != 12 else M.banded_stencil(200003, 27, 31)
    say(f"convert on one stream, product on another: config {ck.CONFIG_NAMES[cid]}")
    Mx = ck.Matrix.from_csr(A)
    x = np.random.default_rng(5).uniform(-1, 1, A.ncols)
    dx = torch.from_numpy(x).cuda()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    cfg = ck.config_from_id(cid)
    dy = torch.empty(A.n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    ck.spmv_convert(Mx.handle, cfg, stream=s1)
    ck.spmv_apply(Mx.handle, dx, dy, 1.0, 0.0, cfg, stream=s2)
    s2.synchronize()
    ref = orc.spmv(A, x)
    bound = spmv_bound(orc, A, x, 1.0, 0.0, None, U64, k_extra=4)
    assert np.all(np.abs(dy.cpu().numpy() - ref) <= bound)
    Mx.close()


def _with_hub_row(A, length):
    """A with row 0 replaced by `length` entries in columns 0, 1, ..."""
    r0 = int(A.rp[1])
    L = min(length, A.ncols)
    col = np.concatenate([np.arange(L, dtype=np.int32), A.col[r0:]])
    val = np.concatenate([np.linspace(0.5, 1.5, L), A.val[r0:]])
    rp = np.concatenate([[0], A.rp[1:] - r0 + L]).astype(np.int32)
    return M.CSR(A.n, A.ncols, rp, col, val, "hub").check()


def _expected_panel_layout(A):
    """The panel count and layout the conversion documents: P8 = 8q panels of
    at most 2 MB of FP64 x; P = 4 when x fits four 2.5 MB slices, the longest
    row is at most 4 ceil(nnz/n) and more than 3/4 of the 4n panel rows hold
    entries; the row-list layout when at most 3/4 of the P n rows do."""
    per = (2 << 20) // 8
    P8 = 8 * max(1, -(-A.ncols // (8 * per)))
    lengths = np.diff(A.rp.astype(np.int64))
    rows = np.repeat(np.arange(A.n, dtype=np.int64), lengths)

    def nonempty(P):
        W = -(-max(A.ncols, 1) // P)
        return len(np.unique(rows * P + A.col.astype(np.int64) // W))

    P = P8
    if (P8 == 8 and A.n > 0 and A.ncols * 8 <= 4 * 5 * (1 << 19)
            and lengths.max() <= 4 * (-(-A.nnz // A.n)) and 4 * nonempty(4) > 3 * 4 * A.n):
        P = 4
    ne = nonempty(P)
    return P, -(-max(A.ncols, 1) // P), (P * A.n if 4 * ne > 3 * P * A.n else ne)


@pytest.mark.parametrize("name", ["uniform", "uniform_hub", "powerlaw", "int_ragged", "banded27",
                                  "column_runs", "single_row", "empty"])
def test_panel_count_and_layout(ck, orc, name):
    """Four panels only for even rows that fill them (uniform); a hub row, short
    rows or sparse panel rows keep eight; the product agrees in both layouts."""
    import torch
    A = _with_hub_row(case("uniform"), 4 * 40) if name == "uniform_hub" else case(name)
    want = _expected_panel_layout(A)
    if name == "uniform":
        assert want[0] == 4
    if name in ("uniform_hub", "powerlaw"):
        assert want[0] == 8
    say(f"panel layout {name} n={A.n} nnz={A.nnz} expect P={want[0]} rows={want[2]}")
    Mx = ck.Matrix.from_csr(A)
    cfg = ck.config_from_id(ck.CONFIG_NAMES.index("csr-panel"))
    ck.spmv_convert(Mx.handle, cfg)
    assert ck.panel_layout(Mx.handle) == want
    rng = np.random.default_rng(31)
    x = rng.uniform(-1, 1, A.ncols)
    y0 = rng.uniform(-1, 1, A.n)
    dy = torch.from_numpy(y0).cuda()
    ck.spmv_apply(Mx.handle, torch.from_numpy(x).cuda(), dy, 1.5, -0.5, cfg)
    ref = orc.spmv(A, x, 1.5, -0.5, y0)
    assert np.all(np.abs(dy.cpu().numpy() - ref) <= spmv_bound(orc, A, x, 1.5, -0.5, y0, U64))
    Mx.close()
