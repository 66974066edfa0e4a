"""Parity at the benchmark's full sizes, with the kernels and launch
configurations the bench times:

* every matrix of the 48-matrix SpMV set (n = 1e4 .. 2e6): integer features
  and derived features bit-exact, the cascade's decision (host and
  device-resident) equal to the oracle's, and every one of the 14 SpMV
  configurations element by element
  against the oracle's FP64 product (the oracle computes the whole product in
  well under a second);
* ELL, COO, DIA and HYB conversions byte-exact on the largest member of each
  family;
* CG on the 3D Poisson 128^3 and 2^20-row graph Laplacian systems (async
  executor) and GMRES(30) on convection-diffusion 1024^2, FP64 and mixed,
  checked by the oracle's true FP64 residual.
"""
import numpy as np
import pytest

from helpers import MODEL, parse_model, say, spmv_bound
from synth import matrices as M
from synth import workloads as W

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
SPECS = W.spmv_set_specs()


@pytest.fixture(scope="module")
def ck():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_10143_amd as ck
    ck.lib()
    return ck


@pytest.mark.parametrize("spec", SPECS, ids=[s[0] for s in SPECS])
def test_spmv_set_member(ck, orc, spec):
    import torch
    A = W.spmv_set_matrix(spec)
    say(f"fullsize {A.name} n={A.n} nnz={A.nnz}")
    Mx = ck.Matrix.from_csr(A)
    # features and decision
    F = ck.spmv_features(Mx.handle)
    ints, der, f15 = orc.features(A)
    assert F.ints() == [int(v) for v in ints]
    assert np.array_equal(np.array(F.derived()).view(np.int64), der.view(np.int64))
    assert ck.select_stages(F) == orc.cascade(parse_model(MODEL), f15)
    # the device-resident cascade reaches the same decision on the device
    out = torch.full((8,), -9, dtype=torch.int32, device="cuda")
    ck.select_device(Mx.handle, out)
    dev = out.cpu().tolist()
    assert dev[4:7] == orc.cascade(parse_model(MODEL), f15), (A.name, dev)
    assert dev[7] == ck.config_id(ck.spmv_select(F)), (A.name, dev)
    # every configuration against the oracle product
    x = np.random.default_rng(spec[4]).uniform(-1, 1, A.ncols)
    ref = orc.spmv(A, x)
    bound = spmv_bound(orc, A, x, 1.0, 0.0, None, U64)
    bound_hyb = spmv_bound(orc, A, x, 1.0, 0.0, None, U64, k_extra=4)
    normA = float(np.max(orc.spmv(M.CSR(A.n, A.ncols, A.rp, A.col, np.abs(A.val)),
                                  np.ones(A.ncols))))
    dx = torch.from_numpy(x).cuda()
    dy = torch.empty(A.n, dtype=torch.float64, device="cuda")
    refused = {ck.ID_ELL: orc.ell_shape(A)[0] != orc.OK,
               ck.ID_DIA: orc.dia_shape(A)[0] != orc.OK}
    for cid in range(ck.NUM_CONFIGS):
        cfg = ck.config_from_id(cid)
        say(f"  config {ck.CONFIG_NAMES[cid]}")
        if refused.get(cid, False):
            with pytest.raises(ck.CkError) as e:
                ck.spmv_convert(Mx.handle, cfg)
            assert e.value.status == ck.CK_E_UNSUPPORTED
            continue
        ck.spmv_convert(Mx.handle, cfg)
        dy.fill_(float("nan"))
        ck.spmv_apply(Mx.handle, dx, dy, 1.0, 0.0, cfg)
        got = dy.cpu().numpy()
        err = np.abs(got - ref)
        assert np.all(err <= (bound_hyb if cid == 13 else bound)), \
            (A.name, cid, float(np.max(err - bound)))
        assert float(np.max(err)) <= 1e-13 * normA * float(np.max(np.abs(x)))
    Mx.close()


LARGEST = [s for s in SPECS if s[0].endswith("_k11_n2000000")]


@pytest.mark.parametrize("spec", LARGEST, ids=[s[0] for s in LARGEST])
def test_conversions_largest(ck, orc, spec):
    A = W.spmv_set_matrix(spec)
    say(f"fullsize conversions {A.name}")
    Mx = ck.Matrix.from_csr(A)
    ck.spmv_convert(Mx.handle, ck.config_from_id(10))
    assert np.array_equal(ck.export_coo_rows(Mx.handle, A.nnz).cpu().numpy(), orc.to_coo_rows(A))
    st, K, pitch, ec, ev = orc.to_ell(A)
    if st == orc.OK:
        ck.spmv_convert(Mx.handle, ck.config_from_id(9))
        gK, gp, gc, gv = ck.export_ell(Mx.handle)
        assert (gK, gp) == (K, pitch)
        assert np.array_equal(gc.cpu().numpy(), ec)
        assert np.array_equal(gv.cpu().numpy().view(np.int64), ev.view(np.int64))
    else:
        with pytest.raises(ck.CkError):
            ck.spmv_convert(Mx.handle, ck.config_from_id(9))
    st, nd, pitch, off, dv = orc.to_dia(A)
    if st == orc.OK:
        ck.spmv_convert(Mx.handle, ck.config_from_id(ck.ID_DIA))
        gnd, gp, goff, gdv = ck.export_dia(Mx.handle)
        assert (gnd, gp) == (nd, pitch) and np.array_equal(goff.cpu().numpy(), off)
        assert np.array_equal(gdv.cpu().numpy().view(np.uint64), dv.view(np.uint64))
        del gdv
    K, pitch, ec, ev, tr = orc.to_hyb(A)
    ck.spmv_convert(Mx.handle, ck.config_from_id(13))
    gK, gp, lanes, gc, gv, gtr = ck.export_hyb(Mx.handle)
    assert (gK, gp) == (K, pitch) and np.array_equal(gtr.cpu().numpy(), tr)
    assert np.array_equal(gc.cpu().numpy(), ec)
    assert np.array_equal(gv.cpu().numpy().view(np.uint64), ev.view(np.uint64))
    Mx.close()


def _solve(ck, solver, A, xs, **kw):
    import torch
    Mx = ck.Matrix.from_csr(A, keep_fp32=kw.get("precision", 0) == ck.CK_PREC_MIXED)
    db = torch.empty(A.n, dtype=torch.float64, device="cuda")
    ck.spmv_apply(Mx.handle, torch.from_numpy(xs).cuda(), db, 1.0, 0.0)
    dx = torch.zeros_like(db)
    r = solver(Mx.handle, db, dx, **kw)
    Mx.close()
    return xs, db.cpu().numpy(), dx.cpu().numpy(), r


@pytest.mark.parametrize("which", ["poisson3d_128", "graph_laplacian_2^20"])
def test_cg_async_full(ck, orc, which):
    A, xs = W.poisson3d_128() if which == "poisson3d_128" else W.graph_laplacian_1m()
    say(f"fullsize async cg {which} n={A.n} nnz={A.nnz}")
    xs, b, x, r = _solve(ck, ck.cg_solve, A, xs, tol=1e-10, async_=True)
    assert r["status"] == ck.CK_OK, r
    rel = orc.relres(A, b, x)
    assert rel <= 1e-10
    assert abs(rel - r["true_relres"]) <= 1e-3 * rel
    assert r["switch_iter"][0] >= 0


def test_gmres_convdiff_1024_fp64_and_mixed(ck, orc):
    A, xs = W.convdiff_1024()
    say(f"fullsize gmres fp64 n={A.n} nnz={A.nnz}")
    xs, b, x64, r64 = _solve(ck, ck.gmres_solve, A, xs, tol=1e-10, restart=30, max_iter=50000)
    assert r64["status"] == ck.CK_OK, r64
    assert orc.relres(A, b, x64) <= 1e-10
    say("fullsize gmres mixed")
    _, b2, xm, rm = _solve(ck, ck.gmres_solve, A, xs, tol=1e-10, restart=30, max_iter=50000,
                           precision=ck.CK_PREC_MIXED)
    assert np.array_equal(b, b2)
    assert rm["status"] == ck.CK_OK, rm
    assert orc.relres(A, b, xm) <= 1e-10
    # both solutions agree to the accuracy a 1e-10 residual allows
    fe64 = np.linalg.norm(x64 - xs) / np.linalg.norm(xs)
    fem = np.linalg.norm(xm - xs) / np.linalg.norm(xs)
    assert fem <= 10 * fe64 + 1e-8, (fem, fe64)
