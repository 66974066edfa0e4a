"""The multi-kernel CG and GMRES drivers (systems above the one-launch sizes,
n > 16384) against the oracle, step by step: the iterate after k iterations
equals the oracle's after k iterations (both form the same Krylov iterate;
only rounding differs), the iteration count to convergence matches the
oracle's, and the mixed FP32/FP64 drivers reach the FP64 tolerance on the
oracle's own residual."""
import numpy as np
import pytest

from helpers import say
from synth import matrices as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ck():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_10143_amd as ck
    ck.lib()
    return ck


def problem(orc, A, seed):
    xs = M.vector(A.n, seed)
    return xs, orc.spmv(A, xs)


def run(ck, solver, Mx, b, x0=None, **kw):
    import torch
    db = torch.from_numpy(b).cuda()
    dx = torch.zeros_like(db) if x0 is None else torch.from_numpy(x0).cuda()
    res = solver(Mx.handle, db, dx, **kw)
    return dx.cpu().numpy(), res


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def lap2d_160(orc):
    A = M.laplacian_2d(160)                      # n = 25,600
    xs, b = problem(orc, A, 21)
    x0 = M.vector(A.n, 22) * 0.1
    return A, b, x0


# default CSR-vector, CSR-scalar, CSR-merge, COO, CSR-panel, DIA, HYB
CG_CONFIGS = [None, 7, 8, 10, 11, 12, 13]


@pytest.mark.parametrize("cid", CG_CONFIGS)
def test_cg_multikernel_iterates_match_oracle(ck, orc, lap2d_160, cid):
    A, b, x0 = lap2d_160
    assert A.n > 16384
    kw = {} if cid is None else {"config": ck.config_from_id(cid)}
    Mx = ck.Matrix.from_csr(A)
    for k in (1, 7, 60):
        say(f"cg multi-kernel lap2d_160 config={cid} k={k}")
        x, r = run(ck, ck.cg_solve, Mx, b, x0=x0, tol=1e-14, max_iter=k, **kw)
        assert r["status"] == ck.CK_E_NOT_CONVERGED and r["iterations"] == k, r
        refk = orc.cg(A, b, x0=x0, tol=1e-14, maxit=k)
        assert rel(x, refk["x"]) <= 1e-9, (k, rel(x, refk["x"]))
    say(f"cg multi-kernel lap2d_160 config={cid} to 1e-10")
    x, r = run(ck, ck.cg_solve, Mx, b, x0=x0, tol=1e-10, **kw)
    ref = orc.cg(A, b, x0=x0, tol=1e-10)
    assert r["status"] == ck.CK_OK, r
    rr = orc.relres(A, b, x)
    assert rr <= 1e-10 and abs(rr - r["true_relres"]) <= 1e-3 * rr
    assert abs(r["iterations"] - ref["iters"]) <= max(2, 0.02 * ref["iters"]), \
        (r["iterations"], ref["iters"])
    if cid is None:
        assert r["final_config"] == ck.config_id(ck.default_config(Mx.handle))
    else:
        assert r["final_config"] == cid
    Mx.close()


def test_cg_multikernel_graph_laplacian(ck, orc):
    """Hub rows (power-law degrees) on the merge and panel paths.  On this
    matrix finite-precision CG amplifies rounding differences quickly: a
    second CPU CG that only sums in another order leaves the oracle's iterate
    1e-14 apart after 10 iterations, 8e-12 after 15 and 1e-4 after 25, so
    the step-by-step comparison stops at 12 iterations.  The iteration count
    to 1e-10 moves with the summation order too: the oracle takes 1110, CPU
    CGs that differ only in how they sum take 1088 and 1095, so counts are
    compared within 5 %."""
    A = M.graph_laplacian_chung_lu(40000, 23)
    xs, b = problem(orc, A, 24)
    Mx = ck.Matrix.from_csr(A)
    ref = orc.cg(A, b, tol=1e-10)
    for cid in (None, 8, 11):
        kw = {} if cid is None else {"config": ck.config_from_id(cid)}
        say(f"cg multi-kernel graph_40000 config={cid}")
        for k in (5, 12):
            x, r = run(ck, ck.cg_solve, Mx, b, tol=1e-14, max_iter=k, **kw)
            assert r["status"] == ck.CK_E_NOT_CONVERGED and r["iterations"] == k, r
            refk = orc.cg(A, b, tol=1e-14, maxit=k)
            assert rel(x, refk["x"]) <= 1e-9, (k, rel(x, refk["x"]))
        x, r = run(ck, ck.cg_solve, Mx, b, tol=1e-10, **kw)
        assert r["status"] == ck.CK_OK and orc.relres(A, b, x) <= 1e-10, r
        assert abs(r["iterations"] - ref["iters"]) <= 0.05 * ref["iters"], \
            (r["iterations"], ref["iters"])
    Mx.close()


@pytest.fixture(scope="module")
def convdiff_160(orc):
    A = M.convection_diffusion_2d(160, 10.0)      # n = 25,600, nonsymmetric
    xs, b = problem(orc, A, 31)
    x0 = M.vector(A.n, 32) * 0.1
    return A, b, x0


@pytest.mark.parametrize("cid", [None, 8, 11, 12])
def test_gmres_multikernel_iterates_match_oracle(ck, orc, convdiff_160, cid):
    """After k Arnoldi steps (inside the first cycle, at its end, and past a
    restart) the GPU iterate is the oracle's; the oracle orthogonalises by
    modified Gram-Schmidt, the GPU by classical Gram-Schmidt applied twice,
    so only rounding separates them."""
    A, b, x0 = convdiff_160
    kw = {} if cid is None else {"config": ck.config_from_id(cid)}
    Mx = ck.Matrix.from_csr(A)
    for k in (5, 30, 47):
        say(f"gmres multi-kernel convdiff_160 config={cid} k={k}")
        x, r = run(ck, ck.gmres_solve, Mx, b, x0=x0, tol=1e-14, max_iter=k, restart=30, **kw)
        assert r["status"] == ck.CK_E_NOT_CONVERGED and r["iterations"] == k, r
        refk = orc.gmres(A, b, x0=x0, m=30, tol=1e-14, maxit=k)
        assert rel(x, refk["x"]) <= 1e-9, (k, rel(x, refk["x"]))
    say(f"gmres multi-kernel convdiff_160 config={cid} to 1e-10")
    x, r = run(ck, ck.gmres_solve, Mx, b, x0=x0, tol=1e-10, restart=30, **kw)
    ref = orc.gmres(A, b, x0=x0, m=30, tol=1e-10)
    assert r["status"] == ck.CK_OK, r
    assert orc.relres(A, b, x) <= 1e-10
    assert abs(r["iterations"] - ref["iters"]) <= max(2, 0.02 * ref["iters"]), \
        (r["iterations"], ref["iters"])
    Mx.close()


@pytest.fixture(scope="module")
def lap3d_40(orc):
    A = M.laplacian_3d(40)                        # n = 64,000
    xs, b = problem(orc, A, 41)
    return A, b, xs


@pytest.fixture(scope="module")
def lap3d_64(orc):
    A = M.laplacian_3d(64)                        # n = 262,144
    xs, b = problem(orc, A, 42)
    return A, b, xs


@pytest.mark.parametrize("mode", ["default", "merge", "dia", "async"])
def test_cg_mixed_multikernel(ck, orc, lap3d_40, lap3d_64, mode):
    """Mixed precision CG on the multi-kernel path: FP32 inner CG segments
    with FP64 refinement reach the FP64 tolerance on the oracle's residual,
    and land within the same forward-error bound as the FP64 solve."""
    # async runs on the 64^3 system, whose solve outlasts the feature pass
    A, b, xs = lap3d_64 if mode == "async" else lap3d_40
    kw = {"default": {}, "merge": {"config": ck.config_from_id(8)},
          "dia": {"config": ck.config_from_id(12)}, "async": {"async_": True}}[mode]
    Mx = ck.Matrix.from_csr(A, keep_fp32=True)
    say(f"cg mixed multi-kernel lap3d n={A.n} {mode}")
    xm, rm = run(ck, ck.cg_solve, Mx, b, tol=1e-10, precision=ck.CK_PREC_MIXED, **kw)
    assert rm["status"] == ck.CK_OK, rm
    rr = orc.relres(A, b, xm)
    assert rr <= 1e-10 and abs(rr - rm["true_relres"]) <= 1e-3 * rr, (rr, rm)
    assert rm["outer_steps"] >= 2, rm            # FP32 alone cannot reach 1e-10
    say(f"cg fp64 multi-kernel lap3d n={A.n} {mode}")
    xd, rd = run(ck, ck.cg_solve, Mx, b, tol=1e-10, **kw)
    assert rd["status"] == ck.CK_OK and orc.relres(A, b, xd) <= 1e-10
    # ||x - x*|| <= cond(A) * relres * ||x*||; cond of the N^3 Laplacian < 0.41 (N+1)^2
    cond = 0.41 * (round(A.n ** (1 / 3)) + 1) ** 2
    assert rel(xm, xs) <= cond * 1e-10 and rel(xd, xs) <= cond * 1e-10
    if mode in ("merge", "dia"):
        assert rm["final_config"] == ck.config_id(kw["config"])
    if mode == "async":
        assert rm["switch_iter"][0] >= 0, rm
    Mx.close()


def test_cg_mixed_budget_and_zero_rhs(ck, orc, lap3d_40):
    A, b, xs = lap3d_40
    Mx = ck.Matrix.from_csr(A, keep_fp32=True)
    say("cg mixed multi-kernel budget")
    x, r = run(ck, ck.cg_solve, Mx, b, tol=1e-12, max_iter=30, precision=ck.CK_PREC_MIXED)
    assert r["status"] == ck.CK_E_NOT_CONVERGED and r["iterations"] <= 30, r
    assert abs(orc.relres(A, b, x) - r["true_relres"]) <= 1e-6 * r["true_relres"]
    say("cg mixed multi-kernel zero rhs")
    x, r = run(ck, ck.cg_solve, Mx, np.zeros(A.n), x0=np.ones(A.n),
               precision=ck.CK_PREC_MIXED)
    assert r["status"] == ck.CK_OK and not x.any()
    Mx.close()


@pytest.mark.parametrize("mode", ["default", "dia", "async"])
def test_gmres_mixed_multikernel(ck, orc, convdiff_160, mode):
    A, b, x0 = convdiff_160
    kw = {"default": {}, "dia": {"config": ck.config_from_id(12)},
          "async": {"async_": True}}[mode]
    Mx = ck.Matrix.from_csr(A, keep_fp32=True)
    say(f"gmres mixed multi-kernel convdiff_160 {mode}")
    xm, rm = run(ck, ck.gmres_solve, Mx, b, tol=1e-10, precision=ck.CK_PREC_MIXED, **kw)
    assert rm["status"] == ck.CK_OK, rm
    rr = orc.relres(A, b, xm)
    assert rr <= 1e-10 and abs(rr - rm["true_relres"]) <= 1e-3 * rr
    ref = orc.gmres(A, b, m=30, tol=1e-10)
    # one FP32 cycle per refinement step: the count stays near the FP64 one
    assert rm["iterations"] <= 1.5 * ref["iters"] + 30, (rm["iterations"], ref["iters"])
    Mx.close()


def test_gmres_mixed_odd_rows(ck, orc):
    """Mixed GMRES at an odd n > 16384 (the multi-kernel path, the basis
    columns padded past n): true residual within 1e-10 by the oracle."""
    A = M.convection_diffusion_2d(131, 10.0)      # n = 17,161
    assert A.n % 2 == 1 and A.n > 16384
    xs, b = problem(orc, A, 33)
    Mx = ck.Matrix.from_csr(A, keep_fp32=True)
    say("gmres mixed multi-kernel convdiff_131 (odd n)")
    xm, rm = run(ck, ck.gmres_solve, Mx, b, tol=1e-10, precision=ck.CK_PREC_MIXED)
    assert rm["status"] == ck.CK_OK, rm
    rr = orc.relres(A, b, xm)
    assert rr <= 1e-10 and abs(rr - rm["true_relres"]) <= 1e-3 * rr
    ref = orc.gmres(A, b, m=30, tol=1e-10)
    assert rm["iterations"] <= 1.5 * ref["iters"] + 30, (rm["iterations"], ref["iters"])
    Mx.close()


@pytest.mark.parametrize("cid", [None, 11, 12])
def test_cg_multikernel_breakdown_leaves_x(ck, orc, cid):
    """A = -I with n > 16384 (the multi-kernel path): the first p.Ap is
    negative, so CG stops with CK_E_BREAKDOWN before any x/p update and x is
    still x0 (the oracle stops the same way)."""
    n = 20000
    A = M.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
              -np.ones(n), "neg_identity").check()
    b = M.vector(n, 5)
    x0 = M.vector(n, 6)
    kw = {} if cid is None else {"config": ck.config_from_id(cid)}
    say(f"cg multi-kernel breakdown config={cid}")
    Mx = ck.Matrix.from_csr(A)
    x, r = run(ck, ck.cg_solve, Mx, b, x0=x0, tol=1e-10, **kw)
    assert r["status"] == ck.CK_E_BREAKDOWN, r
    assert np.array_equal(x, x0)
    ref = orc.cg(A, b, x0=x0, tol=1e-10)
    assert np.array_equal(ref["x"], x0)
    Mx.close()
