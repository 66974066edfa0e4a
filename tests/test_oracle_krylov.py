"""Pins for the oracle CG and GMRES(m): exact termination, orthogonality,
closed-form spectra, minimal-residual property, library cross-checks."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from synth import matrices as M


def to_scipy(A):
    return sp.csr_matrix((A.val, A.col, A.rp), shape=(A.n, A.ncols))


@pytest.mark.parametrize("d", [1, 3, 5, 8])
def test_cg_exact_termination_distinct_eigenvalues(orc, d):
    n = 24
    eigs = np.resize(np.linspace(1.0, 100.0, d), n)
    A = M.full_from_dense(M.spd_dense(n, eigs, seed=d))
    b = M.vector(n, 11)
    r = orc.cg(A, b, tol=1e-10, hist=n + 2)
    assert r["status"] == orc.OK and r["iters"] <= d
    assert r["relres"] <= 1e-10


@pytest.mark.parametrize("n", [16, 32])
def test_cg_terminates_within_n_steps(orc, n):
    # n distinct eigenvalues, condition number 10: finite termination in <= n steps
    eigs = np.geomspace(1.0, 10.0, n)
    A = M.full_from_dense(M.spd_dense(n, eigs, seed=4))
    r = orc.cg(A, M.vector(n, 5), tol=1e-10, hist=64)
    assert r["status"] == orc.OK and r["iters"] <= n


def test_cg_laplacian_eigenvector_rhs(orc):
    n = 200
    A = M.laplacian_1d(n)
    i = np.arange(1, n + 1)
    for k in (1, 2, 3):
        # top eigenvectors (eigenvalues near 4) so rounding is not amplified by 1/lambda
        b = sum(np.sin(((i * (n + 1 - j)) % (2 * (n + 1))) * math.pi / (n + 1)) * (j + 1)
                for j in range(1, k + 1))
        r = orc.cg(A, b, tol=1e-12)
        assert r["iters"] == k, (k, r["iters"])


def test_cg_orthogonality_and_conjugacy(orc):
    A = M.laplacian_2d(20)
    b = M.vector(A.n, 3)
    nrec = 15
    r = orc.cg(A, b, tol=1e-14, nrec=nrec)
    R, P = r["R"], r["P"]
    S = to_scipy(A)
    for i in range(nrec):
        for j in range(i):
            cos_r = abs(R[i] @ R[j]) / (np.linalg.norm(R[i]) * np.linalg.norm(R[j]))
            assert cos_r <= 1e-8
            cos_p = abs(P[i] @ (S @ P[j])) / math.sqrt((P[i] @ (S @ P[i])) * (P[j] @ (S @ P[j])))
            assert cos_p <= 1e-8


def test_cg_lanczos_tridiagonal_spectrum(orc):
    N = 32
    A = M.laplacian_2d(N)
    b = M.vector(A.n, 9)
    k = 150
    r = orc.cg(A, b, tol=1e-30, maxit=k, hist=k + 1)
    al, be = r["alpha"][:k], r["beta"][:k]
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1 / al[j] + (be[j - 1] / al[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = math.sqrt(be[j]) / al[j]
    ev = np.linalg.eigvalsh(T)
    lmin = 4 - 4 * math.cos(math.pi / (N + 1))
    lmax = 4 + 4 * math.cos(math.pi / (N + 1))
    assert abs(ev[0] - lmin) / lmin < 1e-6
    assert abs(ev[-1] - lmax) / lmax < 1e-6


def test_cg_lap2d_64_matches_scipy_iterations(orc):
    A = M.laplacian_2d(64)
    xs = M.vector(A.n, 1)
    b = orc.spmv(A, xs)
    r = orc.cg(A, b, tol=1e-10)
    count = [0]
    spla.cg(to_scipy(A), b, rtol=1e-10, atol=0.0, maxiter=10000,
            callback=lambda xk: count.__setitem__(0, count[0] + 1))
    assert r["status"] == orc.OK and r["relres"] <= 1e-10
    assert abs(r["iters"] - count[0]) <= max(2, 0.02 * count[0])
    assert np.linalg.norm(r["x"] - xs) / np.linalg.norm(xs) < 1e-6


def test_cg_breakdown_and_budget_and_zero_rhs(orc):
    A = M.from_dense(-np.eye(5))
    assert orc.cg(A, np.ones(5))["status"] == orc.BREAKDOWN
    L = M.laplacian_2d(32)
    r = orc.cg(L, M.vector(L.n, 2), tol=1e-12, maxit=10)
    assert r["status"] == orc.NOT_CONVERGED and r["iters"] == 10
    r = orc.cg(L, np.zeros(L.n), x0=np.ones(L.n))
    assert r["status"] == orc.OK and not r["x"].any()


def test_arnoldi_relation_and_orthonormality(orc):
    A = M.convection_diffusion_2d(16, 10.0)
    S = to_scipy(A)
    m = 20
    st, V, H, steps = orc.arnoldi(A, M.vector(A.n, 1), m)
    assert st == orc.OK and steps == m
    normA = np.max(np.abs(S).sum(axis=1))
    assert np.linalg.norm(S @ V[:, :m] - V @ H) <= 1e-12 * normA
    assert np.linalg.norm(V.T @ V - np.eye(m + 1)) <= 1e-12
    assert np.all(np.tril(H, -2) == 0)


def test_gmres_full_space_terminates(orc):
    rng = np.random.default_rng(3)
    n = 25
    D = rng.standard_normal((n, n)) + 4 * np.eye(n)
    A = M.full_from_dense(D)
    b = rng.standard_normal(n)
    r = orc.gmres(A, b, m=n, tol=1e-12, hist=n + 2)
    assert r["status"] == orc.OK and r["iters"] <= n and r["relres"] <= 1e-12
    res = r["res"][: r["iters"] + 1]
    assert np.all(np.diff(res) <= 1e-15 * res[0])      # non-increasing in a cycle


def test_gmres_identity_one_step_and_invariant_subspace(orc):
    A = M.from_dense(np.eye(10))
    r = orc.gmres(A, M.vector(10, 1), m=5)
    assert r["iters"] == 1 and r["relres"] <= 1e-15
    Dg = M.from_dense(np.diag(np.arange(1.0, 11.0)))
    b = np.zeros(10)
    b[[1, 4, 7]] = [1.0, -2.0, 3.0]
    r = orc.gmres(Dg, b, m=8, tol=1e-13)
    assert r["status"] == orc.OK and r["iters"] == 3     # happy breakdown at step 3


def test_gmres_minimal_residual_beats_cg(orc):
    A = M.laplacian_2d(24)
    b = M.vector(A.n, 4)
    k = 60
    g = orc.gmres(A, b, m=200, tol=1e-30, maxit=k, hist=k + 2)
    c = orc.cg(A, b, tol=1e-30, maxit=k, hist=k + 2)
    for j in range(1, k + 1):
        assert g["res"][j] <= c["res"][j] * (1 + 1e-8)


def test_gmres30_convdiff_against_scipy(orc):
    A = M.convection_diffusion_2d(48, 10.0)
    xs = M.vector(A.n, 4001)
    b = orc.spmv(A, xs)
    r = orc.gmres(A, b, m=30, tol=1e-10)
    assert r["status"] == orc.OK and r["relres"] <= 1e-10
    count = [0]
    x, info = spla.gmres(to_scipy(A), b, rtol=1e-10, atol=0.0, restart=30, maxiter=10000,
                         callback=lambda pr: count.__setitem__(0, count[0] + 1),
                         callback_type="pr_norm")
    assert info == 0
    assert abs(r["iters"] - count[0]) <= max(5, 0.05 * count[0]), (r["iters"], count[0])


def test_gmres_budget_and_zero_rhs(orc):
    A = M.convection_diffusion_2d(32, 10.0)
    r = orc.gmres(A, M.vector(A.n, 1), m=30, tol=1e-12, maxit=40)
    assert r["status"] == orc.NOT_CONVERGED and r["iters"] == 40
    r = orc.gmres(A, np.zeros(A.n))
    assert r["status"] == orc.OK and r["iters"] == 0


def test_cg_true_residual_restart_branch(orc):
    """The restart branch of CG: started from a huge x0 (1e10 times a random
    vector) on a well-conditioned tridiagonal system, the rounding left in x
    keeps the true residual near 1e-6 while the recurred residual falls past
    tol = 1e-10.  At that stop the true residual (computed here with a dense
    numpy product) must be above tol, CG must restart from the current x with
    the true residual as its first direction -- the next step is a
    steepest-descent step, alpha = r.r / r.Ar, x moves along r -- and the
    restarted run must reach tol."""
    n = 64
    D = 4.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    A = M.from_dense(D)
    xs = M.vector(n, 1)
    b = D @ xs
    x0 = 1e10 * M.vector(n, 2)
    tol = 1e-10
    full = orc.cg(A, b, x0=x0, tol=tol, hist=400)
    res = full["res"]
    crossed = np.flatnonzero(res[~np.isnan(res)] <= tol)
    assert crossed.size > 0
    k = int(crossed[0])                             # first stop on the recurred residual
    xk = orc.cg(A, b, x0=x0, tol=tol, maxit=k)["x"]  # the iterate at that stop
    rk = b - D @ xk
    assert np.linalg.norm(rk) / np.linalg.norm(b) > 100 * tol   # the branch is taken
    alpha_sd = (rk @ rk) / (rk @ (D @ rk))
    assert abs(full["alpha"][k] - alpha_sd) <= 1e-8 * alpha_sd
    x1 = orc.cg(A, b, x0=x0, tol=tol, maxit=k + 1)["x"]
    step = x1 - xk
    assert np.linalg.norm(step - alpha_sd * rk) <= 1e-6 * np.linalg.norm(alpha_sd * rk)
    assert full["status"] == orc.OK and full["iters"] > k
    assert np.linalg.norm(b - D @ full["x"]) / np.linalg.norm(b) <= tol
