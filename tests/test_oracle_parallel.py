"""The OpenMP build of the oracle (the all-core CPU baseline) gives the same
bits as the single-threaded build: rows are shared out among threads, and
each row is still summed alone in ascending order."""
import numpy as np

from synth import matrices as M


def test_parallel_spmv_and_cg_bitwise_equal(orc):
    orc.build(force=False)
    mats = [M.power_law_rows(20000, 1.8, 3, rmax=2000), M.laplacian_3d(20),
            M.uniform_random(5000, 4, 4, 64), M.random_integer(300, 900, 5, density=0.05),
            M.laplacian_1d(1)]
    for A in mats:
        x = M.vector(A.ncols, 6)
        y0 = M.vector(A.n, 7)
        for alpha, beta in ((1.0, 0.0), (-0.5, 2.0)):
            a = orc.spmv(A, x, alpha, beta, y0)
            b = orc.spmv(A, x, alpha, beta, y0, parallel=True)
            assert np.array_equal(a, b), A.name
    A = M.laplacian_2d(40)
    b = orc.spmv(A, M.vector(A.n, 8))
    r1 = orc.cg(A, b, tol=1e-10)
    r2 = orc.cg(A, b, tol=1e-10, parallel=True)
    assert r1["iters"] == r2["iters"] and np.array_equal(r1["x"], r2["x"])
    assert orc.threads(parallel=True) >= 1 and orc.threads(parallel=False) == 1
