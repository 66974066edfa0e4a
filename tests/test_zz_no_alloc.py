"""spmv_apply_noalloc (the allocation-free product) through the C ABI: its
output equals spmv_apply's bit for bit on every configuration, on two calls
in a row (the second on a smaller matrix, over the first call's leftovers in
the shared scratch array), and a product whose workspace exceeds the fixed
array is refused with CK_E_UNSUPPORTED."""
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


def _products(ck, orc, A, seed, cids, alpha, beta):
    import torch
    Mx = ck.Matrix.from_csr(A)
    xs = M.vector(A.ncols, seed)
    y0 = M.vector(A.n, seed + 1)
    dx = torch.from_numpy(xs).cuda()
    ref = orc.spmv(A, xs, alpha, beta, y0)
    for cid in cids:
        cfg = ck.config_from_id(cid)
        try:
            ck.spmv_convert(Mx.handle, cfg)
        except ck.CkError as e:
            if e.status == ck.CK_E_UNSUPPORTED:     # ELL / DIA refused for fill
                continue
            raise
        say(f"noalloc n={A.n} config {cid}")
        y_ref = torch.from_numpy(y0).cuda()
        y_na = torch.from_numpy(y0).cuda()
        y_na_nan = torch.full_like(y_na, float("nan"))
        ck.spmv_apply(Mx.handle, dx, y_ref, alpha, beta, cfg)
        ck.spmv_apply_noalloc(Mx.handle, dx, y_na, alpha, beta, cfg)
        torch.cuda.synchronize()
        assert torch.equal(y_na, y_ref), cid
        scale = np.max(np.abs(ref)) + 1e-300
        assert np.max(np.abs(y_na.cpu().numpy() - ref)) <= 1e-12 * scale, cid
        if beta == 0.0:      # y is not read
            ck.spmv_apply_noalloc(Mx.handle, dx, y_na_nan, alpha, 0.0, cfg)
            torch.cuda.synchronize()
            assert torch.equal(y_na_nan, y_ref), cid
    Mx.close()


def test_noalloc_equals_spmv_apply_two_calls(ck, orc):
    cids = list(range(14))
    # first a larger matrix, then a smaller one over its leftovers
    _products(ck, orc, M.power_law_rows(60000, 1.8, 41, rmax=3000), 1, cids, 1.0, 0.0)
    _products(ck, orc, M.uniform_random(7000, 42, 4, 40), 3, cids, -0.5, 2.0)


def test_noalloc_ragged_and_rectangular(ck, orc):
    A = M.random_integer(333, 1201, 43, density=0.05)
    _products(ck, orc, A, 5, [2, 7, 8, 10, 11], 1.0, 0.0)
    _products(ck, orc, M.laplacian_1d(1), 7, [2, 8, 10, 11], 2.0, 1.0)


def test_noalloc_refuses_a_workspace_above_its_array(ck):
    import torch
    n = 3_000_000          # CSR-panel: 16 panels x 3M rows x 8 B of partial sums > 64 MiB
    rp = torch.arange(n + 1, dtype=torch.int32, device="cuda")
    col = torch.arange(n, dtype=torch.int32, device="cuda")
    val = torch.ones(n, dtype=torch.float64, device="cuda")
    Mx = ck.Matrix(rp, col, val)
    cfg = ck.config_from_id(11)
    ck.spmv_convert(Mx.handle, cfg)
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    say("noalloc refusal")
    with pytest.raises(ck.CkError) as e:
        ck.spmv_apply_noalloc(Mx.handle, x, y, cfg=cfg)
    assert e.value.status == ck.CK_E_UNSUPPORTED
    # the merge path on the same matrix fits, and matches spmv_apply
    m = ck.config_from_id(8)
    ck.spmv_convert(Mx.handle, m)
    y2 = torch.zeros_like(y)
    ck.spmv_apply_noalloc(Mx.handle, x, y, cfg=m)
    ck.spmv_apply(Mx.handle, x, y2, cfg=m)
    torch.cuda.synchronize()
    assert torch.equal(y, y2) and bool((y == 1.0).all())
    Mx.close()
