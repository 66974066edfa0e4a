"""The caller-supplied allocator of spmv_create: every device block a handle
needs (its copies in every format, feature and conversion temporaries,
product carries, solve workspaces) comes from it and goes back to it."""
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


class Counting:
    """Wraps torch's caching allocator and records every block."""

    def __init__(self, ck, fail_above=None):
        import torch
        self.live, self.allocs, self.frees, self.streams = {}, 0, 0, set()
        self.fail_above = fail_above

        def alloc(nbytes, stream):
            if self.fail_above is not None and nbytes > self.fail_above:
                return 0
            p = torch.cuda.caching_allocator_alloc(nbytes, torch.cuda.current_device(), stream)
            self.live[p] = nbytes
            self.allocs += 1
            self.streams.add(stream)
            return p

        def free(p, stream):
            assert p in self.live, "free of a block this allocator did not give"
            del self.live[p]
            self.frees += 1
            torch.cuda.caching_allocator_delete(p)

        self.a = ck.CallbackAllocator(alloc, free)


def upload(A):
    import torch
    return (torch.from_numpy(A.rp).cuda(), torch.from_numpy(A.col).cuda(),
            torch.from_numpy(A.val).cuda())


def test_counting_allocator_sees_every_block(ck, orc):
    import torch
    A = M.laplacian_3d(40)                     # n = 64,000: multi-kernel solves
    xs = M.vector(A.n, 1)
    b = orc.spmv(A, xs)
    cnt = Counting(ck)
    rp, col, val = upload(A)
    say("allocator: create")
    Mx = ck.Matrix(rp, col, val, keep_fp32=True, allocator=cnt.a)
    handle_bytes = sum(cnt.live.values())
    assert handle_bytes >= 4 * (A.n + 1) + 16 * A.nnz
    assert cnt.allocs >= 4                     # rowptr, col, val, FP32 val (+ validation flag)
    say("allocator: features and every conversion")
    a0 = cnt.allocs
    n_before = len(cnt.live)
    ck.spmv_features(Mx.handle)
    assert cnt.allocs > a0 and len(cnt.live) == n_before   # scratch taken and given back
    for cid in (8, 9, 10, 11, 12, 13):
        ck.spmv_convert(Mx.handle, ck.config_from_id(cid))
    assert len(cnt.live) > n_before            # the copies live in the caller's memory
    say("allocator: products with carries")
    dx = torch.from_numpy(xs).cuda()
    for cid in range(14):
        dy = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        ck.spmv_apply(Mx.handle, dx, dy, cfg=ck.config_from_id(cid))
        assert np.max(np.abs(dy.cpu().numpy() - b)) <= 1e-12 * np.max(np.abs(b))
    torch.cuda.synchronize()
    resident = set(cnt.live)
    for fn, kw in ((ck.cg_solve, {}), (ck.cg_solve, {"async_": True}),
                   (ck.cg_solve, {"precision": ck.CK_PREC_MIXED}),
                   (ck.gmres_solve, {"config": ck.config_from_id(12)})):
        say(f"allocator: {fn.__name__} {kw}")
        a0 = cnt.allocs
        db = torch.from_numpy(b).cuda()
        x = torch.zeros_like(db)
        r = fn(Mx.handle, db, x, tol=1e-10, **kw)
        assert r["status"] == ck.CK_OK, r
        assert orc.relres(A, b, x.cpu().numpy()) <= 1e-10
        assert cnt.allocs > a0                 # the solve's workspace came from the caller
        # every format is already converted: the workspace is back by the
        # time the call returns, and only the handle's own blocks stay
        assert set(cnt.live) == resident, "a solve workspace is still held"
    say("allocator: destroy")
    Mx.close()
    assert cnt.live == {} and cnt.allocs == cnt.frees


def test_torch_default_allocator_grows_memory_allocated(ck, orc):
    import torch
    A = M.uniform_random(200000, 3, 4, 32)
    rp, col, val = upload(A)
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    say("allocator: torch default")
    Mx = ck.Matrix(rp, col, val)               # the binding's default: torch's allocator
    m1 = torch.cuda.memory_allocated()
    assert m1 - m0 >= 4 * (A.n + 1) + 12 * A.nnz, (m0, m1)
    ck.spmv_convert(Mx.handle, ck.config_from_id(11))   # CSR-panel copy
    m2 = torch.cuda.memory_allocated()
    assert m2 - m1 >= 12 * A.nnz
    Mx.close()
    assert torch.cuda.memory_allocated() == m0


def test_library_cache_without_allocator(ck, orc):
    import torch
    A = M.power_law_rows(30000, 2.0, 5)
    xs = M.vector(A.n, 2)
    b = orc.spmv(A, xs)
    rp, col, val = upload(A)
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    Mx = ck.Matrix(rp, col, val, allocator=None)
    assert torch.cuda.memory_allocated() == m0   # nothing from torch
    for cid in (2, 8, 10, 11, 13):
        dy = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        ck.spmv_convert(Mx.handle, ck.config_from_id(cid))
        ck.spmv_apply(Mx.handle, torch.from_numpy(xs).cuda(), dy, cfg=ck.config_from_id(cid))
        assert np.max(np.abs(dy.cpu().numpy() - b)) <= 1e-12 * max(1.0, np.max(np.abs(b)))
    Mx.close()


def test_allocator_failure_is_nomem(ck, orc):
    import torch
    A = M.laplacian_2d(300)                    # 90,000 rows
    rp, col, val = upload(A)
    say("allocator: NULL at ingest")
    with pytest.raises(ck.CkError) as e:
        ck.Matrix(rp, col, val, allocator=Counting(ck, fail_above=100000).a)
    assert e.value.status == ck.CK_E_NOMEM
    say("allocator: NULL at conversion")
    cnt = Counting(ck)
    Mx = ck.Matrix(rp, col, val, allocator=cnt.a)
    cnt.fail_above = 1 << 20                   # the ELL copy (> 1 MB) cannot be had
    with pytest.raises(ck.CkError) as e:
        ck.spmv_convert(Mx.handle, ck.config_from_id(9))
    assert e.value.status == ck.CK_E_NOMEM
    cnt.fail_above = None
    # the handle still works, and the failed copy left nothing behind on destroy
    xs = M.vector(A.n, 3)
    dy = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    ck.spmv_apply(Mx.handle, torch.from_numpy(xs).cuda(), dy)
    assert np.max(np.abs(dy.cpu().numpy() - orc.spmv(A, xs))) <= 1e-12 * 8
    Mx.close()
    assert cnt.live == {} and cnt.allocs == cnt.frees
