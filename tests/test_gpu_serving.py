"""Request loop through the C ABI: every result meets the tolerance by the
oracle's FP64 residual, and each result is the same alone and in the mix."""
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


def small_pool():
    return [(M.laplacian_2d(20), True), (M.laplacian_3d(10), True),
            (M.graph_laplacian_chung_lu(3000, 21, wmax=300), True),
            (M.convection_diffusion_2d(30, 10.0), False),
            (M.diagonally_dominant(M.power_law_rows(2500, 2.0, 22, rmax=200)), False),
            (M.diagonally_dominant(M.uniform_random(4000, 23, 4, 32)), False),
            (M.laplacian_2d(70), True),                     # n = 4900: worker-stream path
            (M.convection_diffusion_2d(72, 10.0), False)]   # n = 5184: worker-stream path


@pytest.mark.parametrize("precision", [1, 0])
def test_alone_equals_mix_and_tolerance(ck, orc, precision):
    import torch

    from paper_2411_10143_amd.serving import ServingWorkload
    pool = small_pool()
    tol = 1e-8
    say(f"serving precision={precision}")
    W = ServingWorkload(pool, 24, seed=77, tol=tol, precision=precision, small_n=4096,
                        max_slots=8, chunk_iters=16, large_workers=2)
    alone = {}
    for t in range(len(W.mid)):
        say(f"alone request {t} matrix {W.mid[t]}")
        done = W.run(which=[t])
        assert len(done) == 1 and done[0]["status"] == ck.CK_OK, done
        alone[t] = W.x[t].clone()
    say("mix")
    for x in W.x:
        x.fill_(float("nan"))
    done = W.run()
    assert len(done) == len(W.mid)
    st = W.stats()
    for c in done:
        t = c["tag"]
        A = pool[W.mid[t]][0]
        assert c["status"] == ck.CK_OK, c
        x = W.x[t].cpu().numpy()
        assert orc.relres(A, W.b[t].cpu().numpy(), x) <= tol
        if c["path"] == 0:   # batched: the slot's arithmetic does not depend on the mix
            assert torch.equal(W.x[t], alone[t]), (t, c)
        else:                # worker path: same cached configuration, same kernels
            d = (W.x[t] - alone[t]).abs().max().item()
            assert d <= 1e-6 * alone[t].abs().max().item(), (t, d)
    # each matrix is predicted once; every other admission reuses the cached prediction
    assert st["prediction_cache_misses"] <= len(pool)
    assert st["prediction_cache_hits"] + st["prediction_cache_misses"] >= len(done)
    assert st["batched_launches"] > 0
    W.close()


def test_budget_admission_and_eviction(ck, orc):
    from paper_2411_10143_amd.serving import ServingWorkload
    pool = small_pool()
    say("serving tiny budget")
    # room for roughly one matrix and one request at a time: requests queue,
    # idle matrices get evicted and re-ingested, and every solve still finishes
    W = ServingWorkload(pool, 16, seed=5, tol=1e-8, budget_bytes=3 << 20, small_n=4096,
                        max_slots=4, chunk_iters=8, large_workers=1)
    done = W.run()
    st = W.stats()
    assert len(done) == 16 and all(c["status"] == ck.CK_OK for c in done)
    for c in done:
        A = pool[W.mid[c["tag"]]][0]
        assert orc.relres(A, W.b[c["tag"]].cpu().numpy(), W.x[c["tag"]].cpu().numpy()) <= 1e-8
    assert st["evictions"] > 0
    W.close()


def test_poisson_arrivals_latency(ck):
    from paper_2411_10143_amd.serving import ServingWorkload, latency_summary, poisson_arrivals
    say("serving poisson")
    W = ServingWorkload(small_pool(), 40, seed=9, tol=1e-8, small_n=4096)
    cap = latency_summary(W.run())
    arr = poisson_arrivals(40, 0.8 * cap["solves_per_s"], seed=5001)
    done = W.run(arrivals_s=arr)
    lat = latency_summary(done)
    assert lat["ok"] == 40 and lat["p99_ms"] >= lat["p50_ms"] > 0
    # the server's own statistics over the same completions
    st = W.stats()
    assert st["window_completed"] == 40
    assert abs(st["p50_latency_us"] * 1e-3 - lat["p50_ms"]) <= 1e-9 * lat["p50_ms"] + 1e-9
    assert abs(st["p99_latency_us"] * 1e-3 - lat["p99_ms"]) <= 1e-9 * lat["p99_ms"] + 1e-9
    assert abs(st["solves_per_s"] - lat["solves_per_s"]) <= 1e-9 * lat["solves_per_s"]
    W.close()


def _csr_bytes_mixed(A):
    return 4 * (A.n + 1) + 16 * A.nnz


def test_eviction_makes_room_for_a_workspace(ck, orc):
    """The budget holds the second matrix and its GMRES workspace only after
    the first, idle matrix is evicted: the request must still complete
    (it used to wait for memory that nothing would free)."""
    from paper_2411_10143_amd.serving import ServingWorkload
    A = M.laplacian_2d(200)                        # n = 40,000, CG
    B = M.convection_diffusion_2d(200, 10.0)       # n = 40,000, GMRES(30)
    ws_b = (31 * 4 + 24) * ((B.n + 63) // 64 * 64)   # FP32 basis + FP64 vectors
    budget = _csr_bytes_mixed(A) + _csr_bytes_mixed(B) + ws_b - _csr_bytes_mixed(A) // 2
    assert _csr_bytes_mixed(B) + ws_b <= budget < _csr_bytes_mixed(A) + _csr_bytes_mixed(B) + ws_b
    say(f"serving eviction for a workspace, budget {budget}")
    W = ServingWorkload([(A, True), (B, False)], 12, seed=3, tol=1e-8, budget_bytes=budget,
                        small_n=4096, large_workers=1)
    ta = [t for t in range(len(W.mid)) if W.mid[t] == 0][0]
    tb = [t for t in range(len(W.mid)) if W.mid[t] == 1][0]
    for t in (ta, tb, ta):
        done = W.run(which=[t], timeout_s=60)
        assert len(done) == 1 and done[0]["status"] == ck.CK_OK, done
        P = (A, B)[W.mid[t]]
        assert orc.relres(P, W.b[t].cpu().numpy(), W.x[t].cpu().numpy()) <= 1e-8
    assert W.stats()["evictions"] >= 1          # A made way for B's workspace
    W.close()


def test_request_that_can_never_fit_fails(ck):
    from paper_2411_10143_amd.serving import ServingWorkload
    A = M.laplacian_2d(200)
    say("serving request larger than the budget")
    W = ServingWorkload([(A, True), (M.laplacian_2d(10), True)], 6, seed=4, tol=1e-8,
                        budget_bytes=_csr_bytes_mixed(A) // 2, small_n=4096, large_workers=1)
    done = W.run(timeout_s=60)
    assert len(done) == 6
    for c in done:
        if W.mid[c["tag"]] == 0:
            assert c["status"] == ck.CK_E_NOMEM, c
        else:
            assert c["status"] == ck.CK_OK, c
    W.close()


@pytest.mark.timeout(400)
def test_serving_pool_at_full_size(ck, orc):
    """The serving workload's own pool (64 matrices, n log-uniform in
    [1e3, 1e6], CG if symmetric else GMRES(30)), 240 requests with Poisson
    arrivals, mixed precision, tol 1e-8, default slot size: every result
    meets the tolerance by the oracle's FP64 residual, and a seeded subset
    re-solved alone gives the same result (bitwise on batched slots, within
    the tolerance's scale on worker streams)."""
    import torch

    from paper_2411_10143_amd.serving import ServingWorkload, poisson_arrivals
    from synth.workloads import serving_pool
    say("serving pool: generating 64 matrices")
    pool = serving_pool()
    tol = 1e-8
    W = ServingWorkload(pool, 240, seed=5003, tol=tol)
    say("serving pool: 240 requests at 40/s")
    done = W.run(arrivals_s=poisson_arrivals(240, 40.0, seed=5001), timeout_s=300)
    assert len(done) == 240
    by_tag = {c["tag"]: c for c in done}
    xs_mix = {}
    for t, c in by_tag.items():
        A = pool[W.mid[t]][0]
        assert c["status"] == ck.CK_OK, c
        x = W.x[t].cpu().numpy()
        rr = orc.relres(A, W.b[t].cpu().numpy(), x)
        assert rr <= tol, (t, A.name, rr)
        assert abs(rr - c["true_relres"]) <= 1e-3 * rr + 1e-300, (t, rr, c["true_relres"])
        xs_mix[t] = W.x[t].clone()
    paths = {p: [t for t in sorted(by_tag) if by_tag[t]["path"] == p] for p in (0, 1)}
    assert paths[0] and paths[1]
    rng = np.random.default_rng(7)
    subset = list(rng.choice(paths[0], min(10, len(paths[0])), replace=False)) + \
        list(rng.choice(paths[1], min(10, len(paths[1])), replace=False))
    assert len(subset) >= 16
    for t in subset:
        say(f"serving pool: alone request {t} n={pool[W.mid[t]][0].n} path {by_tag[t]['path']}")
        W.x[t].fill_(float("nan"))
        d = W.run(which=[int(t)], timeout_s=120)
        assert len(d) == 1 and d[0]["status"] == ck.CK_OK, d
        if by_tag[t]["path"] == 0:
            assert torch.equal(W.x[t], xs_mix[t]), t
        else:
            diff = (W.x[t] - xs_mix[t]).abs().max().item()
            assert diff <= 1e-6 * xs_mix[t].abs().max().item(), (t, diff)
    st = W.stats()
    assert st["prediction_cache_misses"] <= len(pool)
    W.close()


def test_small_requests_pass_a_waiting_large_one(ck, orc):
    from paper_2411_10143_amd.serving import ServingWorkload
    say("serving admission classes")
    # one worker for large systems: the second large request waits for the
    # first to finish, and the small requests queued behind it are admitted
    # to batched slots meanwhile (each class stays in arrival order)
    pool = [(M.laplacian_2d(150), True), (M.laplacian_2d(20), True)]
    W = ServingWorkload(pool, 40, seed=11, tol=1e-10, precision=0, small_n=4096,
                        max_slots=16, chunk_iters=8, large_workers=1)
    large = [t for t in range(len(W.mid)) if W.mid[t] == 0][:2]
    small = [t for t in range(len(W.mid)) if W.mid[t] == 1][:6]
    assert len(large) == 2 and len(small) == 6
    W.run(which=[large[0]])            # makes both matrices resident and predicted
    W.run(which=[small[0]])
    done = {c["tag"]: c for c in W.run(which=large + small)}
    assert all(c["status"] == ck.CK_OK for c in done.values())
    for t in large + small:
        A = pool[W.mid[t]][0]
        assert orc.relres(A, W.b[t].cpu().numpy(), W.x[t].cpu().numpy()) <= 1e-10
    second = done[large[1]]
    assert second["t_admit_us"] > done[large[0]]["t_admit_us"]
    for t in small:
        assert done[t]["path"] == 0
        assert done[t]["t_admit_us"] < second["t_admit_us"], (done[t], second)
    adm = [done[t]["t_admit_us"] for t in small]
    assert adm == sorted(adm)          # FIFO within the class
    W.close()
