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
    lat = latency_summary(W.run(arrivals_s=arr))
    assert lat["ok"] == 40 and lat["p99_ms"] >= lat["p50_ms"] > 0
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
