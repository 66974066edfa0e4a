"""Request driver for the library's solve server (ck_server_*).

The server (C++, inside libcaskrylov.so) does the scheduling; this module
only prepares device buffers, submits requests at their arrival times and
collects completions:

  * closed loop: every request submitted at t = 0; capacity C = requests /
    makespan (solves/s);
  * open loop: Poisson arrivals (seeded exponential gaps) at rate lambda,
    normally 0.8 C; latency = completion time - arrival (submit) time.
"""
from __future__ import annotations

import time

import numpy as np

from . import _binding as ck


class ServingWorkload:
    """A pool of matrices registered with a server, plus per-request RHS."""

    def __init__(self, pool, n_requests, seed=5003, tol=1e-8, precision=ck.CK_PREC_MIXED,
                 budget_bytes=64 << 30, max_slots=256, chunk_iters=8, small_n=8192,
                 large_workers=8, restart=30, max_iter=100000):
        import torch
        self.pool = pool
        self.tol = tol
        self.srv = ck.server_create(budget_bytes, max_slots, chunk_iters, small_n, large_workers,
                                    precision, restart, max_iter, tol)
        self.dev = []
        for i, (A, _sym) in enumerate(pool):
            rp = torch.from_numpy(A.rp).cuda()
            col = torch.from_numpy(A.col).cuda()
            val = torch.from_numpy(A.val).cuda()
            self.dev.append((rp, col, val))
            ck.server_add_matrix(self.srv, i, rp, col, val)
        rng = np.random.default_rng(seed)
        self.mid = rng.integers(0, len(pool), size=n_requests)
        # b = A x* with x* uniform in [-1, 1] (one fresh x* per request)
        self.b, self.x, self.xstar = [], [], []
        handles = {}
        for t, m in enumerate(self.mid):
            A = pool[m][0]
            if m not in handles:
                rp, col, val = self.dev[m]
                handles[m] = ck.Matrix(rp, col, val)
            xs = torch.from_numpy(rng.uniform(-1, 1, A.n)).cuda()
            b = torch.zeros_like(xs)
            ck.spmv_apply(handles[m].handle, xs, b)
            self.b.append(b)
            self.x.append(torch.zeros_like(b))
            self.xstar.append(xs)
        for h in handles.values():
            h.close()
        torch.cuda.synchronize()

    def run(self, arrivals_s=None, which=None, timeout_s=1800.0, progress=None, every_s=30.0):
        """Submit requests (all of `which`, default every one) at the given
        arrival offsets (seconds, None = all at once); returns completions.
        `progress(text)` is called about every `every_s` seconds."""
        idx = list(range(len(self.mid))) if which is None else list(which)
        arr = np.zeros(len(idx)) if arrivals_s is None else np.asarray(arrivals_s)
        done = []
        ck.server_reset_stats(self.srv)    # the server's latency window = this run
        t0 = time.perf_counter()
        last = [t0]

        def tick(submitted):
            now = time.perf_counter()
            if progress and now - last[0] >= every_s:
                last[0] = now
                progress(f"{now - t0:.0f}s: {submitted} submitted, {len(done)} collected")

        for k, t in enumerate(idx):
            while True:
                wait = t0 + arr[k] - time.perf_counter()
                if wait <= 0:
                    break
                done += ck.server_poll(self.srv)
                tick(k)
                time.sleep(min(wait, 2e-4))
            ck.server_submit(self.srv, int(self.mid[t]), self.b[t], self.x[t], t)
        end = time.perf_counter() + timeout_s
        while len(done) < len(idx):
            done += ck.server_poll(self.srv, 1 << 16)
            tick(len(idx))
            if time.perf_counter() > end:
                ck.server_drain(self.srv, 0.0)   # raises: requests still open
            time.sleep(1e-3)
        return done

    def stats(self):
        """Counters since creation; p50/p99 latency and solves/s of the last run."""
        return ck.server_stats(self.srv)

    def close(self):
        if self.srv:
            ck.server_destroy(self.srv)
            self.srv = None


def poisson_arrivals(n, rate, seed=5001):
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, size=n)
    return np.cumsum(gaps) - gaps[0]


def latency_summary(done):
    lat = np.array([(c["t_done_us"] - c["t_submit_us"]) * 1e-3 for c in done])
    span = (max(c["t_done_us"] for c in done) - min(c["t_submit_us"] for c in done)) * 1e-6
    return dict(solves=len(done), solves_per_s=len(done) / span if span > 0 else float("nan"),
                p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                mean_ms=float(lat.mean()), makespan_s=span,
                batched=int(sum(c["path"] == 0 for c in done)),
                ok=int(sum(c["status"] == ck.CK_OK for c in done)))
