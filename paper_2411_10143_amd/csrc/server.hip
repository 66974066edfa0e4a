// Request loop for solve requests (continuous batching, HBM-budget admission,
// resident matrices with a per-matrix prediction cache).
//
// A scheduler thread owns the device-side state:
//   - requests wait in arrival order until their matrix is resident and
//     their workspace fits the memory budget (least-recently-used idle
//     matrices are evicted to make room, for the matrix, for its converted
//     copy and for the workspace; a request that still does not fit waits,
//     and nothing behind it is admitted meanwhile, unless nothing is in
//     flight: then it can never fit and completes with CK_E_NOMEM).  Small and large
//     requests are FIFO within their class, but a request waiting only for a
//     slot (small) or a worker (large) does not hold back the other class;
//   - the first request on a matrix runs GPU features + the cascade once; the
//     decision (configuration, symmetric or not) is cached for the matrix;
//   - small systems (n <= small_n) take a slot of the batched chunk kernel,
//     which advances every occupied slot by `chunk_iters` iterations per
//     launch; finished slots are retired and new requests admitted between
//     launches;
//   - larger systems run cg_solve / gmres_solve with the cached configuration
//     on worker threads, each with its own stream, overlapping the batched
//     launches on the device.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <thread>
#include <vector>

#include "admit.hpp"
#include "batched.hpp"
#include "matrix.hpp"
#include "panel.hpp"
#include "predictor.hpp"
#include "solvers.hpp"

namespace ck {
ck_status compute_features(ck_matrix &M, ck_features &F, hipStream_t s, bool symmetry);
ck_status convert_format(ck_matrix &M, const ck_config &c, hipStream_t s);
}  // namespace ck

using namespace ck;

namespace {

using Clock = std::chrono::steady_clock;

struct MatEntry {
    int id = 0;
    int64_t n = 0, nnz = 0;
    const int32_t *rp = nullptr, *col = nullptr;   // caller's arrays (kept alive by the caller)
    const double *val = nullptr;
    ck_handle h = nullptr;          // resident copy, or null when evicted
    int64_t bytes = 0;              // bytes of the resident copy
    int in_flight = 0;
    bool predicted = false;
    bool symmetric = false;
    ck_config cfg{};                // cached cascade decision
    int64_t conv_bytes = 0;         // estimated bytes of its converted copy
    ck_config run_cfg{};            // what the resident copy runs (cfg, or the
                                    // default when cfg's copy did not fit)
    uint64_t last_use = 0;
};

struct Request {
    int64_t tag = 0;
    int matrix = 0;
    const double *b = nullptr;
    double *x = nullptr;
    double t_submit = 0, t_admit = 0;
    int64_t bytes = 0;
    int slot = -1;
    void *work = nullptr;
    double *r64 = nullptr;
};

}  // namespace

struct ck_server {
    ck_server_opts o{};
    Clock::time_point t0;
    hipStream_t stream = nullptr;
    int device = 0;
    // batched slots
    BSlot *slots = nullptr;
    BStat *stat = nullptr;
    BStat *stat_host = nullptr;
    int *active_dev = nullptr;
    int *active_host = nullptr;
    std::vector<Request *> slot_req;
    std::vector<BSlot> slot_init;
    // bookkeeping
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> submitted, pending;
    std::vector<ck_completion> done;
    std::map<int, MatEntry> mats;
    int64_t bytes_in_use = 0;
    uint64_t use_clock = 0;
    uint64_t epoch = 0;             // completions so far (wakes the scheduler)
    ck_server_stats st{};
    // latency window (since creation or ck_server_reset_stats)
    std::vector<double> lat_us;
    double win_first_submit = 0, win_last_done = 0;
    // large-system workers
    std::deque<Request *> large_q;
    std::mutex lq_mu;
    std::condition_variable lq_cv;
    std::vector<std::thread> workers;
    int large_running = 0;
    std::thread sched;
    std::atomic<bool> stop{false};
    double now() const { return std::chrono::duration<double, std::micro>(Clock::now() - t0).count(); }
};

namespace {

int64_t handle_bytes(const ck_matrix &M) {
    int64_t b = 4 * (M.n + 1) + 12 * M.nnz;
    if (M.val32)
        b += 4 * M.nnz;
    if (M.has_ell.load())
        b += M.ell_K * M.ell_pitch * (12 + (M.ell_val32 ? 4 : 0));
    if (M.has_coo.load())
        b += 4 * M.nnz;
    if (M.has_dia.load())
        b += 4 * M.dia_nd + M.dia_nd * M.dia_pitch * (8 + (M.dia_val32 ? 4 : 0));
    if (M.has_hyb.load())
        b += 4 * M.hyb_nt + M.hyb_K * M.hyb_pitch * (12 + (M.hyb_val32 ? 4 : 0));
    if (M.has_panel.load())
        b += 4 * (M.panel_rows + 1) + M.nnz * (12 + (M.panel_val32 ? 4 : 0)) +
             (M.panel_row ? 4 * M.panel_rows + 4 * (int64_t)M.panel_P * (M.panel_B + 1) : 0);
    return b;
}

int64_t csr_bytes(const ck_server &S, const MatEntry &e) {
    return 4 * (e.n + 1) + (S.o.precision == CK_PREC_MIXED ? 16 : 12) * e.nnz;
}

// Bytes a conversion to c adds to the handle (upper estimates from the
// features; 0 for a configuration that needs no copy or is refused), plus
// the conversion's own temporaries.
int64_t converted_bytes(const ck_features &F, const ck_config &c, bool fp32) {
    const int64_t n = F.nrows, nnz = F.nnz;
    const int64_t pitch = ceil_div(std::max<int64_t>(n, 1), 64) * 64;
    const int64_t vb = fp32 ? 12 : 8;          // value bytes per slot (FP64 + FP32 copy)
    const int64_t tmp = 8 * (n + F.ncols) + 4096;
    if (c.format == CK_FMT_ELL)
        return F.max_r * pitch > 8 * nnz ? 0 : F.max_r * pitch * (4 + vb) + tmp;
    if (c.format == CK_FMT_COO)
        return 4 * nnz + tmp;
    if (c.format == CK_FMT_DIA)
        return F.ndiag * pitch > 8 * nnz ? 0 : F.ndiag * pitch * vb + 4 * F.ndiag + tmp;
    if (c.format == CK_FMT_HYB)   // width K <= 3 nnz / n
        return (3 * nnz + pitch) * (4 + vb) + 4 * n + tmp;
    if (c.format == CK_FMT_CSR && c.algorithm == CK_ALG_PANEL) {
        const int64_t P = panel_count_for(F.ncols, 8);
        return 4 * (P * n + 1) + nnz * (4 + vb) + 8 * (P * n + 1) + tmp;
    }
    if (c.format == CK_FMT_CSR && c.algorithm == CK_ALG_MERGE)
        return 4 * ((n + nnz) / 1024 + 2) + tmp;
    return 0;
}

int64_t request_bytes(const ck_server &S, const MatEntry &e, bool small) {
    const int m = S.o.restart > 0 ? S.o.restart : 30;
    const int64_t ld = ceil_div(std::max<int64_t>(e.n, 1), 64) * 64;
    const int s = S.o.precision == CK_PREC_MIXED ? 4 : 8;
    if (small)
        return bslot_work_elems(e.symmetric ? B_CG : B_GMRES, e.n, m) * s + 8 * ld;
    // large solver workspace (upper estimate)
    return e.symmetric ? (8 + 6 * s) * ld : (int64_t)(m + 1) * s * ld + 24 * ld;
}

// Posts a completion (S.mu held).
void post(ck_server &S, Request *r, int status, int iters, double relres, int path, int cfg) {
    ck_completion c{};
    c.tag = r->tag;
    c.matrix_id = r->matrix;
    c.status = status;
    c.iterations = iters;
    c.path = path;
    c.config_id = cfg;
    c.true_relres = relres;
    c.t_submit_us = r->t_submit;
    c.t_admit_us = r->t_admit;
    c.t_done_us = S.now();
    S.done.push_back(c);
    S.st.completed += 1;
    if (S.lat_us.empty() || c.t_submit_us < S.win_first_submit)
        S.win_first_submit = c.t_submit_us;
    S.win_last_done = std::max(S.win_last_done, c.t_done_us);
    S.lat_us.push_back(c.t_done_us - c.t_submit_us);
    S.epoch += 1;
    S.cv.notify_all();
}

void complete(ck_server &S, Request *r, int status, int iters, double relres, int path,
              int cfg) {
    std::lock_guard<std::mutex> lk(S.mu);
    post(S, r, status, iters, relres, path, cfg);
    S.st.in_flight -= 1;
    S.bytes_in_use -= r->bytes;
    S.mats[r->matrix].in_flight -= 1;
}

// Evicts least-recently-used idle matrices other than `keep` until `need`
// more bytes fit the budget; false if they still do not.  Scheduler thread,
// S.mu held.
bool make_room(ck_server &S, const MatEntry *keep, int64_t need) {
    while (S.bytes_in_use + need > S.o.budget_bytes) {
        MatEntry *victim = nullptr;
        for (auto &kv : S.mats) {
            MatEntry &c = kv.second;
            if (c.h && c.in_flight == 0 && &c != keep && (!victim || c.last_use < victim->last_use))
                victim = &c;
        }
        if (!victim)
            return false;   // in-flight work holds the memory
        (void)hipStreamSynchronize(S.stream);
        spmv_destroy(victim->h);
        victim->h = nullptr;
        S.bytes_in_use -= victim->bytes;
        victim->bytes = 0;
        S.st.evictions += 1;
        S.st.resident_matrices -= 1;
    }
    return true;
}

// Makes the matrix resident (evicting idle ones if needed) and fills its
// prediction cache; the cascade's configuration runs only if its converted
// copy fits the budget too (else the default configuration).  CK_E_NOMEM:
// it does not fit now.  Called by the scheduler thread only, S.mu held.
ck_status ensure_resident(ck_server &S, MatEntry &e) {
    e.last_use = ++S.use_clock;
    if (e.h) {
        S.st.prediction_cache_hits += 1;   // resident, and predicted when first made so
        return CK_OK;
    }
    const bool fp32 = S.o.precision == CK_PREC_MIXED;
    // the CSR copy, plus the feature pass's scratch the first time
    const int64_t feat = e.predicted ? 0 : 2 * e.n + 4096;
    if (!make_room(S, &e, csr_bytes(S, e) + feat))
        return CK_E_NOMEM;
    CK_TRY(spmv_create(&e.h, e.n, e.n, e.nnz, e.rp, e.col, e.val, fp32 ? CK_KEEP_FP32 : 0u,
                       nullptr, S.stream));
    e.bytes = handle_bytes(*e.h);
    S.bytes_in_use += e.bytes;
    S.st.resident_matrices += 1;
    if (!e.predicted) {
        S.st.prediction_cache_misses += 1;
        ck_features F;
        if (compute_features(*e.h, F, S.stream, true) == CK_OK) {
            e.symmetric = F.is_symmetric != 0;
            if (spmv_select(&F, nullptr, &e.cfg) != CK_OK)
                e.cfg = default_config(e.n, e.nnz);
            e.conv_bytes = converted_bytes(F, e.cfg, fp32);
        } else {   // no features: the default kernel, and GMRES (no symmetry known)
            e.symmetric = false;
            e.cfg = default_config(e.n, e.nnz);
            e.conv_bytes = 0;
        }
        e.predicted = true;
    } else {
        S.st.prediction_cache_hits += 1;
    }
    e.run_cfg = e.cfg;
    if (e.n > S.o.small_n) {
        // the copy must leave room for a request's workspace beside it
        if (!make_room(S, &e, e.conv_bytes + request_bytes(S, e, false)) ||
            convert_format(*e.h, e.cfg, S.stream) != CK_OK)
            e.run_cfg = default_config(e.n, e.nnz);   // no room, or refused: default kernel
        S.bytes_in_use -= e.bytes;
        e.bytes = handle_bytes(*e.h);
        S.bytes_in_use += e.bytes;
    }
    return CK_OK;
}

int lanes_for(const MatEntry &e) {
    if (e.run_cfg.format == CK_FMT_CSR && e.run_cfg.algorithm == CK_ALG_VECTOR &&
        e.run_cfg.lanes >= 1)
        return e.run_cfg.lanes;
    return default_config(e.n, e.nnz).lanes;
}

// A request that does not fit: it waits while in-flight work holds memory
// that will come back; with nothing in flight it can never fit, and is
// completed with CK_E_NOMEM (S.mu held).
Admit no_room(ck_server &S, Request *r) {
    if (S.st.in_flight > 0)
        return WAIT_MEMORY;
    r->t_admit = S.now();
    post(S, r, CK_E_NOMEM, 0, -1.0, S.mats[r->matrix].n <= S.o.small_n ? 0 : 1, -1);
    delete r;
    return REJECTED;
}

// Tries to admit a request.  WAIT_CLASS: every slot (small) or worker (large)
// is taken; WAIT_MEMORY: the matrix or the workspace does not fit the budget
// (or an allocation failed), so no later request may pass it; REJECTED: it
// can never fit (completed with an error).  S.mu held.
Admit admit_one(ck_server &S, Request *r) {
    MatEntry &e = S.mats[r->matrix];
    const bool small = e.n <= S.o.small_n;
    int slot = -1;
    if (small) {
        for (int i = 0; i < S.o.max_slots; ++i)
            if (!S.slot_req[i]) {
                slot = i;
                break;
            }
        if (slot < 0)
            return WAIT_CLASS;
    } else if (S.large_running >= S.o.large_workers) {
        return WAIT_CLASS;
    }
    // prediction first (needs the matrix), then the request's own workspace
    if (ensure_resident(S, e) != CK_OK)
        return no_room(S, r);
    const int64_t need = request_bytes(S, e, small);
    if (!make_room(S, &e, need))
        return no_room(S, r);
    r->bytes = need;
    r->t_admit = S.now();
    S.bytes_in_use += need;
    e.in_flight += 1;
    S.st.in_flight += 1;
    if (!small) {
        S.large_running += 1;
        std::lock_guard<std::mutex> lk(S.lq_mu);
        S.large_q.push_back(r);
        S.lq_cv.notify_one();
        return ADMITTED;
    }
    // batched slot: workspace + slot record
    const int m = std::min(S.o.restart > 0 ? S.o.restart : 30, kBMaxM);
    const int kind = e.symmetric ? B_CG : B_GMRES;
    const bool fp32 = S.o.precision == CK_PREC_MIXED;
    const int64_t ld = ceil_div(std::max<int64_t>(e.n, 1), 64) * 64;
    if (hipMallocAsync(&r->work, (size_t)bslot_work_elems(kind, e.n, m) * (fp32 ? 4 : 8),
                       S.stream) != hipSuccess ||
        hipMallocAsync((void **)&r->r64, (size_t)ld * 8, S.stream) != hipSuccess) {
        (void)hipGetLastError();
        if (r->work)
            (void)hipFreeAsync(r->work, S.stream);
        r->work = nullptr;
        S.bytes_in_use -= need;
        e.in_flight -= 1;
        S.st.in_flight -= 1;
        return no_room(S, r);
    }
    BSlot &b = S.slot_init[slot];
    std::memset(&b, 0, sizeof b);
    b.kind = kind;
    b.n = (int)e.n;
    b.lanes = lanes_for(e);
    b.m = m;
    b.rp = e.h->rp;
    b.col = e.h->col;
    b.val64 = e.h->val;
    b.val32 = e.h->val32;
    b.b = r->b;
    b.x = r->x;
    b.r64 = r->r64;
    b.work = r->work;
    b.ld = ld;
    b.bnorm = -1.0;
    b.tol = S.o.tol;
    b.max_iter = S.o.max_iter;
    b.inner_cap = std::max(50, (int)(4.0 * std::sqrt((double)e.n)));
    b.phase = B_OUTER;
    b.status = RUN;
    if (hipMemcpyAsync(S.slots + slot, &b, sizeof b, hipMemcpyHostToDevice, S.stream) !=
        hipSuccess) {
        (void)hipGetLastError();
        (void)hipFreeAsync(r->work, S.stream);
        (void)hipFreeAsync(r->r64, S.stream);
        r->work = nullptr;
        r->r64 = nullptr;
        S.bytes_in_use -= need;
        e.in_flight -= 1;
        S.st.in_flight -= 1;
        return no_room(S, r);
    }
    S.slot_req[slot] = r;
    r->slot = slot;
    return ADMITTED;
}

void scheduler(ck_server *Sp) {
    ck_server &S = *Sp;
    (void)hipSetDevice(S.device);
    const bool fp32 = S.o.precision == CK_PREC_MIXED;
    bool stalled = false;   // the last scan admitted nothing and no slot ran
    while (true) {
        {
            std::unique_lock<std::mutex> lk(S.mu);
            bool busy = false;
            for (Request *r : S.slot_req)
                busy |= r != nullptr;
            // nothing to launch and nothing admissible: sleep until a request
            // arrives or one completes (submit and complete notify cv)
            if (!busy && S.submitted.empty() && !S.stop && (S.pending.empty() || stalled)) {
                const uint64_t ep = S.epoch;
                S.cv.wait_for(lk, std::chrono::milliseconds(20), [&] {
                    return S.stop || !S.submitted.empty() || S.epoch != ep;
                });
            }
            if (S.stop)
                break;
            while (!S.submitted.empty()) {
                S.pending.push_back(S.submitted.front());
                S.submitted.pop_front();
            }
            S.st.queued = (int64_t)S.pending.size();
        }
        // admit in arrival order while slots, workers and memory allow (each
        // path first-come first-served; a request waiting for memory stops
        // both)
        int moved = 0;
        admit_scan(S.pending, [&](Request *r, const bool *blocked) {
            std::lock_guard<std::mutex> lk(S.mu);
            const int cls = S.mats.at(r->matrix).n <= S.o.small_n ? 0 : 1;
            const Admit a = blocked[cls] ? WAIT_CLASS : admit_one(S, r);
            moved += a == ADMITTED || a == REJECTED;
            return std::make_pair(cls, a);
        });
        // one batched launch over the occupied slots
        int na = 0;
        for (int i = 0; i < S.o.max_slots; ++i)
            if (S.slot_req[i])
                S.active_host[na++] = i;
        stalled = moved == 0 && na == 0;
        if (na > 0) {
            if (hipMemcpyAsync(S.active_dev, S.active_host, na * sizeof(int),
                               hipMemcpyHostToDevice, S.stream) != hipSuccess ||
                launch_batched_chunk(S.slots, S.stat, S.active_dev, na, S.o.chunk_iters, fp32,
                                     S.stream) != CK_OK ||
                hipMemcpyAsync(S.stat_host, S.stat, S.o.max_slots * sizeof(BStat),
                               hipMemcpyDeviceToHost, S.stream) != hipSuccess ||
                hipStreamSynchronize(S.stream) != hipSuccess) {
                // a failed launch ends the occupied slots with an error
                (void)hipGetLastError();
                for (int t = 0; t < na; ++t) {
                    const int i = S.active_host[t];
                    Request *r = S.slot_req[i];
                    S.slot_req[i] = nullptr;
                    complete(S, r, CK_E_HIP, 0, -1.0, 0, -1);
                    delete r;
                }
                continue;
            }
            {
                std::lock_guard<std::mutex> lk(S.mu);
                S.st.batched_launches += 1;
            }
            for (int t = 0; t < na; ++t) {
                const int i = S.active_host[t];
                const BStat &bs = S.stat_host[i];
                if (bs.phase != B_DONE)
                    continue;
                Request *r = S.slot_req[i];
                S.slot_req[i] = nullptr;
                const int status = bs.status == CONVERGED ? CK_OK
                                   : bs.status == BREAKDOWN ? CK_E_BREAKDOWN
                                                            : CK_E_NOT_CONVERGED;
                (void)hipFreeAsync(r->work, S.stream);
                (void)hipFreeAsync(r->r64, S.stream);
                int cid;
                {
                    std::lock_guard<std::mutex> lk(S.mu);
                    cid = ck_config_id(&S.mats[r->matrix].run_cfg);
                }
                complete(S, r, status, bs.iter, bs.relres, 0, cid);
                delete r;
            }
        }
    }
}

void large_worker(ck_server *Sp) {
    ck_server &S = *Sp;
    (void)hipSetDevice(S.device);
    hipStream_t s = nullptr;
    (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    while (true) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(S.lq_mu);
            S.lq_cv.wait(lk, [&] { return S.stop || !S.large_q.empty(); });
            if (S.large_q.empty())
                break;
            r = S.large_q.front();
            S.large_q.pop_front();
        }
        MatEntry *e;
        ck_config run_cfg;
        {
            std::lock_guard<std::mutex> lk(S.mu);
            e = &S.mats[r->matrix];
            run_cfg = e->run_cfg;
        }
        ck_solve_opts o{};
        o.tol = S.o.tol;
        o.max_iter = S.o.max_iter;
        o.restart = S.o.restart > 0 ? S.o.restart : 30;
        o.precision = S.o.precision;
        o.check_every = 8;
        o.use_config = 1;
        o.config = run_cfg;
        ck_solve_result res{};
        ck_status st = launch_fill<double>(e->n, r->x, 0.0, s);   // x0 = 0
        if (st == CK_OK)
            st = e->symmetric ? cg_solve(e->h, r->b, r->x, &o, &res, s)
                              : gmres_solve(e->h, r->b, r->x, &o, &res, s);
        {
            std::lock_guard<std::mutex> lk(S.mu);
            S.large_running -= 1;
        }
        complete(S, r, st, res.iterations, res.true_relres, 1, ck_config_id(&run_cfg));
        delete r;
    }
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
}

}  // namespace

extern "C" {

ck_status ck_server_create(const ck_server_opts *o, ck_server_t *out) {
    if (!o || !out)
        return fail(CK_E_INVALID, "NULL argument");
    *out = nullptr;
    if (o->max_slots <= 0 || o->max_slots > 4096 || o->chunk_iters <= 0 || o->budget_bytes <= 0 ||
        o->large_workers <= 0 || o->large_workers > 16 || o->restart > kMaxRestart ||
        !(o->tol >= 0))
        return fail(CK_E_INVALID, "bad server options");
    ck_server *S = new ck_server();
    S->o = *o;
    if (S->o.max_iter <= 0)
        S->o.max_iter = 100000;
    S->t0 = Clock::now();
    (void)hipGetDevice(&S->device);
    ck_status st = CK_OK;
    if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc((void **)&S->slots, sizeof(BSlot) * o->max_slots) != hipSuccess ||
        hipMalloc((void **)&S->stat, sizeof(BStat) * o->max_slots) != hipSuccess ||
        hipMalloc((void **)&S->active_dev, sizeof(int) * o->max_slots) != hipSuccess ||
        hipHostMalloc((void **)&S->stat_host, sizeof(BStat) * o->max_slots, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&S->active_host, sizeof(int) * o->max_slots, hipHostMallocDefault) != hipSuccess)
        st = fail(CK_E_HIP, "server allocation failed");
    if (st != CK_OK) {
        (void)hipGetLastError();
        ck_server_destroy(S);
        return st;
    }
    S->slot_req.assign(o->max_slots, nullptr);
    S->slot_init.resize(o->max_slots);
    S->sched = std::thread(scheduler, S);
    for (int i = 0; i < o->large_workers; ++i)
        S->workers.emplace_back(large_worker, S);
    *out = S;
    return CK_OK;
}

ck_status ck_server_add_matrix(ck_server_t S, int32_t id, int64_t n, int64_t nnz,
                               const int32_t *d_rowptr, const int32_t *d_col,
                               const double *d_val) {
    if (!S || n <= 0 || nnz < 0 || !d_rowptr || (nnz > 0 && (!d_col || !d_val)))
        return fail(CK_E_INVALID, "bad matrix");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->mats.count(id))
        return fail(CK_E_INVALID, "matrix id %d already registered", id);
    MatEntry e;
    e.id = id;
    e.n = n;
    e.nnz = nnz;
    e.rp = d_rowptr;
    e.col = d_col;
    e.val = d_val;
    S->mats[id] = e;
    return CK_OK;
}

ck_status ck_server_submit(ck_server_t S, int32_t matrix_id, const double *d_b, double *d_x,
                           int64_t tag) {
    if (!S || !d_b || !d_x)
        return fail(CK_E_INVALID, "NULL argument");
    Request *r = new Request();
    r->tag = tag;
    r->matrix = matrix_id;
    r->b = d_b;
    r->x = d_x;
    std::lock_guard<std::mutex> lk(S->mu);
    if (!S->mats.count(matrix_id)) {
        delete r;
        return fail(CK_E_INVALID, "unknown matrix id %d", matrix_id);
    }
    r->t_submit = S->now();
    S->submitted.push_back(r);
    S->st.submitted += 1;
    S->cv.notify_all();
    return CK_OK;
}

int32_t ck_server_poll(ck_server_t S, ck_completion *out, int32_t cap) {
    if (!S || !out || cap <= 0)
        return 0;
    std::lock_guard<std::mutex> lk(S->mu);
    const int k = (int)std::min<size_t>(cap, S->done.size());
    for (int i = 0; i < k; ++i)
        out[i] = S->done[i];
    S->done.erase(S->done.begin(), S->done.begin() + k);
    return k;
}

ck_status ck_server_drain(ck_server_t S, double timeout_s) {
    if (!S)
        return fail(CK_E_INVALID, "NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    const bool ok = S->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] {
        return S->st.completed == S->st.submitted;
    });
    return ok ? CK_OK : fail(CK_E_NOT_CONVERGED, "drain timed out");
}

// q-quantile of sorted v by linear interpolation between closest ranks
static double quantile(const std::vector<double> &v, double q) {
    if (v.empty())
        return 0.0;
    const double pos = q * (double)(v.size() - 1);
    const size_t lo = (size_t)pos;
    const size_t hi = std::min(lo + 1, v.size() - 1);
    return v[lo] + (pos - (double)lo) * (v[hi] - v[lo]);
}

ck_status ck_server_get_stats(ck_server_t S, ck_server_stats *out) {
    if (!S || !out)
        return fail(CK_E_INVALID, "NULL argument");
    std::vector<double> lat;
    double span;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        *out = S->st;
        out->bytes_in_use = S->bytes_in_use;
        lat = S->lat_us;
        span = S->win_last_done - S->win_first_submit;
    }
    std::sort(lat.begin(), lat.end());
    out->window_completed = (int64_t)lat.size();
    out->p50_latency_us = quantile(lat, 0.50);
    out->p99_latency_us = quantile(lat, 0.99);
    out->solves_per_s = span > 0 ? (double)lat.size() / (span * 1e-6) : 0.0;
    return CK_OK;
}

ck_status ck_server_reset_stats(ck_server_t S) {
    if (!S)
        return fail(CK_E_INVALID, "NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    S->lat_us.clear();
    S->win_first_submit = 0;
    S->win_last_done = 0;
    return CK_OK;
}

double ck_server_clock_us(ck_server_t S) { return S ? S->now() : 0.0; }

void ck_server_destroy(ck_server_t S) {
    if (!S)
        return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    {
        std::lock_guard<std::mutex> lk(S->lq_mu);
        S->lq_cv.notify_all();
    }
    if (S->sched.joinable())
        S->sched.join();
    for (auto &w : S->workers)
        if (w.joinable())
            w.join();
    for (Request *r : S->slot_req)
        if (r) {   // stream-ordered, like every other slot workspace
            (void)hipFreeAsync(r->work, S->stream);
            (void)hipFreeAsync(r->r64, S->stream);
            delete r;
        }
    if (S->stream)
        (void)hipStreamSynchronize(S->stream);
    for (Request *r : S->pending)
        delete r;
    for (Request *r : S->submitted)
        delete r;
    for (Request *r : S->large_q)
        delete r;
    for (auto &kv : S->mats)
        if (kv.second.h)
            spmv_destroy(kv.second.h);
    (void)hipFree(S->slots);
    (void)hipFree(S->stat);
    (void)hipFree(S->active_dev);
    (void)hipHostFree(S->stat_host);
    (void)hipHostFree(S->active_host);
    if (S->stream)
        (void)hipStreamDestroy(S->stream);
    delete S;
}

}  // extern "C"
