// Host drivers of CG and GMRES(m), plain FP64 and mixed FP32/FP64, and the
// asynchronous executor that predicts and swaps the SpMV configuration while
// the solve runs (Section III-C-2, asynchronous execution).
//
// The drivers only enqueue: every scalar of the iteration (alpha, beta, the
// Hessenberg/Givens update, convergence tests) lives on the device, and every
// iteration kernel turns into a no-op once the device state leaves RUN.  The
// host polls that state through pinned memory every few iterations, one poll
// behind, so the GPU never waits for the host inside a solve.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <thread>

#include <mutex>
#include <vector>

#include "batched.hpp"
#include "devcache.hpp"
#include "matrix.hpp"
#include "panel.hpp"
#include "predictor.hpp"
#include "solvers.hpp"

namespace ck {

ck_status compute_features(ck_matrix &M, ck_features &F, hipStream_t s, bool symmetry);
ck_status convert_format(ck_matrix &M, const ck_config &c, hipStream_t s);

namespace {

using Clock = std::chrono::steady_clock;
double us_since(Clock::time_point t0) {
    return std::chrono::duration<double, std::micro>(Clock::now() - t0).count();
}

// ---------------------------------------------------------------------------
// Device workspace owned by one solve, from the handle's memory source (the
// caller's allocator, or the handle-memory cache); it goes back once the
// solve's stream has finished with it.
struct Workspace {
    ck_matrix &M;
    hipStream_t s;
    std::vector<void *> blocks;
    Workspace(ck_matrix &m, hipStream_t st) : M(m), s(st) {}
    template <typename T>
    ck_status get(T **p, int64_t count) {
        T *q = nullptr;
        CK_TRY(mat_alloc(M, &q, std::max<int64_t>(count, 1), s));
        blocks.push_back(q);
        *p = q;
        return CK_OK;
    }
    ~Workspace() {
        if (blocks.empty())
            return;
        (void)hipStreamSynchronize(s);
        for (void *q : blocks)
            mat_free(M, q);
    }
};

// Pinned host staging for status polls (one buffer per host thread).
struct Pinned {
    char *buf = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    ck_status init() {
        if (!buf) {
            CK_HIP(hipHostMalloc((void **)&buf, 4096, hipHostMallocDefault));
            CK_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
            CK_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
        }
        return CK_OK;
    }
};
thread_local Pinned tl_pinned;

// ---------------------------------------------------------------------------
// Asynchronous executor: a worker thread runs features (GPU, side stream),
// the three-stage cascade (host) and the format conversion (GPU, side
// stream) and publishes each stage's configuration as soon as it is known.
// The solver calls poll() at every iteration boundary and adopts a published
// configuration once its conversion (if any) has completed.
//
// Overhead-aware conversion (opt-in, after the overhead-conscious selection
// the paper discusses among related work): before a decision that needs a
// new copy of the matrix is converted, the worker waits for the solver's
// residual reports of at least kGateMinIter iterations, extrapolates the
// remaining iterations R from the residual's decay over the last
// kGateWindow or more iterations and converts only if R * kGain >= C, where
// C is the conversion's cost in products of the matrix (its bytes over one
// product's bytes, plus two for launches and the host read-back) and kGain
// the fraction of a product each remaining iteration is assumed to save.
// A Krylov residual falls fastest in the first iterations (on a 3D
// Laplacian the decay over iterations 2-6 is about 3x the average), so the
// geometric extrapolation is doubled (kSlowdown).
constexpr double kGain = 0.25;
constexpr double kSlowdown = 2.0;
constexpr int kGateMinIter = 8;
constexpr int kGateWindow = 4;

}  // namespace

// Bytes a conversion to `c` moves, in products of the CSR matrix (+2).
double conversion_products(const ck_features &F, const ck_config &c) {
    const double n = (double)F.nrows, nnz = (double)F.nnz;
    const double pitch = (double)ceil_div(F.nrows, 64) * 64;
    const double product = 12.0 * nnz + 20.0 * n + 4.0;
    double b = 0;
    if (c.format == CK_FMT_ELL)
        b = 4 * n + 12 * nnz + 12 * (double)F.max_r * pitch;
    else if (c.format == CK_FMT_COO)
        b = 4 * n + 4 * nnz;
    else if (c.format == CK_FMT_DIA)   // mark, three scan levels, zero-fill + scatter
        b = 8 * nnz + 16 * (n + (double)F.ncols) * 3 + 16 * (double)F.ndiag * pitch + 12 * nnz;
    else if (c.format == CK_FMT_HYB)   // histogram, ELL part (<= 3 nnz slots), long-row list
        b = 4 * n + 12 * nnz + 36 * nnz + 16 * n;
    else if (c.algorithm == CK_ALG_PANEL)
        b = 16.0 * panel_count_for(F.ncols, 8) * n + 24 * nnz;
    return b / product + 2.0;
}

// Remaining iterations extrapolated from two residual reports (t0, r0) and
// (t1, r1), t0 < t1: kSlowdown times the iterations the decay from r0 to r1
// needs, continued geometrically, to reach tol; 1e9 when the residual has
// not decreased.
double remaining_iterations(int t0, double r0, int t1, double r1, double tol) {
    if (!(r1 > 0.0) || r1 <= tol)
        return 0.0;
    if (!(r1 < r0) || !(tol > 0.0) || t1 <= t0)
        return 1e9;
    return std::min(1e9, kSlowdown * (t1 - t0) * std::log(tol / r1) / std::log(r1 / r0));
}

namespace {

// Side streams (with their conversion events) of finished executors, kept
// per device for the next solve: creating and destroying a stream per solve
// costs as much as the feature pass of a mid-size matrix.
struct SideStreams {
    std::mutex mu;
    std::map<int, std::vector<std::pair<hipStream_t, hipEvent_t>>> idle;
};
SideStreams &side_streams() {
    static SideStreams *p = new SideStreams();   // never destroyed: outlives every solve
    return *p;
}

class AsyncExec {
  public:
    AsyncExec(ck_matrix &M, const ck_config &start, bool gate)
        : M_(M), current_(start), gate_(gate) {
        for (int t = 0; t < 3; ++t) {
            published_[t].store(-1);
            applied_[t] = false;
        }
    }
    ~AsyncExec() { finish(); }

    ck_status start() {
        {
            SideStreams &ss = side_streams();
            std::lock_guard<std::mutex> lk(ss.mu);
            auto &v = ss.idle[M_.device];
            if (!v.empty()) {
                side_ = v.back().first;
                conv_done_ = v.back().second;
                v.pop_back();
            }
        }
        if (!side_)
            CK_HIP(hipStreamCreateWithFlags(&side_, hipStreamNonBlocking));
        if (!conv_done_)
            CK_HIP(hipEventCreateWithFlags(&conv_done_, hipEventDisableTiming));
        worker_ = std::thread([this] { run(); });
        return CK_OK;
    }

    // Called by the solver between iterations; `iter` = iterations issued so far.
    void poll(int iter, ck_config &cfg, int32_t switch_iter[3]) {
        for (int t = 0; t < 3; ++t) {
            if (applied_[t])
                continue;
            const int code = published_[t].load(std::memory_order_acquire);
            if (code < 0)
                return;                      // later stages come after this one
            if (code == kNoStage) {          // stage not run (cascade ended earlier)
                applied_[t] = true;
                continue;
            }
            if (conv_needed_[t].load(std::memory_order_acquire)) {
                const hipError_t e = hipEventQuery(conv_done_);
                if (e == hipErrorNotReady)
                    return;
                (void)hipGetLastError();
            }
            ck_config next = decoded_[t];
            cfg = next;
            switch_iter[t] = iter;
            applied_[t] = true;
        }
    }

    // true while a stage decision has not been applied yet
    bool pending() const { return !(applied_[0] && applied_[1] && applied_[2]); }

    // The solver's residual reports (iterations done, relative residual, its
    // tolerance), for the overhead-aware gate.
    void progress(int iter, double relres, double tol) {
        if (!gate_ || iter <= 0 || !(relres > 0.0))
            return;
        std::lock_guard<std::mutex> lk(prog_mu_);
        if (!hist_.empty() && iter <= hist_.back().first)
            return;
        if (hist_.size() >= 256)          // only recent reports matter
            hist_.erase(hist_.begin(), hist_.begin() + 128);
        hist_.emplace_back(iter, relres);
        tol_ = tol;
    }

    void finish() {
        cancel_.store(true);
        if (worker_.joinable())
            worker_.join();
        if (side_ && conv_done_ && hipStreamSynchronize(side_) == hipSuccess) {
            SideStreams &ss = side_streams();
            std::lock_guard<std::mutex> lk(ss.mu);
            ss.idle[M_.device].emplace_back(side_, conv_done_);
        } else {
            if (side_)
                (void)hipStreamDestroy(side_);
            if (conv_done_)
                (void)hipEventDestroy(conv_done_);
        }
        side_ = nullptr;
        conv_done_ = nullptr;
    }

    double t_features = 0, t_infer = 0, t_convert = 0;
    int conversion_failed = 0;
    int gate_decision = -1;      // -1 not asked, 0 converted, 1 skipped
    int est_remaining = -1;      // the gate's estimate of the remaining iterations

  private:
    static constexpr int kNoStage = 1000;

    void publish(int t, const ck_config &c) {
        decoded_[t] = c;
        published_[t].store(ck_config_id(&c) >= 0 ? ck_config_id(&c) : 0,
                            std::memory_order_release);
    }
    void skip_rest(int from) {
        for (int t = from; t < 3; ++t)
            published_[t].store(kNoStage, std::memory_order_release);
    }

    // Overhead-aware gate: true = convert.  Waits (until cancelled) for a
    // residual report at least kGateMinIter iterations after the first.
    bool worth_converting(const ck_features &F, const ck_config &c) {
        if (!gate_)
            return true;
        const double C = conversion_products(F, c);
        while (!cancel_.load()) {
            int t = -1, t_ref = 0;
            double r1 = 0, r_ref = 1.0, tol = 0;   // x0 = 0: relres 1 at iteration 0
            {
                std::lock_guard<std::mutex> lk(prog_mu_);
                if (!hist_.empty()) {
                    t = hist_.back().first;
                    r1 = hist_.back().second;
                    for (const auto &h : hist_)   // latest report >= kGateWindow back
                        if (h.first <= t - kGateWindow) {
                            t_ref = h.first;
                            r_ref = h.second;
                        }
                }
                tol = tol_;
            }
            if (t >= kGateMinIter) {
                const double R = remaining_iterations(t_ref, r_ref, t, r1, tol);
                est_remaining = (int)R;
                const bool go = R * kGain >= C;
                gate_decision = go ? 0 : 1;
                return go;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        return false;
    }

    void run() {
        (void)hipSetDevice(M_.device);
        auto t0 = Clock::now();
        ck_features F;
        if (compute_features(M_, F, side_, false) != CK_OK || cancel_.load()) {
            skip_rest(0);
            return;
        }
        t_features = us_since(t0);
        std::string err;
        const Cascade *C = load_cascade(nullptr, err);
        if (!C) {
            skip_rest(0);
            return;
        }
        double in[kNumModelFeatures];
        model_inputs(F, in);
        auto t1 = Clock::now();
        const int fmt = C->tree[0].eval(in);
        t_infer += us_since(t1);
        ck_config c = stage_config(0, fmt, current_);
        if (fmt != CK_FMT_CSR) {
            if (cancel_.load() || !worth_converting(F, c)) {
                skip_rest(0);
                return;
            }
            auto t2 = Clock::now();
            if (convert_format(M_, c, side_) != CK_OK) {
                // conversion refused or out of memory: keep the current kernel
                conversion_failed = 1;
                skip_rest(0);
                return;
            }
            (void)hipEventRecord(conv_done_, side_);
            conv_needed_[0].store(true, std::memory_order_release);
            publish(0, c);
            skip_rest(1);
            (void)hipEventSynchronize(conv_done_);
            t_convert = us_since(t2);
            return;
        }
        publish(0, c);
        if (cancel_.load()) {
            skip_rest(1);
            return;
        }
        t1 = Clock::now();
        const int alg = C->tree[1].eval(in);
        t_infer += us_since(t1);
        c = stage_config(1, alg, c);
        if (alg == CK_ALG_VECTOR && c.lanes <= 0)   // started on a non-vector kernel
            c.lanes = default_config(M_.n, M_.nnz).lanes;
        if (alg == CK_ALG_PANEL || alg == CK_ALG_MERGE) {
            // the panel-major copy / merge-path partition must exist first
            // (the partition costs a fraction of a product: never gated)
            if (cancel_.load() || (alg == CK_ALG_PANEL && !worth_converting(F, c))) {
                skip_rest(1);
                return;
            }
            auto t2 = Clock::now();
            if (convert_format(M_, c, side_) != CK_OK) {
                conversion_failed = 1;
                skip_rest(1);
                return;
            }
            (void)hipEventRecord(conv_done_, side_);
            conv_needed_[1].store(true, std::memory_order_release);
            publish(1, c);
            skip_rest(2);
            (void)hipEventSynchronize(conv_done_);
            t_convert = us_since(t2);
            return;
        }
        publish(1, c);
        if (alg != CK_ALG_VECTOR) {
            skip_rest(2);
            return;
        }
        t1 = Clock::now();
        const int lg = C->tree[2].eval(in);
        t_infer += us_since(t1);
        c = stage_config(2, lg, c);
        publish(2, c);
    }

    ck_matrix &M_;
    ck_config current_;
    bool gate_ = false;
    std::mutex prog_mu_;
    std::vector<std::pair<int, double>> hist_;   // (iterations, relres) reports
    double tol_ = 0;
    hipStream_t side_ = nullptr;
    hipEvent_t conv_done_ = nullptr;
    std::thread worker_;
    std::atomic<bool> cancel_{false};
    std::atomic<bool> conv_needed_[3] = {false, false, false};   // stage waits for conv_done_
    std::atomic<int> published_[3];
    ck_config decoded_[3];
    bool applied_[3];
};

// ---------------------------------------------------------------------------
struct SolveCtx {
    ck_matrix &M;
    const ck_solve_opts &o;
    ck_solve_result &res;
    hipStream_t s;
    ck_config cfg;
    AsyncExec *exec = nullptr;
    void *carry = nullptr;       // merge-path / COO workspace
    void poll(int iter) {
        if (exec)
            exec->poll(iter, cfg, res.switch_iter);
    }
};

template <typename T>
ck_status spmv(SolveCtx &c, T alpha, const T *x, T beta, T *y, const int *skip,
               CgDev<T> *cg = nullptr, T *partials = nullptr) {
    SpmvArgs<T> a;
    a.alpha = alpha;
    a.beta = beta;
    a.x = x;
    a.y = y;
    a.skip = skip;
    a.cg = cg;
    a.dot_partials = partials;
    a.carry = c.carry;
    return launch_spmv<T>(c.M, c.cfg, a, c.s);
}

// ||v|| in FP64, blocking (used once per solve / refinement step)
ck_status norm_host(SolveCtx &c, const double *v, double *partials, double *dout, double &out) {
    CK_TRY(launch_dot(c.M.n, v, v, partials, dout, c.s));
    double h = 0;
    CK_HIP(hipMemcpyAsync(&h, dout, sizeof h, hipMemcpyDeviceToHost, c.s));
    CK_HIP(hipStreamSynchronize(c.s));
    out = std::sqrt(h);
    return CK_OK;
}

struct Fp64Scratch {
    double *partials = nullptr, *dout = nullptr;
    ck_status init(Workspace &ws, hipStream_t) {
        CK_TRY(ws.get(&partials, kMaxPartials));
        CK_TRY(ws.get(&dout, 4));
        return CK_OK;
    }
};

// true ||b - A x|| / bnorm with the FP64 values
ck_status true_relres(SolveCtx &c, const double *b, const double *x, double *r, Fp64Scratch &f,
                      double bnorm, double &out) {
    CK_TRY(launch_copy<double, double>(c.M.n, r, b, nullptr, c.s));
    CK_TRY(spmv<double>(c, -1.0, x, 1.0, r, nullptr));
    double nr = 0;
    CK_TRY(norm_host(c, r, f.partials, f.dout, nr));
    out = bnorm > 0 ? nr / bnorm : nr;
    return CK_OK;
}

// ---------------------------------------------------------------------------
// One CG run in precision T on A (FP64 or FP32 values) from the residual
// already in r (x is updated in place).  Returns the final device state.
template <typename T>
ck_status cg_core(SolveCtx &c, T *x, T *r, T *p, T *q, T *partials, CgDev<T> *dev,
                  double bnorm, double tol, int &iter_total, int max_iter, int &state_out) {
    Pinned &pin = tl_pinned;
    CK_TRY(pin.init());
    CgDev<T> h{};
    h.bnorm = bnorm;
    h.tol = tol;
    h.state = RUN;
    h.iter = iter_total;
    h.max_iter = max_iter;
    std::memcpy(pin.buf + 2048, &h, sizeof h);
    CK_HIP(hipMemcpyAsync(dev, pin.buf + 2048, sizeof h, hipMemcpyHostToDevice, c.s));
    CK_TRY(launch_cg_start<T>(c.M.n, r, p, partials, dev, c.s));
    const int every = std::max(1, c.o.check_every > 0 ? c.o.check_every : 8);
    const int *state_ptr = &dev->state;
    int slot = 0, polls = 0, since_poll = 0;
    int issued = 0;
    const int budget = max_iter - iter_total;
    while (true) {
        // the host runs up to two polls ahead of the device; while a cascade
        // decision may still arrive, poll every other iteration so that a
        // decision reaches the device within a few iterations
        const int every_now = (c.exec && c.exec->pending()) ? std::min(every, 2) : every;
        c.poll(iter_total + issued);
        const bool fused = spmv_fuses_dot(c.cfg);
        if (fused) {
            CK_TRY(spmv<T>(c, T(1), p, T(0), q, state_ptr, dev, partials));
            CK_TRY(launch_cg_sigma_finish<T>(spmv_dot_blocks(c.M, c.cfg), partials, dev, c.s));
        } else {
            CK_TRY(spmv<T>(c, T(1), p, T(0), q, state_ptr));
            CK_TRY(launch_cg_sigma<T>(c.M.n, p, q, partials, dev, c.s));
        }
        CK_TRY(launch_cg_update<T>(c.M.n, x, r, p, q, partials, dev, c.s));
        ++issued;
        if (++since_poll >= every_now || issued >= budget) {
            since_poll = 0;
            // stage this poll (relres, state, iter: adjacent fields), then
            // read the previous one
            CK_HIP(hipMemcpyAsync(pin.buf + 64 * slot, &dev->relres, sizeof(double) + 2 * sizeof(int),
                                  hipMemcpyDeviceToHost, c.s));
            CK_HIP(hipEventRecord(pin.ev[slot], c.s));
            ++polls;
            if (polls >= 2 || issued >= budget) {
                const int prev = (issued >= budget) ? slot : slot ^ 1;
                CK_HIP(hipEventSynchronize(pin.ev[prev]));
                double rr;
                int st, it;
                std::memcpy(&rr, pin.buf + 64 * prev, sizeof rr);
                std::memcpy(&st, pin.buf + 64 * prev + sizeof(double), sizeof st);
                std::memcpy(&it, pin.buf + 64 * prev + sizeof(double) + sizeof(int), sizeof it);
                if (c.exec)
                    c.exec->progress(it, rr, tol);
                if (st != RUN)
                    break;
            }
            slot ^= 1;
            if (issued >= budget + 2 * every)
                break;   // device budget check has certainly fired
        }
    }
    CK_HIP(hipMemcpyAsync(pin.buf + 2048, dev, sizeof h, hipMemcpyDeviceToHost, c.s));
    CK_HIP(hipStreamSynchronize(c.s));
    std::memcpy(&h, pin.buf + 2048, sizeof h);
    iter_total = h.iter;
    state_out = h.state;
    return CK_OK;
}

ck_status cg_fp64(SolveCtx &c, const double *b, double *x) {
    ck_matrix &M = c.M;
    Workspace ws(c.M, c.s);
    double *r, *p, *q, *partials;
    CgDev<double> *dev;
    Fp64Scratch f;
    CK_TRY(ws.get(&r, M.n));
    CK_TRY(ws.get(&p, M.n));
    CK_TRY(ws.get(&q, M.n));
    CK_TRY(ws.get(&partials, kMaxPartials));
    CK_TRY(ws.get(&dev, 1));
    CK_TRY(f.init(ws, c.s));
    double bnorm = 0;
    CK_TRY(norm_host(c, b, f.partials, f.dout, bnorm));
    if (bnorm == 0.0) {
        CK_TRY(launch_fill<double>(M.n, x, 0.0, c.s));
        c.res.true_relres = 0;
        return CK_OK;
    }
    const int max_iter = c.o.max_iter > 0 ? c.o.max_iter : 100000;
    int iters = 0, state = RUN;
    ck_status out = CK_E_NOT_CONVERGED;
    for (int restart = 0; restart <= 3; ++restart) {
        CK_TRY(launch_copy<double, double>(M.n, r, b, nullptr, c.s));     // r = b - A x
        CK_TRY(spmv<double>(c, -1.0, x, 1.0, r, nullptr));
        CK_TRY(cg_core<double>(c, x, r, p, q, partials, dev, bnorm, c.o.tol, iters, max_iter,
                               state));
        c.res.outer_steps = restart + 1;
        if (state == BREAKDOWN) {
            out = CK_E_BREAKDOWN;
            break;
        }
        double tr = 0;
        CK_TRY(true_relres(c, b, x, r, f, bnorm, tr));
        c.res.true_relres = tr;
        if (tr <= c.o.tol) {
            out = CK_OK;
            break;
        }
        if (state == BUDGET)
            break;
    }
    c.res.iterations = iters;
    return out;
}

// Mixed precision CG: FP64 refinement steps r = b - A64 x, d = CG32(A32, r/||r||),
// x += ||r|| d.  The inner solve stops at relative residual max(tol*||b||/||r||, 1e-5)
// or after max(50, 4 sqrt(n)) iterations.
ck_status cg_mixed(SolveCtx &c, const double *b, double *x) {
    ck_matrix &M = c.M;
    Workspace ws(c.M, c.s);
    double *r64, *scal;
    float *r, *p, *q, *d, *partials;
    CgDev<float> *dev;
    Fp64Scratch f;
    CK_TRY(ws.get(&r64, M.n));
    CK_TRY(ws.get(&scal, 4));
    CK_TRY(ws.get(&r, M.n));
    CK_TRY(ws.get(&p, M.n));
    CK_TRY(ws.get(&q, M.n));
    CK_TRY(ws.get(&d, M.n));
    CK_TRY(ws.get(&partials, kMaxPartials));
    CK_TRY(ws.get(&dev, 1));
    CK_TRY(f.init(ws, c.s));
    double bnorm = 0;
    CK_TRY(norm_host(c, b, f.partials, f.dout, bnorm));
    if (bnorm == 0.0) {
        CK_TRY(launch_fill<double>(M.n, x, 0.0, c.s));
        c.res.true_relres = 0;
        return CK_OK;
    }
    const int max_iter = c.o.max_iter > 0 ? c.o.max_iter : 100000;
    const int inner_cap = std::max(50, (int)(4.0 * std::sqrt((double)M.n)));
    int iters = 0;
    ck_status out = CK_E_NOT_CONVERGED;
    Pinned &pin = tl_pinned;
    CK_TRY(pin.init());
    for (int step = 0; step < 60; ++step) {
        double tr = 0;
        CK_TRY(true_relres(c, b, x, r64, f, bnorm, tr));          // r64 = b - A x
        c.res.true_relres = tr;
        c.res.outer_steps = step;
        if (tr <= c.o.tol) {
            out = CK_OK;
            break;
        }
        if (iters >= max_iter)
            break;
        const double beta = tr * bnorm;
        double hs[2] = {1.0 / beta, beta};
        std::memcpy(pin.buf + 3072, hs, sizeof hs);
        CK_HIP(hipMemcpyAsync(scal, pin.buf + 3072, sizeof hs, hipMemcpyHostToDevice, c.s));
        CK_TRY(launch_scale_cast<float>(M.n, r, r64, scal, nullptr, c.s));   // r32 = r/beta
        CK_TRY(launch_fill<float>(M.n, d, 0.0f, c.s));
        const double inner_tol = std::max(c.o.tol * bnorm / beta, 1e-5);
        int inner_iters = 0, state = RUN;
        const int cap = std::min(inner_cap, max_iter - iters);
        CK_TRY(cg_core<float>(c, d, r, p, q, partials, dev, 1.0, inner_tol, inner_iters, cap,
                              state));
        iters += inner_iters;
        if (state == BREAKDOWN && inner_iters == 0) {
            out = CK_E_BREAKDOWN;
            break;
        }
        CK_TRY(launch_axpy_promote<float>(M.n, x, d, scal + 1, nullptr, c.s));   // x += beta d
    }
    c.res.iterations = iters;
    return out;
}

// ---------------------------------------------------------------------------
// GMRES(m) in precision T (T = float: mixed precision; each cycle is one
// refinement step, since it starts from the FP64 true residual and adds its
// correction to the FP64 x).
template <typename T>
ck_status gmres_run(SolveCtx &c, const double *b, double *x) {
    ck_matrix &M = c.M;
    const int m = c.o.restart > 0 ? c.o.restart : 30;
    if (m > kMaxRestart)
        return fail(CK_E_INVALID, "restart length %d above %d", m, kMaxRestart);
    Workspace ws(c.M, c.s);
    const int64_t ldv = ceil_div(std::max<int64_t>(M.n, 1), 64) * 64;
    T *V, *partials;
    double *r64;
    GmDev<T> *st;
    Fp64Scratch f;
    CK_TRY(ws.get(&V, ldv * (m + 1)));
    CK_TRY(ws.get(&partials, (int64_t)(kMaxRestart + 1) * kGmMaxBlocks));
    CK_TRY(ws.get(&r64, M.n));
    CK_TRY(ws.get(&st, 1));
    CK_TRY(f.init(ws, c.s));
    double bnorm = 0;
    CK_TRY(norm_host(c, b, f.partials, f.dout, bnorm));
    if (bnorm == 0.0) {
        CK_TRY(launch_fill<double>(M.n, x, 0.0, c.s));
        c.res.true_relres = 0;
        return CK_OK;
    }
    Pinned &pin = tl_pinned;
    CK_TRY(pin.init());
    GmDev<T> *h = (GmDev<T> *)std::malloc(sizeof(GmDev<T>));
    std::memset(h, 0, sizeof(GmDev<T>));
    h->m = m;
    h->bnorm = bnorm;
    h->tol = c.o.tol;
    h->max_iter = c.o.max_iter > 0 ? c.o.max_iter : 100000;
    h->final_state = RUN;
    h->halt = 1;
    CK_HIP(hipMemcpyAsync(st, h, sizeof(GmDev<T>), hipMemcpyHostToDevice, c.s));
    CK_HIP(hipStreamSynchronize(c.s));
    const int *final_ptr = &st->final_state;
    const int *halt_ptr = &st->halt;
    // relres, m, j, iter, max_iter, cycle_stop, final_state (adjacent fields)
    const int status_off = (int)offsetof(GmDev<T>, relres);
    int issued = 0, slot = 0, cycles = 0;
    ck_status out = CK_OK;
    while (true) {
        // true residual r = b - A x in FP64, then beta, test, v0 = r / beta
        CK_TRY(launch_copy<double, double>(M.n, r64, b, final_ptr, c.s));
        CK_TRY(spmv<double>(c, -1.0, x, 1.0, r64, final_ptr));
        CK_TRY(launch_gm_cycle_start<T>(M.n, r64, V, f.partials, st, c.s));
        for (int j = 0; j < m; ++j) {
            c.poll(issued);
            CK_TRY(spmv<T>(c, T(1), V + (int64_t)j * ldv, T(0), V + (int64_t)(j + 1) * ldv,
                           halt_ptr));
            CK_TRY(launch_gm_arnoldi<T>(M.n, j, V, ldv, partials, st, c.s));
            ++issued;
        }
        CK_TRY(launch_gm_cycle_end<T>(M.n, x, V, ldv, st, c.s));
        ++cycles;
        CK_HIP(hipMemcpyAsync(pin.buf + 64 * slot, (char *)st + status_off,
                              sizeof(double) + 6 * sizeof(int), hipMemcpyDeviceToHost, c.s));
        CK_HIP(hipEventRecord(pin.ev[slot], c.s));
        if (cycles >= 2) {
            const int prev = slot ^ 1;
            CK_HIP(hipEventSynchronize(pin.ev[prev]));
            double rr;
            int it, fs;
            std::memcpy(&rr, pin.buf + 64 * prev, sizeof rr);
            std::memcpy(&it, pin.buf + 64 * prev + sizeof(double) + 2 * sizeof(int), sizeof it);
            std::memcpy(&fs, pin.buf + 64 * prev + sizeof(double) + 5 * sizeof(int), sizeof fs);
            if (c.exec && sizeof(T) == 8)
                c.exec->progress(it, rr, c.o.tol);
            if (fs != RUN)
                break;
        }
        slot ^= 1;
        // a cycle that ends on the budget is followed by at most one more start
        if (issued > h->max_iter + 2 * m)
            break;
    }
    CK_HIP(hipMemcpyAsync(h, st, sizeof(GmDev<T>), hipMemcpyDeviceToHost, c.s));
    CK_HIP(hipStreamSynchronize(c.s));
    c.res.iterations = h->iter;
    c.res.outer_steps = h->cycles;
    if (h->final_state == CONVERGED)
        out = CK_OK;
    else if (h->final_state == BREAKDOWN)
        out = CK_E_BREAKDOWN;
    else
        out = CK_E_NOT_CONVERGED;
    std::free(h);
    double tr = 0;
    CK_TRY(true_relres(c, b, x, r64, f, bnorm, tr));
    c.res.true_relres = tr;
    return out;
}

enum class Solver { CG, GMRES };

// Systems up to this size run the whole solve inside one 1024-thread
// workgroup (the batched slot kernel): at this size a launch per step costs
// more than the step itself.
constexpr int64_t kSmallN = 16384;

// FP64 CG of a system of at most kWgCgMaxN rows in one single-workgroup launch
ck_status wg_cg_solve(SolveCtx &c, const double *b, double *x) {
    Workspace ws(c.M, c.s);
    WgCgOut *out;
    int *ccol;
    double *cval;
    CK_TRY(ws.get(&out, 1));
    CK_TRY(ws.get(&ccol, (int64_t)kWgCgColMajorK * kWgCgMaxN));
    CK_TRY(ws.get(&cval, (int64_t)kWgCgColMajorK * kWgCgMaxN));
    const int max_iter = c.o.max_iter > 0 ? c.o.max_iter : 100000;
    CK_TRY(launch_cg_wg((int)c.M.n, c.M.rp, c.M.col, c.M.val, b, x, c.o.tol, max_iter, ccol, cval,
                        out, c.s));
    WgCgOut h{};
    CK_HIP(hipMemcpyAsync(&h, out, sizeof h, hipMemcpyDeviceToHost, c.s));
    CK_HIP(hipStreamSynchronize(c.s));
    c.res.iterations = h.iter;
    c.res.outer_steps = h.restarts + 1;
    c.res.true_relres = h.relres;
    if (h.status == CONVERGED)
        return CK_OK;
    if (h.status == BREAKDOWN)
        return fail(CK_E_BREAKDOWN, "breakdown (p.Ap <= 0)");
    return fail(CK_E_NOT_CONVERGED, "iteration budget spent at relative residual %.3e",
                h.relres);
}

ck_status small_solve(SolveCtx &c, const double *b, double *x, bool cg, int m) {
    ck_matrix &M = c.M;
    const bool fp32 = c.o.precision == CK_PREC_MIXED;
    const int kind = cg ? B_CG : B_GMRES;
    const int64_t ld = ceil_div(M.n, 64) * 64;
    Workspace ws(c.M, c.s);
    BSlot *slot;
    BStat *stat;
    int *active;
    char *work;
    double *r64;
    CK_TRY(ws.get(&slot, 1));
    CK_TRY(ws.get(&stat, 1));
    CK_TRY(ws.get(&active, 1));
    CK_TRY(ws.get(&work, bslot_work_elems(kind, M.n, m) * (fp32 ? 4 : 8)));
    CK_TRY(ws.get(&r64, ld));
    BSlot *h = (BSlot *)std::calloc(1, sizeof(BSlot));
    h->kind = kind;
    h->n = (int)M.n;
    h->lanes = c.cfg.lanes;
    h->m = m;
    h->rp = M.rp;
    h->col = M.col;
    h->val64 = M.val;
    h->val32 = M.val32;
    h->b = b;
    h->x = x;
    h->r64 = r64;
    h->work = work;
    h->ld = ld;
    h->bnorm = -1.0;
    h->tol = c.o.tol;
    h->max_iter = c.o.max_iter > 0 ? c.o.max_iter : 100000;
    h->inner_cap = fp32 ? std::max(50, (int)(4.0 * std::sqrt((double)M.n))) : h->max_iter;
    h->keep_x0 = 1;
    h->phase = B_OUTER;
    h->status = RUN;
    const int budget = 3 * h->max_iter + 64;
    BStat hs{};
    hipError_t e = hipMemcpyAsync(slot, h, sizeof(BSlot), hipMemcpyHostToDevice, c.s);
    std::free(h);
    CK_HIP(e);
    CK_TRY(launch_fill<int>(1, active, 0, c.s));
    CK_TRY(launch_batched_chunk(slot, stat, active, 1, budget, fp32, c.s, true));
    CK_HIP(hipMemcpyAsync(&hs, stat, sizeof hs, hipMemcpyDeviceToHost, c.s));
    CK_HIP(hipStreamSynchronize(c.s));
    c.res.iterations = hs.iter;
    c.res.outer_steps = hs.outer;
    c.res.true_relres = hs.relres;
    if (hs.status == CONVERGED)
        return CK_OK;
    if (hs.status == BREAKDOWN)
        return fail(CK_E_BREAKDOWN, "breakdown (p.Ap <= 0 or a singular least-squares system)");
    return fail(CK_E_NOT_CONVERGED, "iteration budget spent at relative residual %.3e",
                hs.relres);
}

// Sequential execution (the form the asynchronous executor is measured
// against, Section IV): features, the three cascade stages and the format
// conversion all finish before the first iteration, which then runs on the
// prediction.  A refused or failed conversion keeps the default
// configuration (its stages stay unapplied, switch_iter -1).
ck_status sequential_predict(SolveCtx &c) {
    auto t0 = Clock::now();
    ck_features F;
    CK_TRY(compute_features(c.M, F, c.s, false));
    c.res.t_features_us = us_since(t0);
    std::string err;
    const Cascade *C = load_cascade(nullptr, err);
    if (!C)
        return fail(CK_E_INVALID, "%s", err.c_str());
    double in[kNumModelFeatures];
    model_inputs(F, in);
    auto t1 = Clock::now();
    ck_config cfg = c.cfg;
    int stages = 0;
    for (int t = 0; t < 3; ++t) {
        const int cls = C->tree[t].eval(in);
        cfg = stage_config(t, cls, cfg);
        stages = t + 1;
        if ((t == 0 && cls != CK_FMT_CSR) || (t == 1 && cls != CK_ALG_VECTOR))
            break;
    }
    c.res.t_infer_us = us_since(t1);
    auto t2 = Clock::now();
    if (convert_format(c.M, cfg, c.s) == CK_OK) {
        CK_HIP(hipStreamSynchronize(c.s));
        c.cfg = cfg;
        for (int t = 0; t < stages; ++t)
            c.res.switch_iter[t] = 0;
    }
    c.res.t_convert_us = us_since(t2);
    return CK_OK;
}

ck_status solve(ck_handle hnd, const double *b, double *x, const ck_solve_opts *opts,
                ck_solve_result *res, hipStream_t s, Solver which) {
    if (!hnd || !opts || !res || (hnd->n > 0 && (!b || !x)))
        return fail(CK_E_INVALID, "NULL argument");
    ck_matrix &M = *hnd;
    if (M.n != M.ncols)
        return fail(CK_E_INVALID, "the matrix must be square");
    if (!(opts->tol >= 0.0))
        return fail(CK_E_INVALID, "tol must be >= 0");
    if (opts->precision == CK_PREC_MIXED && !M.val32)
        return fail(CK_E_INVALID, "mixed precision needs a handle created with CK_KEEP_FP32");
    if (opts->async < CK_EXEC_DEFAULT || opts->async > CK_EXEC_SEQUENTIAL)
        return fail(CK_E_INVALID, "async must be CK_EXEC_DEFAULT, _ASYNC or _SEQUENTIAL");
    std::memset(res, 0, sizeof *res);
    res->conversion_gated = -1;
    res->est_remaining_iters = -1;
    res->switch_iter[0] = res->switch_iter[1] = res->switch_iter[2] = -1;
    const auto t0 = Clock::now();
    SolveCtx c{M, *opts, *res, s, default_config(M.n, M.nnz)};
    if (opts->use_config) {
        if (!config_valid(opts->config))
            return fail(CK_E_INVALID, "invalid configuration in opts");
        CK_TRY(convert_format(M, opts->config, s));
        c.cfg = opts->config;
    } else if (opts->known_start && opts->async != CK_EXEC_SEQUENTIAL) {
        // the start tree's choice among the configurations that need no copy
        std::string err;
        const Cascade *C = load_cascade(nullptr, err);
        const int id = C && M.n > 0 ? start_config_id(*C, M.n, M.ncols, M.nnz) : -1;
        ck_config sc;
        if (id >= 0 && ck_config_from_id(id, &sc) == CK_OK)
            c.cfg = sc;
    }
    if (M.n == 0) {
        res->status = CK_OK;
        res->final_config = c.cfg;
        return CK_OK;
    }
    const bool run_async = opts->async == CK_EXEC_ASYNC && !opts->use_config;
    if (opts->async == CK_EXEC_SEQUENTIAL && !opts->use_config)
        CK_TRY(sequential_predict(c));
    const int m = opts->restart > 0 ? opts->restart : 30;
    if (M.n <= kWgCgMaxN && which == Solver::CG && opts->precision == CK_PREC_FP64 &&
        opts->async == CK_EXEC_DEFAULT && !opts->use_config) {
        // the whole solve in one single-workgroup launch; its product takes
        // one lane per row
        const ck_status st = wg_cg_solve(c, b, x);
        res->final_config = ck_config{CK_FMT_CSR, CK_ALG_VECTOR, 1, 0};
        res->status = st;
        res->t_total_us = us_since(t0);
        return st;
    }
    const bool vector_cfg = c.cfg.format == CK_FMT_CSR && c.cfg.algorithm == CK_ALG_VECTOR;
    if (M.n <= kSmallN && !run_async && vector_cfg && (which == Solver::CG || m <= kBMaxM)) {
        const ck_status st = small_solve(c, b, x, which == Solver::CG, m);
        res->final_config = c.cfg;
        res->status = st;
        res->t_total_us = us_since(t0);
        return st;
    }
    Workspace ws(M, s);
    int64_t carry = std::max(spmv_carry_bytes(M, ck_config{CK_FMT_CSR, CK_ALG_MERGE, 0, 0}, false),
                             std::max(spmv_carry_bytes(M, ck_config{CK_FMT_COO, 0, 0, 0}, false),
                                      spmv_carry_bytes(M, ck_config{CK_FMT_CSR, CK_ALG_PANEL, 0, 0},
                                                       false)));
    char *cbuf = nullptr;
    CK_TRY(ws.get(&cbuf, carry));
    c.carry = cbuf;
    AsyncExec *exec = nullptr;
    if (run_async) {
        exec = new AsyncExec(M, c.cfg, opts->overhead_aware != 0 &&
                                           opts->precision == CK_PREC_FP64);
        ck_status e = exec->start();
        if (e != CK_OK) {
            delete exec;
            return e;
        }
        c.exec = exec;
    }
    ck_status st;
    if (which == Solver::CG)
        st = opts->precision == CK_PREC_MIXED ? cg_mixed(c, b, x) : cg_fp64(c, b, x);
    else
        st = opts->precision == CK_PREC_MIXED ? gmres_run<float>(c, b, x)
                                              : gmres_run<double>(c, b, x);
    if (exec) {
        exec->finish();
        res->t_features_us = exec->t_features;
        res->t_infer_us = exec->t_infer;
        res->t_convert_us = exec->t_convert;
        res->conversion_gated = exec->gate_decision;
        res->est_remaining_iters = exec->est_remaining;
        delete exec;
    }
    (void)hipStreamSynchronize(s);
    res->final_config = c.cfg;
    res->status = st;
    res->t_total_us = us_since(t0);
    return st;
}

}  // namespace
}  // namespace ck

extern "C" {

ck_status ck_overhead_gate(const ck_features *f, const ck_config *target, int32_t t0, double r0,
                           int32_t t1, double r1, double tol, double *remaining, double *cost,
                           int32_t *convert) {
    if (!f || !target || !remaining || !cost || !convert || !ck::config_valid(*target))
        return ck::fail(CK_E_INVALID, "bad arguments");
    *remaining = ck::remaining_iterations(t0, r0, t1, r1, tol);
    *cost = ck::conversion_products(*f, *target);
    *convert = *remaining * ck::kGain >= *cost ? 1 : 0;
    return CK_OK;
}

ck_status cg_solve(ck_handle h, const double *d_b, double *d_x, const ck_solve_opts *opts,
                   ck_solve_result *res, hipStream_t s) {
    return ck::solve(h, d_b, d_x, opts, res, s, ck::Solver::CG);
}

ck_status gmres_solve(ck_handle h, const double *d_b, double *d_x, const ck_solve_opts *opts,
                      ck_solve_result *res, hipStream_t s) {
    return ck::solve(h, d_b, d_x, opts, res, s, ck::Solver::GMRES);
}

}  // extern "C"
