// Batched small-system solver for the request loop: one workgroup per system
// ("slot"), a bounded number of iterations per launch.  Between launches the
// host retires finished slots and admits new requests, so requests that
// arrive while others run join the next launch (continuous batching).
//
// Each slot runs FP64 iterative refinement around an FP32 inner solve:
//   outer : r = b - A x (FP64 values, FP64 arithmetic), beta = ||r||, test
//           beta/||b|| <= tol; otherwise the inner system A d = r/beta
//   inner : CG (symmetric) until ||r_in|| <= max(tol ||b||/beta, 1e-5), or
//           one GMRES(m) cycle (classical Gram-Schmidt twice, Givens), on
//           the FP32 values with FP32 vectors and FP32 accumulation
//   update: x += beta * d  (FP64)
// With FP64 inner vectors the same loop is plain CG (inner target
// tol ||b||/beta, then the true-residual check) or plain restarted GMRES(m);
// the solvers use it, with 1024 threads, for systems too small to fill the
// GPU, where one workgroup running the whole solve beats a launch per step.
// Every reduction stays inside the workgroup in a fixed order, so a slot's
// bits do not depend on which other slots share the launch.
#include <algorithm>

#include "batched.hpp"

namespace {

// sum over the workgroup of BS threads, returned to every thread (fixed order)
template <int BS, typename T>
__device__ __forceinline__ T wg_sum(T v, T *lds) {
    v = ck::wave_sum_last(v);   // valid in lane 63
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63)
        lds[w] = v;
    __syncthreads();
    T r = (lds[0] + lds[1]) + (lds[2] + lds[3]);
#pragma unroll
    for (int t = 4; t < BS / 64; t += 4)
        r += (lds[t] + lds[t + 1]) + (lds[t + 2] + lds[t + 3]);
    __syncthreads();
    return r;
}

// A small system's matrix and vectors sit in L2, so its products and vector
// sweeps are bound by load latency, not bandwidth.  Every loop below issues
// its loads unconditionally (indices clamped into range) and applies the
// bounds test only to the arithmetic and the stores; a scheduling barrier
// after each group of loads stops the compiler from sinking a load next to
// its use (which it does to save registers), so the group is in flight
// together.  The summation order is the plain one.
constexpr int kVec = 4;   // vector elements in flight per thread

// rows in flight per thread in the workgroup SpMV
template <int BS>
constexpr int rows_in_flight() { return BS >= 1024 ? 8 : 4; }

// Sum over the L lanes of a row (L a run-time power of two, uniform over
// the workgroup) by DPP moves, valid in lane L - 1 of each row's lanes.
template <typename T>
__device__ __forceinline__ T lanes_sum(T a, int L) {
    switch (L) {
    case 1: return a;
    case 2: return ck::group_sum_last<2>(a);
    case 4: return ck::group_sum_last<4>(a);
    case 8: return ck::group_sum_last<8>(a);
    case 16: return ck::group_sum_last<16>(a);
    case 32: return ck::group_sum_last<32>(a);
    default: return ck::group_sum_last<64>(a);
    }
}

// y[i] = s1 * (A x)[i] + s0 * z[i] with L lanes per row (runtime power of
// two).  Per row the lanes sum entries start + lane, start + lane + L, ...
// in order, then a DPP sum over the L lanes.
template <int BS, typename TV, typename TX, typename TA>
__device__ void wg_spmv(int n, int L, const int *__restrict__ rp, const int *__restrict__ col,
                        const TV *__restrict__ val, const TX *__restrict__ x, TA s1, TA s0,
                        const TA *__restrict__ z, TA *__restrict__ y) {
    constexpr int U = rows_in_flight<BS>();
    const int lane = threadIdx.x & (L - 1);
    const int rpp = BS / L;
    for (int r0 = 0; r0 < n; r0 += U * rpp) {
        int kb[U], ke[U];
        TA acc[U];
        int trips = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int row = min(r0 + u * rpp + (int)threadIdx.x / L, n - 1);
            kb[u] = rp[row] + lane;
            ke[u] = r0 + u * rpp + (int)threadIdx.x / L < n ? rp[row + 1] : 0;
            acc[u] = 0;
            trips = max(trips, (ke[u] - kb[u] + L - 1) / L);
        }
        // trips > 0 means some row here has entries, so entry 0 exists and
        // serves as the in-range index of finished rows
        for (int t = 0; t < trips; ++t) {
            int cc[U];
            TV vv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = kb[u] + t * L;
                const int kk = k < ke[u] ? k : 0;
                cc[u] = col[kk];
                vv[u] = val[kk];
            }
            TX xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                xv[u] = x[cc[u]];
            __builtin_amdgcn_sched_barrier(0);   // all gathers in flight before the first use
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (kb[u] + t * L < ke[u])
                    acc[u] += (TA)vv[u] * (TA)xv[u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const TA a = lanes_sum(acc[u], L);   // valid in lane L - 1 of the row's lanes
            const int row = r0 + u * rpp + threadIdx.x / L;
            if (lane == L - 1 && row < n)
                y[row] = z ? s1 * a + s0 * z[row] : s1 * a;
        }
    }
}

template <typename T>
__device__ __forceinline__ T *wsp(ck::BSlot *s, int which) {
    return (T *)s->work + (int64_t)which * s->ld;
}

}  // namespace

// One launch: every listed slot advances by up to `budget` steps; BS threads
// per slot (256 when many slots share the GPU, 1024 for a single system).
template <typename T, int BS>
__global__ __launch_bounds__(BS) void batched_chunk(ck::BSlot *slots, ck::BStat *stat,
                                                    const int *active, int budget) {
    constexpr int NW = BS / 64;
    __shared__ T lds[NW];
    __shared__ double lds64[NW];
    __shared__ T hcol[ck::kBMaxM + 1];
    __shared__ T hacc[ck::kBMaxM + 1];
    __shared__ T wred[NW][ck::kBMaxM + 1];
    ck::BSlot *s = slots + active[blockIdx.x];
    const int tid = threadIdx.x;
    const int n = s->n, L = s->lanes;
    int phase = s->phase;
    if (phase == ck::B_DONE)
        return;
    if (s->bnorm < 0) {   // first launch of this request: ||b||, x0 = 0
        double q = 0;
        for (int i = tid; i < n; i += BS) {
            q += s->b[i] * s->b[i];
            if (!s->keep_x0)
                s->x[i] = 0.0;
        }
        const double bn = sqrt(wg_sum<BS>(q, lds64));
        if (tid == 0)
            s->bnorm = bn;
        __syncthreads();
        if (bn == 0.0) {   // b = 0: x = 0 is the solution
            for (int i = tid; i < n; i += BS)
                s->x[i] = 0.0;
            phase = ck::B_DONE;
            if (tid == 0) {
                s->status = ck::CONVERGED;
                s->relres = 0.0;
            }
        }
    }
    int steps = 0;
    while (steps < budget && phase != ck::B_DONE) {
        ++steps;
        if (phase == ck::B_OUTER) {
            // r = b - A x in FP64; beta = ||r||
            wg_spmv<BS, double, double, double>(n, L, s->rp, s->col, s->val64, s->x, -1.0, 1.0, s->b,
                                            s->r64);
            __syncthreads();
            double q = 0;
            const double *r64 = s->r64;
            for (int i0 = tid; i0 < n; i0 += kVec * BS) {
                double rv[kVec];
#pragma unroll
                for (int u = 0; u < kVec; ++u)
                    rv[u] = r64[min(i0 + u * BS, n - 1)];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < kVec; ++u)
                    if (i0 + u * BS < n)
                        q += rv[u] * rv[u];
            }
            const double beta = sqrt(wg_sum<BS>(q, lds64));
            const double rel = beta / s->bnorm;
            if (tid == 0) {
                s->relres = rel;
                s->beta = beta;
            }
            if (rel <= s->tol) {
                phase = ck::B_DONE;
                if (tid == 0)
                    s->status = ck::CONVERGED;
                break;
            }
            if (s->iter >= s->max_iter) {
                phase = ck::B_DONE;
                if (tid == 0)
                    s->status = ck::BUDGET;
                break;
            }
            const double inv = 1.0 / beta;
            if (s->kind == ck::B_CG) {
                T *r = wsp<T>(s, 0), *p = wsp<T>(s, 1), *d = wsp<T>(s, 3);
                T rr = 0;
                for (int i = tid; i < n; i += BS) {
                    const T ri = (T)(s->r64[i] * inv);
                    r[i] = ri;
                    p[i] = ri;
                    d[i] = 0;
                    rr += ri * ri;
                }
                rr = wg_sum<BS>(rr, lds);
                if (tid == 0) {
                    s->rho = (double)rr;
                    // FP32 inner solves stop at 1e-5 (their attainable
                    // accuracy); FP64 inner solves go to the outer target
                    s->inner_tol = fmax(s->tol * s->bnorm / beta, sizeof(T) == 4 ? 1e-5 : 0.0);
                    s->inner_iter = 0;
                }
            } else {
                T *v0 = wsp<T>(s, 0);
                for (int i = tid; i < n; i += BS)
                    v0[i] = (T)(s->r64[i] * inv);
                if (tid == 0) {
                    s->j = 0;
                    s->g[0] = 1;
                    for (int t = 1; t <= s->m; ++t)
                        s->g[t] = 0;
                }
            }
            if (tid == 0)
                s->outer += 1;
            phase = ck::B_INNER;
            __syncthreads();
            continue;
        }
        if (phase == ck::B_INNER && s->kind == ck::B_CG) {
            T *r = wsp<T>(s, 0), *p = wsp<T>(s, 1), *q = wsp<T>(s, 2), *d = wsp<T>(s, 3);
            const T *val = sizeof(T) == 4 ? (const T *)s->val32 : (const T *)s->val64;
            wg_spmv<BS, T, T, T>(n, L, s->rp, s->col, val, p, T(1), T(0), (const T *)nullptr, q);
            __syncthreads();
            T pq = 0;
            for (int i0 = tid; i0 < n; i0 += kVec * BS) {
                T pv[kVec], qv[kVec];
#pragma unroll
                for (int u = 0; u < kVec; ++u) {
                    const int i = min(i0 + u * BS, n - 1);
                    pv[u] = p[i];
                    qv[u] = q[i];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < kVec; ++u)
                    if (i0 + u * BS < n)
                        pq += pv[u] * qv[u];
            }
            const T sigma = wg_sum<BS>(pq, lds);
            if (!(sigma > T(0))) {
                phase = s->inner_iter == 0 ? ck::B_DONE : ck::B_UPDATE;
                if (phase == ck::B_DONE && tid == 0)
                    s->status = ck::BREAKDOWN;
                __syncthreads();
                continue;
            }
            const T rho = (T)s->rho;
            const T alpha = rho / sigma;
            T rr = 0;
            for (int i0 = tid; i0 < n; i0 += kVec * BS) {
                T dv[kVec], pv[kVec], rv[kVec], qv[kVec];
#pragma unroll
                for (int u = 0; u < kVec; ++u) {
                    const int i = min(i0 + u * BS, n - 1);
                    dv[u] = d[i];
                    pv[u] = p[i];
                    rv[u] = r[i];
                    qv[u] = q[i];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < kVec; ++u) {
                    const int i = i0 + u * BS;
                    if (i < n) {
                        d[i] = dv[u] + alpha * pv[u];
                        const T ri = rv[u] - alpha * qv[u];
                        r[i] = ri;
                        rr += ri * ri;
                    }
                }
            }
            const T rho_new = wg_sum<BS>(rr, lds);
            const int it = s->inner_iter + 1;
            const bool stop = sqrt((double)rho_new) <= s->inner_tol || it >= s->inner_cap ||
                              s->iter + 1 >= s->max_iter;
            const T bcg = rho_new / rho;
            if (!stop)
                for (int i0 = tid; i0 < n; i0 += kVec * BS) {
                    T rv[kVec], pv[kVec];
#pragma unroll
                    for (int u = 0; u < kVec; ++u) {
                        const int i = min(i0 + u * BS, n - 1);
                        rv[u] = r[i];
                        pv[u] = p[i];
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int u = 0; u < kVec; ++u)
                        if (i0 + u * BS < n)
                            p[i0 + u * BS] = rv[u] + bcg * pv[u];
                }
            __syncthreads();
            if (tid == 0) {
                s->rho = (double)rho_new;
                s->inner_iter = it;
                s->iter += 1;
            }
            if (stop)
                phase = ck::B_UPDATE;
            __syncthreads();
            continue;
        }
        if (phase == ck::B_INNER) {   // GMRES: one Arnoldi step (CGS2) + Givens
            const int j = s->j, m = s->m;
            const int64_t ld = s->ld;
            T *V = wsp<T>(s, 0);
            T *w = V + (int64_t)(j + 1) * s->ld;
            const T *val = sizeof(T) == 4 ? (const T *)s->val32 : (const T *)s->val64;
            wg_spmv<BS, T, T, T>(n, L, s->rp, s->col, val, V + (int64_t)j * s->ld, T(1), T(0),
                             (const T *)nullptr, w);
            __syncthreads();
            for (int pass = 0; pass < 2; ++pass) {
                T acc[ck::kBMaxM + 1];
#pragma unroll
                for (int c = 0; c <= ck::kBMaxM; ++c)
                    acc[c] = 0;
                for (int i = tid; i < n; i += BS) {
                    const T wi = w[i];
                    // columns in groups of 8 loads in flight
#pragma unroll
                    for (int g = 0; g <= ck::kBMaxM; g += 8) {
                        if (g <= j) {
                            T vv[8];
#pragma unroll
                            for (int c = 0; c < 8; ++c)
                                vv[c] = V[(int64_t)min(g + c, j) * ld + i];
                            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                            for (int c = 0; c < 8; ++c)
                                if (g + c <= ck::kBMaxM && g + c <= j)
                                    acc[g + c] += vv[c] * wi;
                        }
                    }
                }
#pragma unroll
                for (int c = 0; c <= ck::kBMaxM; ++c)
                    if (c <= j) {
                        const T v = ck::wave_sum_last(acc[c]);   // valid in lane 63
                        if ((tid & 63) == 63)
                            wred[tid >> 6][c] = v;
                    }
                __syncthreads();
                if (tid <= j) {
                    T h = (wred[0][tid] + wred[1][tid]) + (wred[2][tid] + wred[3][tid]);
                    for (int t = 4; t < NW; t += 4)
                        h += (wred[t][tid] + wred[t + 1][tid]) + (wred[t + 2][tid] + wred[t + 3][tid]);
                    hcol[tid] = h;
                    hacc[tid] = pass == 0 ? h : hacc[tid] + h;
                }
                __syncthreads();
                for (int i = tid; i < n; i += BS) {
                    T wi = w[i];
                    for (int g = 0; g <= j; g += 8) {
                        T vv[8];
#pragma unroll
                        for (int c = 0; c < 8; ++c)
                            vv[c] = V[(int64_t)min(g + c, j) * ld + i];
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int c = 0; c < 8; ++c)
                            if (g + c <= j)
                                wi -= hcol[min(g + c, j)] * vv[c];
                    }
                    w[i] = wi;
                }
                __syncthreads();
            }
            T nn = 0;
            for (int i0 = tid; i0 < n; i0 += kVec * BS) {
                T wv[kVec];
#pragma unroll
                for (int u = 0; u < kVec; ++u)
                    wv[u] = w[min(i0 + u * BS, n - 1)];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < kVec; ++u)
                    if (i0 + u * BS < n)
                        nn += wv[u] * wv[u];
            }
            const T hn = sqrt(wg_sum<BS>(nn, lds));
            __shared__ int stop_sh;
            __shared__ T inv_sh;
            if (tid == 0) {
                // Hessenberg column j in the inner precision (stored as double)
                double *Hj = s->H + j * (m + 1);
                for (int c = 0; c <= j; ++c)
                    Hj[c] = (double)hacc[c];
                Hj[j + 1] = (double)hn;
                for (int i = 0; i < j; ++i) {
                    const T a = (T)Hj[i], c2 = (T)Hj[i + 1];
                    const T ci = (T)s->cs[i], si = (T)s->sn[i];
                    Hj[i] = (double)(ci * a + si * c2);
                    Hj[i + 1] = (double)(-si * a + ci * c2);
                }
                const T a = (T)Hj[j], c2 = (T)Hj[j + 1];
                const T dd = sqrt(a * a + c2 * c2);
                int stop = 0;
                if (dd == T(0)) {
                    stop = 2;           // singular least-squares problem
                } else {
                    const T cj = a / dd, sj = c2 / dd, gj = (T)s->g[j];
                    s->cs[j] = (double)cj;
                    s->sn[j] = (double)sj;
                    Hj[j] = (double)dd;
                    Hj[j + 1] = 0;
                    s->g[j + 1] = (double)(-sj * gj);
                    s->g[j] = (double)(cj * gj);
                    s->j = j + 1;
                    s->iter += 1;
                    const double est = fabs((double)s->g[j + 1]) * s->beta / s->bnorm;
                    if (est <= s->tol || hn == T(0) || j + 1 == m || s->iter >= s->max_iter)
                        stop = 1;
                }
                stop_sh = stop;
                inv_sh = hn > T(0) ? T(1) / hn : T(0);
            }
            __syncthreads();
            const int stop = stop_sh;
            if (stop == 2) {
                phase = s->j == 0 ? ck::B_DONE : ck::B_UPDATE;
                if (phase == ck::B_DONE && tid == 0)
                    s->status = ck::BREAKDOWN;
            } else if (stop == 1) {
                phase = ck::B_UPDATE;
            } else {
                const T inv = inv_sh;
                for (int i = tid; i < n; i += BS)
                    w[i] *= inv;
            }
            __syncthreads();
            continue;
        }
        // B_UPDATE: x += beta * d
        const double beta = s->beta;
        if (s->kind == ck::B_CG) {
            const T *d = wsp<T>(s, 3);
            for (int i = tid; i < n; i += BS)
                s->x[i] += beta * (double)d[i];
        } else {
            const int k = s->j, m = s->m;
            if (tid == 0) {
                for (int i = k - 1; i >= 0; --i) {
                    T acc = (T)s->g[i];
                    for (int t = i + 1; t < k; ++t)
                        acc -= (T)s->H[t * (m + 1) + i] * (T)s->y[t];
                    s->y[i] = (double)(acc / (T)s->H[i * (m + 1) + i]);
                }
            }
            __syncthreads();
            const T *V = wsp<T>(s, 0);
            for (int i = tid; i < n; i += BS) {
                double acc = 0;
                for (int c = 0; c < k; ++c)
                    acc += (double)s->y[c] * (double)V[(int64_t)c * s->ld + i];
                s->x[i] += beta * acc;
            }
        }
        phase = ck::B_OUTER;
        __syncthreads();
    }
    __syncthreads();
    if (tid == 0) {
        s->phase = phase;
        s->launches += 1;
        ck::BStat &o = stat[active[blockIdx.x]];
        o.phase = phase;
        o.status = s->status;
        o.iter = s->iter;
        o.outer = s->outer;
        o.relres = s->relres;
    }
}

namespace ck {

int64_t bslot_work_elems(int kind, int64_t n, int m) {
    const int64_t ld = ceil_div(std::max<int64_t>(n, 1), 64) * 64;
    return kind == B_CG ? 4 * ld : (int64_t)(m + 1) * ld;
}

ck_status launch_batched_chunk(BSlot *slots, BStat *stat, const int *active, int nactive,
                               int budget, bool fp32, hipStream_t s, bool wide) {
    if (nactive <= 0)
        return CK_OK;
    if (wide) {
        if (fp32)
            hipLaunchKernelGGL((batched_chunk<float, 1024>), dim3(nactive), dim3(1024), 0, s,
                               slots, stat, active, budget);
        else
            hipLaunchKernelGGL((batched_chunk<double, 1024>), dim3(nactive), dim3(1024), 0, s,
                               slots, stat, active, budget);
    } else if (fp32) {
        hipLaunchKernelGGL((batched_chunk<float, 256>), dim3(nactive), dim3(256), 0, s, slots,
                           stat, active, budget);
    } else {
        hipLaunchKernelGGL((batched_chunk<double, 256>), dim3(nactive), dim3(256), 0, s, slots,
                           stat, active, budget);
    }
    CK_HIP(hipGetLastError());
    return CK_OK;
}

}  // namespace ck
