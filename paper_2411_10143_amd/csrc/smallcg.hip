// Single-workgroup FP64 conjugate gradient for small systems (n <= 4096).
//
// A system this small cannot fill the GPU, and a launch per CG step would
// make launch latency the bound.  One 1024-thread workgroup runs the whole
// solve in one launch: thread t owns rows t, t + 1024, ... (R <= 4 of them);
// x, r, p and q of its rows live in registers, p also in LDS (the product
// gathers it from there), and only the matrix (L2-resident after the first
// step) and, at the rare residual steps, b are read from memory.  When no
// row has more than 5 entries (1D and 2D stencils, convection-diffusion) the
// matrix itself is loaded into registers once per solve and every product
// only gathers p from LDS.  Otherwise, when no
// row has more than 16 entries, the matrix is first copied column-major into
// a scratch buffer, so that each product reads it in whole cache lines (the
// row-major arrays, read one entry per lane per step, re-fetched partly used
// lines at every step).  The product sums each row with one lane in
// ascending entry order; the loads of all R rows' next entries are issued
// together.  Dot products reduce in a fixed
// order (wave butterfly, then the 16 wave sums in order), so the result is
// deterministic.  (Eight rows per thread would spill registers.)
//
// The iteration is the same Hestenes-Stiefel CG as the multi-kernel path:
// r = b - A x, p = r; then q = A p, alpha = rho / p.q, x += alpha p,
// r -= alpha q, stop when ||r|| / ||b|| <= tol; at a stop the true residual
// b - A x is recomputed and CG restarts from the current x (at most three
// times) if it is above tol.
#include "batched.hpp"

namespace {

constexpr int kWgThreads = 1024;
constexpr int kWgWaves = kWgThreads / 64;
constexpr int kWgCgRegK = 5;   // longest row kept in registers

// sum over the workgroup, returned to every thread (fixed order).  Successive
// calls alternate between the two halves of `red` (2 x kWgWaves doubles), so
// one barrier per call suffices: a half is rewritten only two calls later,
// after every thread has passed the barrier of the call in between, and so
// has finished reading it.
__device__ __forceinline__ double wg_sum_1024(double v, double *red, int &parity) {
    double *buf = red + parity * kWgWaves;
    parity ^= 1;
    v = ck::wave_sum_last(v);   // valid in lane 63
    if ((threadIdx.x & 63) == 63)
        buf[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0;
#pragma unroll
    for (int w = 0; w < kWgWaves; ++w)
        s += buf[w];
    return s;
}

// q[u] = (A v)[row u of this thread], v in LDS.  (Issuing step t + 1's loads
// before step t's gathers measured 6 % slower here.)
template <int R>
__device__ __forceinline__ void wg_matvec(const int (&kb)[R], const int (&ke)[R], int trips,
                                          const int *__restrict__ col,
                                          const double *__restrict__ val, const double *v,
                                          double (&q)[R]) {
#pragma unroll
    for (int u = 0; u < R; ++u)
        q[u] = 0;
    for (int t = 0; t < trips; ++t) {
        int cc[R];
        double vv[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int k = kb[u] + t;
            const int kk = k < ke[u] ? k : 0;   // entry 0 exists when trips > 0
            cc[u] = col[kk];
            vv[u] = val[kk];
        }
        __builtin_amdgcn_sched_barrier(0);   // every row's loads in flight together
#pragma unroll
        for (int u = 0; u < R; ++u)
            if (kb[u] + t < ke[u])
                q[u] += vv[u] * v[cc[u]];
    }
}

// The same product from the column-major copy, slots in pairs: slots 2q and
// 2q + 1 of local row i are the int2 / double2 at q * RW + i.  A step's loads
// are consecutive across the lanes and bring two slots of every row, so each
// product reads the matrix once, in whole cache lines, in ceil(K / 2) rounds
// (the row-major arrays, read one entry per lane per step, re-fetched partly
// used lines at every step).  Entries are summed in the same order, so the
// result is the same.
template <int R>
__device__ __forceinline__ void wg_matvec_cm(const int (&len)[R], int K,
                                             const int2 *__restrict__ ccol,
                                             const double2 *__restrict__ cval, const double *v,
                                             double (&q)[R]) {
    constexpr int RW = R * kWgThreads;
#pragma unroll
    for (int u = 0; u < R; ++u)
        q[u] = 0;
    for (int s = 0; s < K; s += 2) {
        int2 cc[R];
        double2 vv[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int i = threadIdx.x + u * kWgThreads;
            cc[u] = ccol[(s >> 1) * RW + i];
            vv[u] = cval[(s >> 1) * RW + i];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < R; ++u) {
            if (s < len[u])
                q[u] += vv[u].x * v[cc[u].x];
            if (s + 1 < len[u])
                q[u] += vv[u].y * v[cc[u].y];
        }
    }
}

// The product with the matrix in registers: slot k of local row u holds
// rv[k][u] and its column, the 16-bit half k % 2 of rcp[k / 2][u] (columns
// are below 4096), loaded once per solve.  Slots past the row's length hold
// value 0 and column 0: p[0] is finite while the solve runs (a non-finite
// p.q ends it first) and q starts at +0, so adding 0 * p[0] leaves q's bits
// unchanged, and every row's sum equals, bit for bit, the other forms' sum
// of its entries in the same order.
constexpr int kWgRegPairs = (kWgCgRegK + 1) / 2;
template <int R>
__device__ __forceinline__ void wg_matvec_reg(const unsigned (&rcp)[kWgRegPairs][R],
                                              const double (&rv)[kWgCgRegK][R], const double *v,
                                              double (&q)[R]) {
#pragma unroll
    for (int u = 0; u < R; ++u)
        q[u] = 0;
    // gathers in rounds of G slots (all rows' loads of a round in flight
    // together; more at once would spill registers at four rows per lane)
    constexpr int G = R >= 4 ? 1 : kWgCgRegK;
#pragma unroll
    for (int k0 = 0; k0 < kWgCgRegK; k0 += G) {
        double g[G][R];
#pragma unroll
        for (int k = k0; k < k0 + G && k < kWgCgRegK; ++k)
#pragma unroll
            for (int u = 0; u < R; ++u) {
                // an empty statement that claims to change w: the columns are
                // unpacked here, at each use, instead of being hoisted out of
                // the CG loop as 20 loop-invariant registers
                unsigned w = rcp[k >> 1][u];
                asm volatile("" : "+v"(w));
                g[k - k0][u] = v[(k & 1) ? (w >> 16) : (w & 0xffffu)];
            }
#pragma unroll
        for (int k = k0; k < k0 + G && k < kWgCgRegK; ++k)
#pragma unroll
            for (int u = 0; u < R; ++u)
                q[u] += rv[k][u] * g[k - k0][u];
        __builtin_amdgcn_sched_barrier(0);
    }
}

}  // namespace

// The solve after the prologue, one instantiation per product form (the
// form is fixed for the whole solve, so each keeps only its own state live):
// the matrix in registers, the column-major copy, or the row-major arrays.
enum { kWgRows = 0, kWgColMajor = 1, kWgReg = 2 };
template <int R, int MODE>
__device__ __forceinline__ void cg_wg_run(int n, const int (&kb)[R], const int (&ke)[R],
                                          const int (&len)[R], int trips, int K,
                                          double (&xr)[R], double bb,
                                          const int *__restrict__ col,
                                          const double *__restrict__ val,
                                          const double *__restrict__ b, double *__restrict__ x,
                                          double tol, int max_iter, int2 *__restrict__ ccol,
                                          double2 *__restrict__ cval, ck::WgCgOut *out,
                                          double *v, double *red, int parity) {
    constexpr int RW = R * kWgThreads;
    const int t = threadIdx.x;
    double rr[R], pr[R], q[R];
    constexpr bool reg = MODE == kWgReg, cm = MODE == kWgColMajor;
    unsigned rcp[kWgRegPairs][R];
    double rv[kWgCgRegK][R];
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
        for (int k = 0; k < kWgRegPairs; ++k)
            rcp[k][u] = 0;
#pragma unroll
    for (int k = 0; k < kWgCgRegK; ++k)
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const bool in = reg && k < len[u];
            rcp[k >> 1][u] |= (in ? (unsigned)col[kb[u] + k] : 0u) << (16 * (k & 1));
            rv[k][u] = in ? val[kb[u] + k] : 0.0;
        }
    auto matvec = [&]() {
        if constexpr (reg)
            wg_matvec_reg<R>(rcp, rv, v, q);
        else if constexpr (cm)
            wg_matvec_cm<R>(len, K, ccol, cval, v, q);
        else
            wg_matvec<R>(kb, ke, trips, col, val, v, q);
    };
    if constexpr (cm) {
        for (int s = 0; s < K; s += 2) {
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const int i = t + u * kWgThreads;
                const bool in0 = s < len[u], in1 = s + 1 < len[u];   // rows past n: len 0
                ccol[(s >> 1) * RW + i] = make_int2(in0 ? col[kb[u] + s] : 0,
                                                    in1 ? col[kb[u] + s + 1] : 0);
                cval[(s >> 1) * RW + i] = make_double2(in0 ? val[kb[u] + s] : 0.0,
                                                       in1 ? val[kb[u] + s + 1] : 0.0);
            }
        }
        // the copy is read by other waves of this workgroup: the barrier
        // below (in the first workgroup sum) orders it
        __threadfence_block();
    }
    const double bnorm = sqrt(wg_sum_1024(bb, red, parity));
    int status = ck::BUDGET, iters = 0, restarts = 0;
    double relres = 0;
    if (bnorm == 0.0) {
#pragma unroll
        for (int u = 0; u < R; ++u)
            xr[u] = 0;
        status = ck::CONVERGED;
    } else {
        for (restarts = 0; restarts <= 3; ++restarts) {
            // r = b - A x
#pragma unroll
            for (int u = 0; u < R; ++u)
                if (t + u * kWgThreads < n)
                    v[t + u * kWgThreads] = xr[u];
            __syncthreads();
            matvec();
            double rho = 0;
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const int i = t + u * kWgThreads;
                rr[u] = (i < n ? b[i] : 0.0) - q[u];
                pr[u] = rr[u];
                rho += rr[u] * rr[u];
            }
            rho = wg_sum_1024(rho, red, parity);   // its barrier also retires the reads of v
            relres = sqrt(rho) / bnorm;
            if (relres <= tol) {
                status = ck::CONVERGED;
                break;
            }
            int state = ck::RUN;
            while (state == ck::RUN) {
                if (iters >= max_iter) {
                    state = ck::BUDGET;
                    break;
                }
#pragma unroll
                for (int u = 0; u < R; ++u)
                    if (t + u * kWgThreads < n)
                        v[t + u * kWgThreads] = pr[u];
                __syncthreads();
                matvec();
                double pq = 0;
#pragma unroll
                for (int u = 0; u < R; ++u)
                    pq += pr[u] * q[u];
                const double sigma = wg_sum_1024(pq, red, parity);
                if (!(sigma > 0.0)) {
                    state = ck::BREAKDOWN;
                    break;
                }
                const double alpha = rho / sigma;
                double rn = 0;
#pragma unroll
                for (int u = 0; u < R; ++u) {
                    xr[u] += alpha * pr[u];
                    rr[u] -= alpha * q[u];
                    rn += rr[u] * rr[u];
                }
                const double rho_new = wg_sum_1024(rn, red, parity);
                ++iters;
                if (sqrt(rho_new) / bnorm <= tol) {
                    state = ck::CONVERGED;
                    break;
                }
                const double beta = rho_new / rho;
#pragma unroll
                for (int u = 0; u < R; ++u)
                    pr[u] = rr[u] + beta * pr[u];
                rho = rho_new;
            }
            if (state == ck::BREAKDOWN) {
                status = ck::BREAKDOWN;
                break;
            }
            // true residual of the current x
#pragma unroll
            for (int u = 0; u < R; ++u)
                if (t + u * kWgThreads < n)
                    v[t + u * kWgThreads] = xr[u];
            __syncthreads();
            matvec();
            double tr = 0;
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const int i = t + u * kWgThreads;
                const double d = (i < n ? b[i] : 0.0) - q[u];
                tr += d * d;
            }
            relres = sqrt(wg_sum_1024(tr, red, parity)) / bnorm;
            if (relres <= tol) {
                status = ck::CONVERGED;
                break;
            }
            if (state == ck::BUDGET) {
                status = ck::BUDGET;
                break;
            }
        }
        if (restarts > 3)
            restarts = 3;
    }
#pragma unroll
    for (int u = 0; u < R; ++u)
        if (t + u * kWgThreads < n)
            x[t + u * kWgThreads] = xr[u];
    if (t == 0) {
        out->status = status;
        out->iter = iters;
        out->restarts = restarts;
        out->relres = relres;
    }
}

// ccol / cval: scratch of kWgCgColMajorK / 2 * R * 1024 pairs for the
// column-major copy, used when no row has more than kWgCgColMajorK entries.
template <int R>
__global__ __launch_bounds__(kWgThreads) void cg_wg(int n, const int *__restrict__ rp,
                                                    const int *__restrict__ col,
                                                    const double *__restrict__ val,
                                                    const double *__restrict__ b,
                                                    double *__restrict__ x, double tol,
                                                    int max_iter, int2 *__restrict__ ccol,
                                                    double2 *__restrict__ cval,
                                                    ck::WgCgOut *out) {
    __shared__ double v[kWgThreads * R];   // p (or x while forming the residual)
    __shared__ double red[2 * kWgWaves];
    __shared__ int kmax[kWgWaves];
    int parity = 0;
    const int t = threadIdx.x;
    int kb[R], ke[R], len[R];
    double xr[R];
    int trips = 0;
    double bb = 0;
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int i = t + u * kWgThreads;
        const bool in = i < n;
        kb[u] = in ? rp[i] : 0;
        ke[u] = in ? rp[i + 1] : 0;
        len[u] = ke[u] - kb[u];
        const double bi = in ? b[i] : 0.0;
        xr[u] = in ? x[i] : 0.0;
        trips = max(trips, ke[u] - kb[u]);
        bb += bi * bi;
    }
    // longest row of the system: it picks the product form for the solve
    int K = trips;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        K = max(K, __shfl_xor(K, off, 64));
    if ((t & 63) == 0)
        kmax[t >> 6] = K;
    __syncthreads();
    K = 0;
#pragma unroll
    for (int w = 0; w < kWgWaves; ++w)
        K = max(K, kmax[w]);
    if (K <= kWgCgRegK)
        cg_wg_run<R, kWgReg>(n, kb, ke, len, trips, K, xr, bb, col, val, b, x, tol, max_iter,
                             ccol, cval, out, v, red, parity);
    else if (K <= ck::kWgCgColMajorK)
        cg_wg_run<R, kWgColMajor>(n, kb, ke, len, trips, K, xr, bb, col, val, b, x, tol,
                                  max_iter, ccol, cval, out, v, red, parity);
    else
        cg_wg_run<R, kWgRows>(n, kb, ke, len, trips, K, xr, bb, col, val, b, x, tol, max_iter,
                              ccol, cval, out, v, red, parity);
}

namespace ck {

ck_status launch_cg_wg(int n, const int *rp, const int *col, const double *val, const double *b,
                       double *x, double tol, int max_iter, void *cm_col, void *cm_val,
                       WgCgOut *out, hipStream_t s) {
    int2 *ccol = (int2 *)cm_col;
    double2 *cval = (double2 *)cm_val;
    if (n < 1 || n > kWgCgMaxN)
        return fail(CK_E_INVALID, "single-workgroup CG takes 1..%d rows, got %d", kWgCgMaxN, n);
    const dim3 grid(1), block(kWgThreads);
    if (n <= kWgThreads)
        hipLaunchKernelGGL((cg_wg<1>), grid, block, 0, s, n, rp, col, val, b, x, tol, max_iter,
                           ccol, cval, out);
    else if (n <= 2 * kWgThreads)
        hipLaunchKernelGGL((cg_wg<2>), grid, block, 0, s, n, rp, col, val, b, x, tol, max_iter,
                           ccol, cval, out);
    else
        hipLaunchKernelGGL((cg_wg<4>), grid, block, 0, s, n, rp, col, val, b, x, tol, max_iter,
                           ccol, cval, out);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

}  // namespace ck
