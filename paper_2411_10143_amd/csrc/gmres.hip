// GMRES(m) kernels (the solver of the paper's evaluation, Section IV).
//
// One Arnoldi step j is classical Gram-Schmidt applied twice (CGS2):
//   h1 = V_j^T w, w' = w - V_j h1, h2 = V_j^T w',
//   h_{j+1,j} = ||w' - V_j h2|| = sqrt(||w'||^2 - ||h2||^2) (Pythagoras: the
//   subtracted part is w''s projection on the orthonormal V_j),
//   v_{j+1} = (w' - V_j h2) / h_{j+1,j},  column j of H = h1 + h2,
// with w = A v_j.  Forming v_{j+1} would take a third sweep over the basis;
// instead it is left for the next step, which applies the SpMV to w' itself
// (z = A w', written to column j+2) and opens with one sweep that forms both
// v_{j+1} = (w' - V_j h2) / h and A v_{j+1} = (z - V_{j+1} u) / h, where
// u = Hbar_j h2 is A (V_j h2) expressed in the basis through the Arnoldi
// relation A V_j = V_{j+1} Hbar_j, and that also sums the partials of
// V_{j+1}^T A v_{j+1}.  So each step streams the basis twice:
//   step 0:  pass 1 (partials of V_0^T w)               -> finish: h1
//   step j:  pass 3+1 (v_j, A v_j in place, partials of V_j^T A v_j) -> h1
//   then     pass 2: w' = w - V_j h1, partials of V_j^T w' (h2) and ||w'||^2
//            givens: one workgroup sums the pass-2 partials, forms h_{j+1,j},
//            H column j (kept unrotated for u, and rotated), the previous
//            Givens rotations, rotation j, residual estimate |g_{j+1}|, the
//            cycle stop decision, and u = Hbar_j h2 for the next step.
// After the first projection h2 is of rounding size relative to w', so the
// corrections through h2 and u change w' and z by rounding-size amounts.
// The last step of a cycle needs no v_{j+1}: the update x += V_k y uses
// v_0 .. v_{k-1}.  Per-column sums are reduced in a fixed order (wave
// butterfly, 4 waves, then block order), so results are deterministic.  The
// least-squares solve and the solution update close the cycle on the
// device; nothing returns to the host inside a cycle.
#include "solvers.hpp"

using ck::GmDev;

namespace {

// The passes below are written for NC >= ncols columns with no branch per
// column: column c >= ncols reloads column ncols - 1 (an L2 hit), its
// coefficient h[c] is 0 (so the subtraction is exact) and its accumulator is
// never written out.  Without branches every column's load of an element is
// in flight at once; with a branch per column each load waited for the one
// before it.
__device__ __forceinline__ int64_t clampc(int c, int ncols) { return c < ncols ? c : ncols - 1; }

// partials[c*G + b] = block b's sum of acc[c]  (c < ncols).  The NC wave
// sums run back to back at the end of the pass, so they use register-to-
// register (DPP) moves, valid in lane 63.
template <typename T, int NC>
__device__ __forceinline__ void block_cols(const T (&acc)[NC], int ncols, T *partials, int64_t b,
                                           int64_t G) {
    __shared__ T lds[4][NC];
    const int w = threadIdx.x / 64, lane = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (c < ncols) {
            const T v = ck::wave_sum_last(acc[c]);
            if (lane == 63)
                lds[w][c] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < ncols) {
        const int c = threadIdx.x;
        partials[c * G + b] = (lds[0][c] + lds[1][c]) + (lds[2][c] + lds[3][c]);
    }
}

}  // namespace

template <typename T, int NC>
__global__ __launch_bounds__(256) void gm_pass1(int64_t n, int64_t G, int ncols,
                                                const T *__restrict__ V, int64_t ldv,
                                                const T *__restrict__ w,
                                                T *__restrict__ partials, const GmDev<T> *st) {
    if (st->halt)
        return;
    const int64_t b = blockIdx.x;
    T acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c)
        acc[c] = 0;
    for (int64_t i = b * 256 + threadIdx.x; i < n; i += G * 256) {
        const T wi = w[i];
        T vv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c)
            vv[c] = V[clampc(c, ncols) * ldv + i];
        __builtin_amdgcn_sched_barrier(0);   // every load issued before the first use
#pragma unroll
        for (int c = 0; c < NC; ++c)
            acc[c] += vv[c] * wi;
    }
    block_cols<T, NC>(acc, ncols, partials, b, G);
}

template <typename T, int NC>
__global__ __launch_bounds__(256) void gm_pass2(int64_t n, int64_t G, int ncols,
                                                const T *__restrict__ V, int64_t ldv,
                                                T *__restrict__ w, T *__restrict__ partials,
                                                const GmDev<T> *st) {
    // A halted solve runs no rows (and leaves zero partials, which no later
    // kernel reads): the flag only sets the loop bound, so the coefficient
    // loads are issued with it rather than after an early exit.  h1 holds
    // kMaxRestart + 1 >= NC entries.
    const int64_t nl = st->halt ? 0 : n;
    T h[NC], acc[NC], nn = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const T hc = st->h1[c];   // unconditional: the loads merge
        h[c] = c < ncols ? hc : T(0);
        acc[c] = 0;
    }
    const int64_t b = blockIdx.x;
    for (int64_t i = b * 256 + threadIdx.x; i < nl; i += G * 256) {
        T vv[NC];
        T wi = w[i];
#pragma unroll
        for (int c = 0; c < NC; ++c)
            vv[c] = V[clampc(c, ncols) * ldv + i];
        __builtin_amdgcn_sched_barrier(0);   // every load issued before the first use
#pragma unroll
        for (int c = 0; c < NC; ++c)
            wi -= h[c] * vv[c];
        w[i] = wi;
        nn += wi * wi;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            acc[c] += vv[c] * wi;
    }
    block_cols<T, NC>(acc, ncols, partials, b, G);
    __shared__ T lds[4];
    nn = ck::block_sum(nn, lds);
    if (threadIdx.x == 0)
        partials[ncols * G + b] = nn;
}

// Step j >= 1 opens here: column j holds w' of step j - 1 (after its first
// projection, not yet corrected by h2 nor normalised) and column j + 1 holds
// z = A w'.  One sweep over V_{j-1} forms, in place, v_j = (w' - V_{j-1} h2)
// * inv and A v_j = (z - V_{j-1} u_{0..j-1} - u_j v_j) * inv, and the
// partials of V_j^T A v_j (columns 0..j).  h2, u and inv are step j - 1's.
template <typename T, int NC>
__global__ __launch_bounds__(256) void gm_pass31(int64_t n, int64_t G, int j,
                                                 T *__restrict__ V, int64_t ldv,
                                                 T *__restrict__ partials, const GmDev<T> *st) {
    const int nold = j;   // finished columns 0 .. j-1, read from memory (NC >= j + 1)
    T h2[NC], u[NC], acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const T hc = st->h2[c], uc = st->u[c];   // unconditional: the loads merge
        h2[c] = c < nold ? hc : T(0);
        u[c] = c < nold ? uc : T(0);
        acc[c] = 0;
    }
    const T uj = st->u[j];
    const T inv = st->inv;
    const int64_t nl = st->halt ? 0 : n;   // as in gm_pass2: no rows once halted
    const int64_t b = blockIdx.x;
    T *wv = V + (int64_t)j * ldv;         // w' in, v_j out
    T *zw = V + (int64_t)(j + 1) * ldv;   // z in, A v_j out
    T accj = 0;
    for (int64_t i = b * 256 + threadIdx.x; i < nl; i += G * 256) {
        T a = wv[i], zz = zw[i];
        T vv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c)
            vv[c] = V[clampc(c, nold) * ldv + i];
        __builtin_amdgcn_sched_barrier(0);   // every load issued before the first use
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            a -= h2[c] * vv[c];
            zz -= u[c] * vv[c];
        }
        const T vj = a * inv;
        zz -= uj * vj;
        const T wi = zz * inv;
        wv[i] = vj;
        zw[i] = wi;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            acc[c] += vv[c] * wi;
        accj += vj * wi;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (c == j)
            acc[c] = accj;   // column j is v_j itself (the loop's acc[j] saw a reloaded column)
    block_cols<T, NC>(acc, j + 1, partials, b, G);
}

// out[c] = sum_b partials[c*G + b]; block c reduces column c in block order
template <typename T>
__global__ __launch_bounds__(256) void gm_finish_cols(int64_t G, const T *__restrict__ partials,
                                                      int which, GmDev<T> *st) {
    __shared__ T lds[4];
    // the partials are read whether or not the solve has halted (they are
    // always allocated); only the store depends on the flag
    const int halt = st->halt;
    const int c = blockIdx.x;
    const T s = ck::sum_partials(partials + c * G, G, lds);
    if (!halt && threadIdx.x == 0)
        (which == 1 ? st->h1 : st->h2)[c] = s;
}

// Pass-2 finish and Givens step in one 1024-thread workgroup:
//  1. wave w sums the G block partials of columns w, w + 16, ... (h2[c] for
//     c <= j, and ||w'||^2 as column j + 1), lanes striding the blocks, then a
//     wave butterfly (fixed order);
//  2. h_{j+1,j} = sqrt(||w'||^2 - ||h2||^2), Hessenberg column j (h1 + h2),
//     previous rotations, new rotation, residual estimate -- one thread, from
//     LDS, with no global-memory round trip per rotation.
template <typename T>
__global__ __launch_bounds__(1024) void gm_finish_givens(int64_t G, const T *__restrict__ partials,
                                                         GmDev<T> *st) {
    constexpr int U = 8;
    __shared__ T col[ck::kMaxRestart], h2[ck::kMaxRestart + 1], cs[ck::kMaxRestart],
        sn[ck::kMaxRestart];
    __shared__ T hr[ck::kMaxRestart * (ck::kMaxRestart + 1)];   // Hraw columns 0 .. j-1
    const int halt = st->halt, m = st->m, j = st->j;   // one round trip
    if (halt)
        return;
    // Loads that do not depend on the partial sums are issued first, into
    // registers, so that their latency overlaps the sums': the unrotated
    // columns 0 .. j-1 (for u below; one entry per thread up to m = 31),
    // the previous rotations and this column's first-pass coefficients.
    const int t = threadIdx.x;
    const int nh = j * (m + 1);
    const T hr0 = t < nh ? st->Hraw[t] : T(0);
    const T cs0 = t < j ? st->cs[t] : T(0), sn0 = t < j ? st->sn[t] : T(0);
    const T h10 = t <= j ? st->h1[t] : T(0);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int c = w; c <= j + 1; c += 16) {
        const T *pc = partials + (int64_t)c * G;
        T acc = 0;
        for (int64_t b0 = lane; b0 < G; b0 += 64 * U) {
            T v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t b = b0 + 64 * u;
                v[u] = __builtin_nontemporal_load(&pc[b < G ? b : G - 1]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (b0 + 64 * u < G)
                    acc += v[u];
        }
        acc = ck::wave_sum_last(acc);   // valid in lane 63
        if (lane == 63) {
            h2[c] = acc;
            st->h2[c] = acc;   // pass 3 subtracts V h2
        }
    }
    if (t < nh)
        hr[t] = hr0;
    for (int k = t + 1024; k < nh; k += 1024)   // m > 31 only
        hr[k] = st->Hraw[k];
    if (t < j) {   // j < kMaxRestart <= 1024
        cs[t] = cs0;
        sn[t] = sn0;
    }
    __syncthreads();
    if (t <= j)
        col[t] = h10 + h2[t];
    __shared__ T hn_s;
    if (threadIdx.x == 0) {
        T proj = 0;
        for (int c = 0; c <= j; ++c)
            proj += h2[c] * h2[c];
        const T nrm2 = h2[j + 1] - proj;
        hn_s = nrm2 > T(0) ? sqrt(nrm2) : T(0);
    }
    __syncthreads();
    const T hn = hn_s;
    // unrotated column j, then u = Hbar_j h2 (row i sums columns c >= i - 1)
    T *Rj = st->Hraw + (int64_t)j * (m + 1);
    for (int c = threadIdx.x; c <= j; c += 1024)
        Rj[c] = col[c];
    if (threadIdx.x == 0)
        Rj[j + 1] = hn;
    for (int i = threadIdx.x; i <= j + 1; i += 1024) {
        T acc = 0;
        for (int c = i > 0 ? i - 1 : 0; c < j; ++c)
            acc += hr[c * (m + 1) + i] * h2[c];
        acc += (i <= j ? col[i] : hn) * h2[j];
        st->u[i] = acc;
    }
    if (threadIdx.x != 0)
        return;
    T *Hj = st->H + (int64_t)j * (m + 1);
    // previous rotations applied to (h_0j, ..., h_jj, hn); `a` carries entry i
    T a = col[0];
    for (int i = 0; i < j; ++i) {
        const T c2 = col[i + 1];
        Hj[i] = cs[i] * a + sn[i] * c2;
        a = -sn[i] * a + cs[i] * c2;
    }
    const T c2 = hn;
    Hj[j] = a;
    Hj[j + 1] = c2;
    const T d = sqrt(a * a + c2 * c2);
    if (d == T(0)) {
        st->final_state = ck::BREAKDOWN;
        st->cycle_stop = ck::BREAKDOWN;
        st->halt = 1;
        return;
    }
    const T cj = a / d, sj = c2 / d;
    const T gj = st->g[j];
    const double bnorm = st->bnorm, tol = st->tol;
    const int iter = st->iter + 1, max_iter = st->max_iter;
    st->cs[j] = cj;
    st->sn[j] = sj;
    Hj[j] = d;
    Hj[j + 1] = 0;
    const T gj1 = -sj * gj;
    st->g[j + 1] = gj1;
    st->g[j] = cj * gj;
    st->j = j + 1;
    st->iter = iter;
    const double relres = fabs((double)gj1) / bnorm;
    st->relres = relres;
    int stop = ck::RUN;
    if (relres <= tol)
        stop = ck::CONVERGED;
    else if (hn == T(0))
        stop = ck::BREAKDOWN;
    else if (iter >= max_iter)
        stop = ck::BUDGET;
    else if (j + 1 == m)
        stop = ck::FULL;
    st->cycle_stop = stop;
    st->halt = stop != ck::RUN;
    st->inv = hn > T(0) ? T(1) / hn : T(0);
}

// Cycle start: partials of ||r||^2 (FP64)
template <typename T>
__global__ __launch_bounds__(256) void gm_start_norm(int64_t n, int64_t G,
                                                     const double *__restrict__ r,
                                                     double *__restrict__ partials,
                                                     const GmDev<T> *st) {
    __shared__ double lds[4];
    if (st->final_state != ck::RUN)
        return;
    const int64_t b = blockIdx.x;
    double s = 0;
    for (int64_t i = b * 256 + threadIdx.x; i < n; i += G * 256)
        s += r[i] * r[i];
    s = ck::block_sum(s, lds);
    if (threadIdx.x == 0)
        partials[b] = s;
}

// beta = ||r||, true-residual convergence test, g = beta e1
template <typename T>
__global__ __launch_bounds__(256) void gm_start_finish(int64_t G,
                                                       const double *__restrict__ partials,
                                                       GmDev<T> *st) {
    __shared__ double lds[4];
    if (st->final_state != ck::RUN)
        return;
    const double tot = ck::sum_partials(partials, G, lds);
    if (threadIdx.x != 0)
        return;
    const double beta = sqrt(tot);
    st->beta = beta;
    st->relres = beta / st->bnorm;
    if (st->relres <= st->tol) {
        st->final_state = ck::CONVERGED;
        st->halt = 1;
        return;
    }
    if (st->iter >= st->max_iter) {
        st->final_state = ck::BUDGET;
        st->halt = 1;
        return;
    }
    st->inv_beta = 1.0 / beta;
    st->j = 0;
    st->cycle_stop = ck::RUN;
    st->halt = 0;
    st->cycles += 1;
    st->g[0] = (T)beta;
    for (int t = 1; t <= st->m; ++t)
        st->g[t] = 0;
}

template <typename T>
__global__ __launch_bounds__(256) void gm_start_v0(int64_t n, T *__restrict__ v0,
                                                   const double *__restrict__ r,
                                                   const GmDev<T> *st) {
    if (st->halt)
        return;
    const double inv = st->inv_beta;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256)
        v0[i] = (T)(r[i] * inv);
}

// Cycle end: back substitution R y = g over the k = j columns formed.
template <typename T>
__global__ void gm_solve_y(GmDev<T> *st) {
    if (st->final_state != ck::RUN || threadIdx.x != 0)
        return;
    const int m = st->m, k = st->j;
    for (int i = k - 1; i >= 0; --i) {
        T s = st->g[i];
        for (int t = i + 1; t < k; ++t)
            s -= st->H[(int64_t)t * (m + 1) + i] * st->y[t];
        st->y[i] = s / st->H[(int64_t)i * (m + 1) + i];
    }
}

// x += V_k y, accumulated in FP64 (the basis may be FP32).
template <typename T>
__global__ __launch_bounds__(256) void gm_update_x(int64_t n, double *__restrict__ x,
                                                   const T *__restrict__ V, int64_t ldv,
                                                   const GmDev<T> *st) {
    __shared__ double ys[ck::kMaxRestart];
    if (st->final_state != ck::RUN)
        return;
    const int k = st->j;
    for (int c = threadIdx.x; c < k; c += 256)
        ys[c] = (double)st->y[c];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        double acc = 0;
        for (int c = 0; c < k; ++c)
            acc += ys[c] * (double)V[c * ldv + i];
        x[i] += acc;
    }
}

namespace ck {

// Blocks of the Gram-Schmidt passes: 2048 rows each (eight per thread),
// which keeps the passes at full bandwidth while halving the partials the
// finish kernels sum (1024 rows per block measured the same pass times).
int64_t gm_blocks(int64_t n) {
    int64_t g = ceil_div(n, 2048);
    if (g < 1)
        g = 1;
    return g < kGmMaxBlocks ? g : kGmMaxBlocks;
}

static int64_t gm_stream_grid(int64_t n) {
    int64_t g = ceil_div(n, 1024);
    if (g < 1)
        g = 1;
    return g < 8192 ? g : 8192;
}

template <typename T>
ck_status launch_gm_cycle_start(int64_t n, const double *r64, T *v0, double *partials64,
                                GmDev<T> *st, hipStream_t s) {
    const int64_t G = gm_blocks(n);
    hipLaunchKernelGGL((gm_start_norm<T>), dim3(G), dim3(256), 0, s, n, G, r64, partials64, st);
    hipLaunchKernelGGL((gm_start_finish<T>), dim3(1), dim3(256), 0, s, G, partials64, st);
    hipLaunchKernelGGL((gm_start_v0<T>), dim3(gm_stream_grid(n)), dim3(256), 0, s, n, v0, r64, st);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

template <typename T, int NC>
static void arnoldi_nc(int64_t n, int64_t G, int j, T *V, int64_t ldv, T *w, T *partials,
                       GmDev<T> *st, hipStream_t s) {
    const int ncols = j + 1;
    if (j == 0)
        hipLaunchKernelGGL((gm_pass1<T, NC>), dim3(G), dim3(256), 0, s, n, G, ncols, V, ldv, w,
                           partials, st);
    else
        hipLaunchKernelGGL((gm_pass31<T, NC>), dim3(G), dim3(256), 0, s, n, G, j, V, ldv,
                           partials, st);
    hipLaunchKernelGGL((gm_finish_cols<T>), dim3(ncols), dim3(256), 0, s, G, partials, 1, st);
    hipLaunchKernelGGL((gm_pass2<T, NC>), dim3(G), dim3(256), 0, s, n, G, ncols, V, ldv, w,
                       partials, st);
    hipLaunchKernelGGL((gm_finish_givens<T>), dim3(1), dim3(1024), 0, s, G, partials, st);
}

// Step j after the SpMV of column j into column j+1 (column j is v_0 for
// j = 0, else the previous step's w', see the file comment): ends with
// w' of step j in column j+1 and h2, u, inv of step j in the state.
template <typename T>
ck_status launch_gm_arnoldi(int64_t n, int j, T *V, int64_t ldv, T *partials, GmDev<T> *st,
                            hipStream_t s) {
    const int64_t G = gm_blocks(n);
    const int ncols = j + 1;
    T *w = V + (int64_t)(j + 1) * ldv;
    if (ncols <= 8)
        arnoldi_nc<T, 8>(n, G, j, V, ldv, w, partials, st, s);
    else if (ncols <= 16)
        arnoldi_nc<T, 16>(n, G, j, V, ldv, w, partials, st, s);
    else if (ncols <= 24)
        arnoldi_nc<T, 24>(n, G, j, V, ldv, w, partials, st, s);
    else if (ncols <= 32)
        arnoldi_nc<T, 32>(n, G, j, V, ldv, w, partials, st, s);
    else if (ncols <= 40)
        arnoldi_nc<T, 40>(n, G, j, V, ldv, w, partials, st, s);
    else if (ncols <= 48)
        arnoldi_nc<T, 48>(n, G, j, V, ldv, w, partials, st, s);
    else if (ncols <= 56)
        arnoldi_nc<T, 56>(n, G, j, V, ldv, w, partials, st, s);
    else if (ncols <= 64)
        arnoldi_nc<T, 64>(n, G, j, V, ldv, w, partials, st, s);
    else
        return fail(CK_E_INVALID, "restart length above %d", kMaxRestart);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

template <typename T>
ck_status launch_gm_cycle_end(int64_t n, double *x, const T *V, int64_t ldv, GmDev<T> *st,
                              hipStream_t s) {
    hipLaunchKernelGGL((gm_solve_y<T>), dim3(1), dim3(64), 0, s, st);
    hipLaunchKernelGGL((gm_update_x<T>), dim3(gm_stream_grid(n)), dim3(256), 0, s, n, x, V, ldv,
                       st);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

#define CK_GM_INST(T)                                                                          \
    template ck_status launch_gm_cycle_start<T>(int64_t, const double *, T *, double *,        \
                                                GmDev<T> *, hipStream_t);                      \
    template ck_status launch_gm_arnoldi<T>(int64_t, int, T *, int64_t, T *, GmDev<T> *,       \
                                            hipStream_t);                                      \
    template ck_status launch_gm_cycle_end<T>(int64_t, double *, const T *, int64_t,           \
                                              GmDev<T> *, hipStream_t);
CK_GM_INST(double)
CK_GM_INST(float)

}  // namespace ck
