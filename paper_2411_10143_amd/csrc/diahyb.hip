// DIA and HYB: the two remaining formats of the paper's configuration space
// (Section III-B-2 lists COO, CSR, ELL, DIA and HYB).
//
// DIA stores every diagonal that holds an entry (offset d = column - row,
// ascending) as a dense column of `pitch` values, diagonal-major: diagonal
// k of row i at k*pitch + i, absent entries +0.0.  A product reads no column
// index at all: lane i reads value k*pitch + i (coalesced) and x[i + d]
// (coalesced, and shared by neighbouring diagonals through the cache), so a
// banded matrix moves 8 bytes per stored entry instead of CSR's 12.
//
// HYB is ELL of width K plus the remainder of the rows longer than K.  K is
// Bell and Garland's rule: the largest K such that at least a third of the
// rows have K or more entries, so every ELL slot column is at least a third
// full.  The remainder is NOT copied: it is the list of long rows, and their
// entries K.. stay in the CSR arrays.  A product runs the ELL part for every
// row (y = alpha*ell + beta*y), then adds alpha * (the row's remaining
// entries) to each long row with L lanes per row, L from the mean remainder
// length.  Each row is written by one lane of each pass, in a fixed order,
// so the result is deterministic.
#include <algorithm>
#include <climits>
#include <vector>

#include "devcache.hpp"
#include "diahyb.hpp"
#include "panel.hpp"
#include "solvers.hpp"

using ck::ld_stream;

// ---- conversions -----------------------------------------------------------

// flags[d + n - 1] = 1 for every offset d = col - row that holds an entry.
// Eight lanes per row; a flag is read before it is written, so a diagonal
// crossed by every row is stored once per cache copy instead of per entry.
__global__ __launch_bounds__(256) void dia_mark(int64_t n, const int *__restrict__ rp,
                                                const int *__restrict__ col,
                                                int *__restrict__ flags) {
    constexpr int L = 8;
    const int lane = threadIdx.x & (L - 1);
    const int64_t i = (int64_t)blockIdx.x * (256 / L) + threadIdx.x / L;
    if (i >= n)
        return;
    const int k1 = rp[i + 1];
    for (int k = rp[i] + lane; k < k1; k += L) {
        const int64_t t = (int64_t)col[k] - i + n - 1;
        if (flags[t] == 0)
            flags[t] = 1;
    }
}

// off[pos[t]] = t - (n - 1) for every flagged t (pos = exclusive scan of flags)
__global__ __launch_bounds__(256) void dia_offsets(int64_t N, int64_t n,
                                                   const int *__restrict__ flags,
                                                   const int *__restrict__ pos,
                                                   int *__restrict__ off) {
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < N;
         t += (int64_t)gridDim.x * 256)
        if (flags[t] != 0)
            off[pos[t]] = (int)(t - (n - 1));
}

// Every stored entry (i, c) goes to diagonal pos[c - i + n - 1], row i.
template <bool F32>
__global__ __launch_bounds__(256) void dia_fill(int64_t n, int64_t pitch,
                                                const int *__restrict__ rp,
                                                const int *__restrict__ col,
                                                const double *__restrict__ val,
                                                const int *__restrict__ pos,
                                                double *__restrict__ dv,
                                                float *__restrict__ dv32) {
    constexpr int L = 8;
    const int lane = threadIdx.x & (L - 1);
    const int64_t i = (int64_t)blockIdx.x * (256 / L) + threadIdx.x / L;
    if (i >= n)
        return;
    const int k1 = rp[i + 1];
    for (int k = rp[i] + lane; k < k1; k += L) {
        const int64_t at = (int64_t)pos[(int64_t)col[k] - i + n - 1] * pitch + i;
        dv[at] = val[k];
        if (F32)
            dv32[at] = (float)val[k];
    }
}

// Row-length histogram with bins 0..B-1, the last bin open-ended.  Small bin
// counts are gathered in LDS first (one global atomic per bin and block).
__global__ __launch_bounds__(256) void hyb_hist(int64_t n, int B, const int *__restrict__ rp,
                                                unsigned *__restrict__ hist) {
    constexpr int kLdsBins = 4096;
    __shared__ unsigned h[kLdsBins];
    const bool lds = B <= kLdsBins;
    if (lds) {
        for (int t = threadIdx.x; t < B; t += 256)
            h[t] = 0;
        __syncthreads();
    }
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const int r = rp[i + 1] - rp[i];
        const int bin = r < B - 1 ? r : B - 1;
        if (lds)
            atomicAdd(&h[bin], 1u);
        else
            atomicAdd(&hist[bin], 1u);
    }
    if (lds) {
        __syncthreads();
        for (int t = threadIdx.x; t < B; t += 256)
            if (h[t] != 0)
                atomicAdd(&hist[t], h[t]);
    }
}

// flag[i] = 1 if row i is longer than K
__global__ __launch_bounds__(256) void hyb_long_flags(int64_t n, int K, const int *__restrict__ rp,
                                                      int *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        flag[i] = rp[i + 1] - rp[i] > K ? 1 : 0;
}

__global__ __launch_bounds__(256) void hyb_long_rows(int64_t n, const int *__restrict__ flag,
                                                     const int *__restrict__ pos,
                                                     int *__restrict__ rows) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n && flag[i] != 0)
        rows[pos[i]] = (int)i;
}

// ---- products ----------------------------------------------------------------

// DIA: one lane per row.  ND > 0: exactly ND diagonals (the common
// stencils and block diagonals), all value and x loads in flight before the
// first use.  ND == 0:
// any count, eight diagonals per step; slots past the last diagonal repeat
// its loads (masked), which costs less than branching around them.  Columns
// outside [0, ncols) are masked, x[0] standing in for their load (nd > 0
// implies ncols > 0).
template <typename T, bool BETA, bool DOT, int ND>
__global__ __launch_bounds__(256) void spmv_dia(int n, int ncols, int64_t G, int nd,
                                                int64_t pitch, const int *__restrict__ off,
                                                const T *__restrict__ dv, T alpha,
                                                const T *__restrict__ x, T beta,
                                                T *__restrict__ y, const int *__restrict__ skip,
                                                T *__restrict__ partials) {
    if (skip != nullptr && *skip != 0)
        return;
    const int64_t b = ck::xcd_block(G);
    if (b < 0)
        return;
    const int64_t groups = ((int64_t)n + 255) / 256;
    T mine = 0;
    for (int64_t g = b; g < groups; g += G) {
        const int64_t row = g * 256 + threadIdx.x;
        if (row < n) {
            constexpr int S = ND > 0 ? ND : 8;
            const int steps = ND > 0 ? ND : nd;
            T sum = 0;
            for (int d0 = 0; d0 < steps; d0 += S) {
                T v[S], xv[S];
                bool ok[S];
#pragma unroll
                for (int u = 0; u < S; ++u) {
                    const int d = ND > 0 ? u : min(d0 + u, nd - 1);
                    const int64_t j = row + off[d];
                    ok[u] = (ND > 0 || d0 + u < nd) && j >= 0 && j < ncols;
                    v[u] = ld_stream(&dv[(int64_t)d * pitch + row]);
                    xv[u] = x[ok[u] ? j : 0];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < S; ++u)
                    if (ok[u])
                        sum += v[u] * xv[u];
            }
            T out = alpha * sum;
            if (BETA)
                out += beta * y[row];
            y[row] = out;
            if (DOT)
                mine += out * x[row];
        }
    }
    if constexpr (DOT) {
        __shared__ T lds[4];
        const T d = ck::block_sum(mine, lds);
        if (threadIdx.x == 0)
            partials[b] = d;
    }
}

// HYB remainder: L lanes per long row t, entries rp[i] + K .. rp[i+1] - 1 of
// row i = rows[t], two accumulators per lane, a DPP sum over the L lanes;
// y[i] += alpha * sum (the ELL pass has already written y[i]).
template <int L, typename T>
__global__ __launch_bounds__(256) void spmv_hyb_tail(int64_t nt, int64_t G, int K,
                                                     const int *__restrict__ rows,
                                                     const int *__restrict__ rp,
                                                     const int *__restrict__ col,
                                                     const T *__restrict__ val, T alpha,
                                                     const T *__restrict__ x, T *__restrict__ y,
                                                     const int *__restrict__ skip) {
    if (skip != nullptr && *skip != 0)
        return;
    const int64_t b = ck::xcd_block(G);
    if (b < 0)
        return;
    constexpr int R = 256 / L;
    const int lane = threadIdx.x & (L - 1);
    const int64_t groups = (nt + R - 1) / R;
    for (int64_t g = b; g < groups; g += G) {
        const int64_t t = g * R + threadIdx.x / L;
        T sum = 0;
        int i = 0;
        if (t < nt) {
            i = rows[t];
            const int k1 = rp[i + 1];
            T s0 = 0, s1 = 0;
            int k = rp[i] + K + lane;
            for (; k + L < k1; k += 2 * L) {
                s0 += ld_stream(&val[k]) * x[ld_stream(&col[k])];
                s1 += ld_stream(&val[k + L]) * x[ld_stream(&col[k + L])];
            }
            if (k < k1)
                s0 += ld_stream(&val[k]) * x[ld_stream(&col[k])];
            sum = s0 + s1;
        }
        sum = ck::group_sum_last<L>(sum);   // valid in lane L - 1
        if (lane == L - 1 && t < nt)
            y[i] += alpha * sum;
    }
}

// ---------------------------------------------------------------------------
namespace ck {

ck_status launch_to_ell(const ck_matrix &M, int64_t K, int64_t pitch, int *ecol, double *evl,
                        float *evl32, hipStream_t s);

namespace {

// Temporary device memory of one conversion, from the handle's memory
// source, given back once the conversion's stream has finished with it.
struct Tmp {
    ck_matrix &M;
    hipStream_t s;
    void *p = nullptr;
    Tmp(ck_matrix &m, hipStream_t st) : M(m), s(st) {}
    ck_status get(size_t bytes) { return mem_alloc(M.mem, &p, bytes, s); }
    ~Tmp() {
        if (p) {
            (void)hipStreamSynchronize(s);
            mat_free(M, p);
        }
    }
};

int lanes_for_mean(int64_t total, int64_t rows) {
    const int64_t mean = rows > 0 ? total / rows : 0;
    int L = 1;
    while ((int64_t)L * 2 <= mean && L < 64)
        L *= 2;
    return L;
}

}  // namespace

ck_status convert_to_dia(ck_matrix &M, hipStream_t s) {
    const int64_t n = M.n, pitch = ceil_div(n, 64) * 64;
    int64_t nd = 0;
    Tmp tmp(M, s);
    int *flags = nullptr, *pos = nullptr;
    const int64_t N = n + M.ncols - 1;   // offsets -(n-1) .. ncols-1
    if (n > 0 && M.nnz > 0) {
        const int64_t scan_tmp = panel_scan_tmp_elems(N);
        CK_TRY(tmp.get((size_t)(2 * N + 1 + scan_tmp) * sizeof(int)));
        flags = (int *)tmp.p;
        pos = flags + N;
        CK_TRY(launch_fill<int>(N, flags, 0, s));
        hipLaunchKernelGGL(dia_mark, dim3(ceil_div(n, 256 / 8)), dim3(256), 0, s, n, M.rp, M.col,
                           flags);
        CK_TRY(launch_scan_exclusive(N, flags, pos, pos + N + 1, s));
        int total = 0;
        CK_HIP(hipMemcpyAsync(&total, pos + N, sizeof total, hipMemcpyDeviceToHost, s));
        CK_HIP(hipStreamSynchronize(s));
        nd = total;
    }
    if (nd * pitch > 8 * M.nnz)
        return fail(CK_E_UNSUPPORTED, "DIA refused: %lld diagonals x %lld rows for %lld entries",
                    (long long)nd, (long long)pitch, (long long)M.nnz);
    CK_TRY(mat_alloc(M, &M.dia_off, nd, s));
    CK_TRY(mat_alloc(M, &M.dia_val, nd * pitch, s));
    if (M.val32)
        CK_TRY(mat_alloc(M, &M.dia_val32, nd * pitch, s));
    if (nd > 0) {
        hipLaunchKernelGGL(dia_offsets, dim3(std::min<int64_t>(ceil_div(N, 256), 8192)), dim3(256),
                           0, s, N, n, flags, pos, M.dia_off);
        CK_TRY(launch_fill<double>(nd * pitch, M.dia_val, 0.0, s));
        if (M.val32) {
            CK_TRY(launch_fill<float>(nd * pitch, M.dia_val32, 0.0f, s));
            hipLaunchKernelGGL((dia_fill<true>), dim3(ceil_div(n, 256 / 8)), dim3(256), 0, s, n,
                               pitch, M.rp, M.col, M.val, pos, M.dia_val, M.dia_val32);
        } else {
            hipLaunchKernelGGL((dia_fill<false>), dim3(ceil_div(n, 256 / 8)), dim3(256), 0, s, n,
                               pitch, M.rp, M.col, M.val, pos, M.dia_val, M.dia_val32);
        }
    }
    CK_HIP(hipGetLastError());
    M.dia_nd = nd;
    M.dia_pitch = pitch;
    return CK_OK;
}

ck_status convert_to_hyb(ck_matrix &M, hipStream_t s) {
    const int64_t n = M.n, pitch = ceil_div(n, 64) * 64;
    int64_t K = 0, nt = 0, tail_nnz = 0;
    if (n > 0) {
        // K <= 3 nnz / n: the K-or-longer rows (>= n/3 of them) hold >= K n / 3
        // entries.  Bins 0..Kcap, the last one open-ended, decide every k <= Kcap.
        const int64_t Kcap = 3 * M.nnz / n + 1;
        if (Kcap + 1 > (int64_t)INT_MAX)
            return fail(CK_E_UNSUPPORTED, "HYB: rows too long");
        const int B = (int)(Kcap + 1);
        Tmp tmp(M, s);
        CK_TRY(tmp.get((size_t)B * sizeof(unsigned)));
        unsigned *hist = (unsigned *)tmp.p;
        CK_TRY(launch_fill<int>(B, (int *)hist, 0, s));
        hipLaunchKernelGGL(hyb_hist, dim3(std::min<int64_t>(ceil_div(n, 256), 2048)), dim3(256), 0,
                           s, n, B, M.rp, hist);
        CK_HIP(hipGetLastError());
        std::vector<unsigned> h(B);
        CK_HIP(hipMemcpyAsync(h.data(), hist, (size_t)B * sizeof(unsigned), hipMemcpyDeviceToHost, s));
        CK_HIP(hipStreamSynchronize(s));
        std::vector<int64_t> ge(B + 1, 0);   // ge[k] = rows with length >= k
        for (int k = B - 1; k >= 0; --k)
            ge[k] = ge[k + 1] + h[k];
        for (int64_t k = 1; k <= Kcap; ++k) {
            if (ge[k] == 0 || 3 * ge[k] < n)
                break;
            K = k;
        }
        int64_t ell_entries = 0;
        for (int j = 0; j < B; ++j)
            ell_entries += (int64_t)h[j] * std::min<int64_t>(j, K);
        tail_nnz = M.nnz - ell_entries;
        nt = ge[K + 1];
    }
    CK_TRY(mat_alloc(M, &M.hyb_col, K * pitch, s));
    CK_TRY(mat_alloc(M, &M.hyb_val, K * pitch, s));
    if (M.val32)
        CK_TRY(mat_alloc(M, &M.hyb_val32, K * pitch, s));
    CK_TRY(mat_alloc(M, &M.hyb_rows, nt, s));
    CK_TRY(launch_to_ell(M, K, pitch, M.hyb_col, M.hyb_val, M.hyb_val32, s));
    if (nt > 0) {
        Tmp tmp(M, s);
        const int64_t scan_tmp = panel_scan_tmp_elems(n);
        CK_TRY(tmp.get((size_t)(2 * n + 1 + scan_tmp) * sizeof(int)));
        int *flag = (int *)tmp.p, *pos = flag + n;
        hipLaunchKernelGGL(hyb_long_flags, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, (int)K,
                           M.rp, flag);
        CK_TRY(launch_scan_exclusive(n, flag, pos, pos + n + 1, s));
        hipLaunchKernelGGL(hyb_long_rows, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, flag, pos,
                           M.hyb_rows);
    }
    CK_HIP(hipGetLastError());
    M.hyb_K = K;
    M.hyb_pitch = pitch;
    M.hyb_nt = nt;
    M.hyb_L = lanes_for_mean(tail_nnz, nt);
    return CK_OK;
}

template <typename T, bool BETA, bool DOT>
void launch_dia_spmv(const ck_matrix &M, int64_t G, const T *dv, const SpmvArgs<T> &a,
                     hipStream_t s) {
    const int nd = (int)M.dia_nd;
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(xcd_grid(G)), dim3(256), 0, s, (int)M.n, (int)M.ncols, G,
                           nd, M.dia_pitch, M.dia_off, dv, a.alpha, a.x, a.beta, a.y, a.skip,
                           a.dot_partials);
    };
    switch (nd) {   // stencils (2D: 3, 5, 9 points; 3D: 7, 13, 19, 27) and 8-wide blocks (15)
    case 3: go(spmv_dia<T, BETA, DOT, 3>); break;
    case 5: go(spmv_dia<T, BETA, DOT, 5>); break;
    case 7: go(spmv_dia<T, BETA, DOT, 7>); break;
    case 9: go(spmv_dia<T, BETA, DOT, 9>); break;
    case 13: go(spmv_dia<T, BETA, DOT, 13>); break;
    case 15: go(spmv_dia<T, BETA, DOT, 15>); break;
    case 19: go(spmv_dia<T, BETA, DOT, 19>); break;
    case 27: go(spmv_dia<T, BETA, DOT, 27>); break;
    default: go(spmv_dia<T, BETA, DOT, 0>); break;
    }
}

template <int L, typename T>
static void go_tail(const ck_matrix &M, const T *val, const SpmvArgs<T> &a, hipStream_t s) {
    const int64_t groups = ceil_div(M.hyb_nt, 256 / L);
    const int64_t G = std::min<int64_t>(std::max<int64_t>(groups, 1), kRowBlocks);
    hipLaunchKernelGGL((spmv_hyb_tail<L, T>), dim3(xcd_grid(G)), dim3(256), 0, s, M.hyb_nt, G,
                       (int)M.hyb_K, M.hyb_rows, M.rp, M.col, val, a.alpha, a.x, a.y, a.skip);
}

template <typename T>
void launch_hyb_tail(const ck_matrix &M, const T *val, const SpmvArgs<T> &a, hipStream_t s) {
    if (M.hyb_nt == 0)
        return;
    switch (M.hyb_L) {
    case 1: go_tail<1, T>(M, val, a, s); break;
    case 2: go_tail<2, T>(M, val, a, s); break;
    case 4: go_tail<4, T>(M, val, a, s); break;
    case 8: go_tail<8, T>(M, val, a, s); break;
    case 16: go_tail<16, T>(M, val, a, s); break;
    case 32: go_tail<32, T>(M, val, a, s); break;
    default: go_tail<64, T>(M, val, a, s); break;
    }
}

#define CK_DIA_INST(T, B, D)                                                               \
    template void launch_dia_spmv<T, B, D>(const ck_matrix &, int64_t, const T *,          \
                                           const SpmvArgs<T> &, hipStream_t);
CK_DIA_INST(double, false, false)
CK_DIA_INST(double, false, true)
CK_DIA_INST(double, true, false)
CK_DIA_INST(double, true, true)
CK_DIA_INST(float, false, false)
CK_DIA_INST(float, false, true)
CK_DIA_INST(float, true, false)
CK_DIA_INST(float, true, true)
template void launch_hyb_tail<double>(const ck_matrix &, const double *, const SpmvArgs<double> &,
                                      hipStream_t);
template void launch_hyb_tail<float>(const ck_matrix &, const float *, const SpmvArgs<float> &,
                                     hipStream_t);

}  // namespace ck
