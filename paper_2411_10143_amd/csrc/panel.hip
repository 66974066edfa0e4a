// CSR-panel SpMV: an MI355X-specific CSR algorithm for matrices whose column
// pattern is scattered (the gathered vector x does not fit one XCD's L2).
//
// The GPU has 8 XCDs, each with a private 4 MB L2.  The columns are split
// into P = 8q panels whose slice of x is at most 2 MB; the matrix is stored
// panel-major (all of panel 0, row by row, then panel 1, ...), which is one
// CSR of P*n rows.  Its product runs as a merge path (spmv.hip) whose
// contiguous per-XCD block ranges give each XCD its own consecutive panels,
// so the gathers find their x slice in that XCD's L2 instead of fetching a
// cache line from the fabric for every entry.  Each panel writes its partial
// row sums; a combine kernel adds the P partials in panel order
// (deterministic) and applies alpha/beta (and the fused CG dot).
#include <algorithm>

#include "matrix.hpp"
#include "panel.hpp"
#include "solvers.hpp"


// cnt[p*n + i] = entries of row i whose column lies in panel p
__global__ __launch_bounds__(256) void panel_count(int64_t n, int P, int64_t W,
                                                   const int *__restrict__ rp,
                                                   const int *__restrict__ col,
                                                   int *__restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    const int k0 = rp[i], k1 = rp[i + 1];
    int k = k0;
    for (int p = 0; p < P; ++p) {
        const int64_t hi = (int64_t)(p + 1) * W;   // first column past panel p
        int lo = k, top = k1;                        // first entry with col >= hi
        while (lo < top) {
            const int mid = (lo + top) >> 1;
            if (col[mid] < hi)
                lo = mid + 1;
            else
                top = mid;
        }
        cnt[(int64_t)p * n + i] = lo - k;
        k = lo;
    }
}

// Panel-major copy: row i's panel-p entries go to prp[p*n + i] onwards.
// Eight lanes per row.  For panels p0 .. p0 + 7, lane l holds panel p0 + l's
// destination and length; an exclusive sum over the eight lengths gives each
// panel's first entry within the row (columns are sorted, so a row's entries
// of consecutive panels are consecutive).  The eight lanes then copy the
// row's entries of those panels together, lane l taking entries l, l + 8, ...
// (coalesced loads): an entry's panel is its column / W, and the lane holding
// that panel supplies the destination by a shuffle.  Every lane of a row runs
// the same number of steps, so the shuffles always read active lanes.
template <bool F32>
__global__ __launch_bounds__(256) void panel_fill(int64_t n, int P, int W,
                                                  const int *__restrict__ rp,
                                                  const int *__restrict__ col,
                                                  const double *__restrict__ val,
                                                  const int *__restrict__ prp,
                                                  int *__restrict__ pcol, double *__restrict__ pval,
                                                  float *__restrict__ pval32) {
    constexpr int L = 8;
    const int lane = threadIdx.x & (L - 1);
    const int64_t i = (int64_t)blockIdx.x * (256 / L) + threadIdx.x / L;
    if (i >= n)
        return;   // whole groups leave together (8 divides the wave)
    int base = rp[i];
    for (int p0 = 0; p0 < P; p0 += L) {
        // lanes past the last panel (P not a multiple of 8) hold an empty segment
        const bool has = p0 + lane < P;
        const int64_t at = (int64_t)(p0 + lane) * n + i;
        const int dst0 = has ? prp[at] : 0;
        const int len = has ? prp[at + 1] - dst0 : 0;
        int ex = len;   // inclusive scan over the group's lanes, then exclusive
#pragma unroll
        for (int off = 1; off < L; off <<= 1) {
            const int o = __shfl_up(ex, off, L);
            if (lane >= off)
                ex += o;
        }
        const int total = __shfl(ex, L - 1, L);
        ex -= len;
        for (int k0 = 0; k0 < total; k0 += L) {
            const int k = k0 + lane;
            const bool in = k < total;
            const int c = in ? col[base + k] : p0 * W;
            const int q = c / W - p0;   // 0 <= q < 8 for the row's entries of these panels
            const int d0 = __shfl(dst0, q, L);
            const int e0 = __shfl(ex, q, L);
            if (in) {
                const int dst = d0 + (k - e0);
                const double v = val[base + k];
                pcol[dst] = c;
                pval[dst] = v;
                if (F32)
                    pval32[dst] = (float)v;
            }
        }
        base += total;
    }
}

// Exclusive scan of Nin int counts into Nout >= Nin outputs (inputs past Nin
// read as 0, so out[Nin] is the total): 2048 items per workgroup, each thread
// scanning 8 consecutive items, then the 256 thread totals in order.  The
// block totals go to sums[] for the next level.
__global__ __launch_bounds__(256) void scan_blocks(int64_t Nin, int64_t Nout,
                                                   const int *__restrict__ in,
                                                   int *__restrict__ out, int *__restrict__ sums) {
    __shared__ int s[2048];
    const int64_t base = (int64_t)blockIdx.x * 2048;
    for (int t = threadIdx.x; t < 2048; t += 256)
        s[t] = base + t < Nin ? in[base + t] : 0;
    __syncthreads();
    int local[8];
    int acc = 0;
    for (int t = 0; t < 8; ++t) {
        local[t] = acc;
        acc += s[threadIdx.x * 8 + t];
    }
    __shared__ int tsum[256];
    tsum[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int t = 0; t < 256; ++t) {
            const int v = tsum[t];
            tsum[t] = run;
            run += v;
        }
        sums[blockIdx.x] = run;
    }
    __syncthreads();
    const int off = tsum[threadIdx.x];
    for (int t = 0; t < 8; ++t) {
        const int64_t g = base + threadIdx.x * 8 + t;
        if (g < Nout)
            out[g] = off + local[t];
    }
}

__global__ __launch_bounds__(256) void scan_add(int64_t N, int *__restrict__ out,
                                                const int *__restrict__ offs) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g < N)
        out[g] += offs[g / 2048];
}

// *total += number of nonzero counts (one atomic per block)
__global__ __launch_bounds__(256) void count_nonzero(int64_t N, const int *__restrict__ cnt,
                                                     unsigned long long *total) {
    unsigned long long c = 0;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < N;
         k += (int64_t)gridDim.x * 256)
        c += cnt[k] > 0 ? 1ull : 0ull;
    __shared__ unsigned long long part[4];
    c = ck::wave_sum(c);
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = part[0] + part[1] + part[2] + part[3];
        if (t)
            atomicAdd(total, t);
    }
}

// flag[k] = 1 if panel row k holds entries (in place over the counts)
__global__ __launch_bounds__(256) void panel_nonempty(int64_t N, int *__restrict__ cnt) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < N)
        cnt[k] = cnt[k] > 0 ? 1 : 0;
}

// Row list of the non-empty panel rows: panel row k = p*n + i with entries
// becomes list entry pos[k] (row i, start prp[k]); the list ends at nnz.
__global__ __launch_bounds__(256) void panel_compact(int64_t N, int64_t n, int64_t NE, int nnz,
                                                     const int *__restrict__ prp,
                                                     const int *__restrict__ pos,
                                                     int *__restrict__ prow,
                                                     int *__restrict__ prp_ne) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k == 0)
        prp_ne[NE] = nnz;
    if (k >= N)
        return;
    const int start = prp[k];
    if (prp[k + 1] > start) {
        const int j = pos[k];
        prow[j] = (int)(k % n);
        prp_ne[j] = start;
    }
}

// boff[p*(B+1) + j] = list position of panel p's first row >= 256 j (rows
// past n clamp to n, so boff[p*(B+1) + B] ends panel p)
__global__ __launch_bounds__(256) void panel_block_offsets(int64_t n, int P, int64_t B,
                                                           const int *__restrict__ pos,
                                                           int *__restrict__ boff) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)P * (B + 1))
        return;
    const int64_t p = t / (B + 1), j = t % (B + 1);
    boff[t] = pos[p * n + min(j * 256, n)];
}

// Row-list combine: workgroup row block [256 blk, 256 blk + 256) adds, panel
// by panel in order, the partials of its rows' non-empty panel rows into an
// LDS accumulator (a row appears at most once per panel, so the threads of
// one panel step never share a slot); rows absent from a panel add nothing,
// which gives the dense combine's sum bit for bit (a partial is never -0).
template <typename T, bool BETA, bool DOT>
__global__ __launch_bounds__(256) void panel_combine_rows(
    int64_t n, int P, int64_t B, int64_t G, const int *__restrict__ boff,
    const int *__restrict__ prow, const T *__restrict__ ypart, T alpha, T beta,
    T *__restrict__ y, const T *__restrict__ x, T *__restrict__ partials,
    const int *__restrict__ skip) {
    if (skip != nullptr && *skip != 0)
        return;
    const int64_t b = ck::xcd_block(G);
    if (b < 0)
        return;
    __shared__ T acc[256];
    const int tid = threadIdx.x;
    T mine = 0;
    for (int64_t blk = b; blk < B; blk += G) {
        const int64_t r0 = blk * 256;
        acc[tid] = 0;
        __syncthreads();
        for (int p = 0; p < P; ++p) {
            const int lo = boff[(int64_t)p * (B + 1) + blk];
            const int hi = boff[(int64_t)p * (B + 1) + blk + 1];
            for (int k = lo + tid; k < hi; k += 256)
                acc[prow[k] - r0] += ypart[k];
            __syncthreads();
        }
        const int64_t i = r0 + tid;
        if (i < n) {
            T out = alpha * acc[tid];
            if (BETA)
                out += beta * y[i];
            y[i] = out;
            if (DOT)
                mine += out * x[i];
        }
        __syncthreads();   // acc is cleared for the next block only after every read
    }
    if constexpr (DOT) {
        __shared__ T lds[4];
        const T d = ck::block_sum(mine, lds);
        if (threadIdx.x == 0)
            partials[b] = d;
    }
}

// y = alpha * sum_p ypart[p] + beta * y   (+ per-block partial of y.x for CG)
template <typename T, bool BETA, bool DOT>
__global__ __launch_bounds__(256) void panel_combine(int64_t n, int P, int64_t G,
                                                     const T *__restrict__ ypart, T alpha, T beta,
                                                     T *__restrict__ y, const T *__restrict__ x,
                                                     T *__restrict__ partials,
                                                     const int *__restrict__ skip) {
    if (skip != nullptr && *skip != 0)
        return;
    const int64_t b = ck::xcd_block(G);
    if (b < 0)
        return;
    T mine = 0;
    for (int64_t i = b * 256 + threadIdx.x; i < n; i += G * 256) {
        T s = 0;
        for (int p = 0; p < P; ++p)
            s += ypart[(int64_t)p * n + i];
        T out = alpha * s;
        if (BETA)
            out += beta * y[i];
        y[i] = out;
        if (DOT)
            mine += out * x[i];
    }
    if constexpr (DOT) {
        __shared__ T lds[4];
        const T d = ck::block_sum(mine, lds);
        if (threadIdx.x == 0)
            partials[b] = d;
    }
}

namespace ck {

ck_status launch_scan_exclusive(int64_t N, const int *in, int *out, int *tmp, hipStream_t s);

int panel_count_for(int64_t ncols, int value_bytes) {
    const int64_t per_panel = (2 << 20) / value_bytes;        // x slice <= 2 MB
    const int64_t q = std::max<int64_t>(1, ceil_div(ncols, 8 * per_panel));
    return (int)(8 * q);
}

// A matrix whose x fits four slices of at most 2.5 MB, whose rows are of
// even length (the longest at most four times the mean) and have entries in
// nearly every one of four panels, takes P = 4 (two XCDs share a panel): its
// partial sums, kept dense, halve while each XCD's slice still stays in its
// 4 MB L2 (uniform-random rows of 4-64 entries: 292 -> 253 us at n = 1.2M,
// 185 -> 160 us at n = 0.76M).  Short-row matrices keep P = 8: their row
// lists gain little from fewer panels and lose L2 hits (power-law n = 1.2M:
// 272 -> 304 us with P = 4); so do hub-row graphs (14-31 % slower with P = 4
// on the training graphs) and matrices with a larger x (uniform n = 2M, a
// 4 MB slice: 465 -> 483 us).
constexpr int64_t kSliceP4 = 5 * (int64_t(1) << 19);   // 2.5 MB

ck_status launch_row_max(int64_t n, const int *rp, unsigned long long *out, hipStream_t s);

ck_status panel_choose_count(const ck_matrix &M, int *tmp, hipStream_t s, int *P_out,
                             bool *counted) {
    const int P8 = panel_count_for(M.ncols, 8);
    *P_out = P8;
    *counted = false;
    if (P8 != 8 || M.n == 0 || M.ncols * 8 > 4 * kSliceP4)
        return CK_OK;
    // the longest row (known after the feature pass; else one pass over rowptr)
    int64_t max_r = M.max_row;
    if (max_r < 0) {
        unsigned long long *d = (unsigned long long *)tmp;
        unsigned long long h = 0;
        CK_TRY(launch_fill<int>(2, (int *)d, 0, s));
        CK_TRY(launch_row_max(M.n, M.rp, d, s));
        CK_HIP(hipMemcpyAsync(&h, d, sizeof h, hipMemcpyDeviceToHost, s));
        CK_HIP(hipStreamSynchronize(s));
        max_r = (int64_t)h;
    }
    if (max_r > 4 * ceil_div(M.nnz, M.n))
        return CK_OK;
    const int64_t N4 = 4 * M.n;
    const int64_t W4 = ceil_div(std::max<int64_t>(M.ncols, 1), 4);
    // counts of the four panels, then the number of non-empty panel rows;
    // the counter sits after the counts, 8-byte aligned (tmp holds >= 8n + 2 ints)
    unsigned long long *total = (unsigned long long *)(tmp + ((N4 + 1) / 2) * 2);
    CK_TRY(launch_fill<int>(2, (int *)total, 0, s));
    hipLaunchKernelGGL(panel_count, dim3(ceil_div(M.n, 256)), dim3(256), 0, s, M.n, 4, W4, M.rp,
                       M.col, tmp);
    hipLaunchKernelGGL(count_nonzero, dim3(std::min<int64_t>(ceil_div(N4, 256), 1024)), dim3(256),
                       0, s, N4, tmp, total);
    CK_HIP(hipGetLastError());
    unsigned long long ne = 0;
    CK_HIP(hipMemcpyAsync(&ne, total, sizeof ne, hipMemcpyDeviceToHost, s));
    CK_HIP(hipStreamSynchronize(s));
    if (4 * (int64_t)ne > 3 * N4) {   // the P = 4 layout would be dense
        *P_out = 4;
        *counted = true;              // tmp[0 .. 4n) holds its counts
    }
    return CK_OK;
}

int64_t panel_scan_tmp_elems(int64_t N) {
    const int64_t b1 = ceil_div(N + 1, 2048);
    const int64_t b2 = ceil_div(b1, 2048);
    return b1 + b1 + b2 + b2 + 2048 + 64;
}

// Exclusive scan of N ints (N + 1 outputs: out[N] = total), three levels.
ck_status launch_scan_exclusive(int64_t N, const int *in, int *out, int *tmp, hipStream_t s) {
    const int64_t M = N + 1;                     // in[N] is read as 0 via the bound
    const int64_t b1 = ceil_div(M, 2048);
    int *s1 = tmp, *s1x = tmp + b1;              // block sums and their scan
    const int64_t b2 = ceil_div(b1, 2048);
    int *s2 = s1x + b1, *s2x = s2 + b2;
    int *s3 = s2x + b2;
    if (b2 > 2048)
        return fail(CK_E_UNSUPPORTED, "scan too large");
    hipLaunchKernelGGL(scan_blocks, dim3(b1), dim3(256), 0, s, N, M, in, out, s1);
    hipLaunchKernelGGL(scan_blocks, dim3(b2), dim3(256), 0, s, b1, b1, s1, s1x, s2);
    hipLaunchKernelGGL(scan_blocks, dim3(1), dim3(256), 0, s, b2, b2, s2, s2x, s3);
    hipLaunchKernelGGL(scan_add, dim3(ceil_div(b1, 256)), dim3(256), 0, s, b1, s1x, s2x);
    hipLaunchKernelGGL(scan_add, dim3(ceil_div(M, 256)), dim3(256), 0, s, M, out, s1x);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

ck_status launch_to_panel(const ck_matrix &M, int P, int64_t W, int *cnt, int *tmp, int *prp,
                          int *pcol, double *pval, float *pval32, bool counted, hipStream_t s) {
    const int64_t g = ceil_div(M.n, 256);
    if (!counted)   // else cnt already holds this P's counts (panel_choose_count)
        hipLaunchKernelGGL(panel_count, dim3(g), dim3(256), 0, s, M.n, P, W, M.rp, M.col, cnt);
    CK_TRY(launch_scan_exclusive((int64_t)P * M.n, cnt, prp, tmp, s));
    const int64_t g8 = ceil_div(M.n, 256 / 8);
    const int Wi = (int)W;   // W <= ncols < 2^31
    if (pval32)
        hipLaunchKernelGGL((panel_fill<true>), dim3(g8), dim3(256), 0, s, M.n, P, Wi, M.rp,
                           M.col, M.val, prp, pcol, pval, pval32);
    else
        hipLaunchKernelGGL((panel_fill<false>), dim3(g8), dim3(256), 0, s, M.n, P, Wi, M.rp,
                           M.col, M.val, prp, pcol, pval, pval32);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

ck_status panel_make_rows(ck_matrix &M, int *cnt, hipStream_t s) {
    const int64_t n = M.n, N = (int64_t)M.panel_P * n;
    M.panel_rows = N;
    if (N == 0)
        return CK_OK;
    int *pos = nullptr;
    CK_TRY(mat_alloc(M, &pos, N + 1 + panel_scan_tmp_elems(N), s));
    hipLaunchKernelGGL(panel_nonempty, dim3(ceil_div(N, 256)), dim3(256), 0, s, N, cnt);
    ck_status st = launch_scan_exclusive(N, cnt, pos, pos + N + 1, s);
    int ne = 0;
    if (st == CK_OK && (hipMemcpyAsync(&ne, pos + N, sizeof ne, hipMemcpyDeviceToHost, s) !=
                            hipSuccess ||
                        hipStreamSynchronize(s) != hipSuccess))
        st = fail(CK_E_HIP, "panel row count read-back failed");
    const int64_t NE = ne;
    if (st != CK_OK || 4 * NE > 3 * N) {   // dense rows are cheaper (or failed)
        (void)hipStreamSynchronize(s);
        mat_free(M, pos);
        return st;
    }
    const int64_t B = ceil_div(n, 256);
    int *prow = nullptr, *prp_ne = nullptr, *boff = nullptr;
    st = mat_alloc(M, &prow, NE, s);
    if (st == CK_OK)
        st = mat_alloc(M, &prp_ne, NE + 1, s);
    if (st == CK_OK)
        st = mat_alloc(M, &boff, (int64_t)M.panel_P * (B + 1), s);
    if (st == CK_OK) {
        hipLaunchKernelGGL(panel_compact, dim3(ceil_div(N, 256)), dim3(256), 0, s, N, n, NE,
                           (int)M.nnz, M.panel_rp, pos, prow, prp_ne);
        hipLaunchKernelGGL(panel_block_offsets, dim3(ceil_div((int64_t)M.panel_P * (B + 1), 256)),
                           dim3(256), 0, s, n, M.panel_P, B, pos, boff);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            st = fail(CK_E_HIP, "panel row list failed");
    }
    (void)hipStreamSynchronize(s);
    mat_free(M, pos);
    if (st != CK_OK) {
        mat_free(M, prow);
        mat_free(M, prp_ne);
        mat_free(M, boff);
        return st;
    }
    mat_free(M, M.panel_rp);
    M.panel_rp = prp_ne;
    M.panel_row = prow;
    M.panel_boff = boff;
    M.panel_rows = NE;
    M.panel_B = B;
    return CK_OK;
}

template <typename T>
ck_status launch_panel_combine(const ck_matrix &M, const SpmvArgs<T> &a, const T *ypart,
                               int64_t G_dot, hipStream_t s) {
    const bool beta = a.beta != T(0);
    const bool dot = a.cg != nullptr;
    const int64_t G = dot ? G_dot : std::min<int64_t>(ceil_div(M.n, 256), kRowBlocks);
    const dim3 grid(xcd_grid(G));
    if (M.panel_row != nullptr) {
        const int64_t B = M.panel_B;
        if (dot)
            hipLaunchKernelGGL((panel_combine_rows<T, false, true>), grid, dim3(256), 0, s, M.n,
                               M.panel_P, B, G, M.panel_boff, M.panel_row, ypart, a.alpha, a.beta,
                               a.y, a.x, a.dot_partials, a.skip);
        else if (beta)
            hipLaunchKernelGGL((panel_combine_rows<T, true, false>), grid, dim3(256), 0, s, M.n,
                               M.panel_P, B, G, M.panel_boff, M.panel_row, ypart, a.alpha, a.beta,
                               a.y, a.x, a.dot_partials, a.skip);
        else
            hipLaunchKernelGGL((panel_combine_rows<T, false, false>), grid, dim3(256), 0, s, M.n,
                               M.panel_P, B, G, M.panel_boff, M.panel_row, ypart, a.alpha, a.beta,
                               a.y, a.x, a.dot_partials, a.skip);
        CK_HIP(hipGetLastError());
        return CK_OK;
    }
    if (dot)
        hipLaunchKernelGGL((panel_combine<T, false, true>), grid, dim3(256), 0, s, M.n, M.panel_P,
                           G, ypart, a.alpha, a.beta, a.y, a.x, a.dot_partials, a.skip);
    else if (beta)
        hipLaunchKernelGGL((panel_combine<T, true, false>), grid, dim3(256), 0, s, M.n, M.panel_P,
                           G, ypart, a.alpha, a.beta, a.y, a.x, a.dot_partials, a.skip);
    else
        hipLaunchKernelGGL((panel_combine<T, false, false>), grid, dim3(256), 0, s, M.n,
                           M.panel_P, G, ypart, a.alpha, a.beta, a.y, a.x, a.dot_partials, a.skip);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

template ck_status launch_panel_combine<double>(const ck_matrix &, const SpmvArgs<double> &,
                                                const double *, int64_t, hipStream_t);
template ck_status launch_panel_combine<float>(const ck_matrix &, const SpmvArgs<float> &,
                                               const float *, int64_t, hipStream_t);

}  // namespace ck
