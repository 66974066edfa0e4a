// SpMV kernel family for gfx950: y = alpha*A*x + beta*y.
//
// The configuration space follows the paper's (Section III-B-2): several
// storage formats, several algorithms for CSR, and a thread-count parameter
// for CSR-vector.  On MI355X the kernels are written for wave64:
//
//   spmv_csr_vector<L>  L lanes (1..64) share one row, strided over its
//                       entries; a DPP sum over the L lanes adds them
//                       (Bell & Garland's CSR-vector; the paper's TpV).
//   spmv_csr_scalar     one lane per row; the workgroup first forms the
//                       products of its 256-row block in LDS with coalesced
//                       loads, then each lane sums its row from LDS.
//   spmv_merge          merge-path load balancing (Merrill & Garland): every
//                       thread takes an equal share of the merged sequence
//                       (row ends + entries); rows cut by a thread or block
//                       boundary are completed by a deterministic carry pass.
//   spmv_ell            column-major ELLPACK, one lane per row.
//   spmv_coo            row-sorted triples, equal entry shares per thread,
//                       the same carry scheme as merge-path.
//   spmv_dia, HYB       diahyb.hip (HYB's ELL part is spmv_hyb_ell below).
//
// Matrix arrays are streamed with non-temporal loads so the cache keeps the
// gathered vector; row blocks are mapped so that each XCD works on one
// contiguous slice of rows (its L2 then holds the x entries that slice uses).
// Every reduction has a fixed order, so a configuration always returns the
// same bits for the same input.
#include "diahyb.hpp"
#include "matrix.hpp"
#include "panel.hpp"

using ck::ld_stream;

constexpr int kMergeIPT = 8;   // merged items per thread  (2048 per workgroup)
constexpr int kCooIPT = 8;     // entries per thread       (2048 per workgroup)
constexpr int kScalarCap = 4096;  // products staged per LDS chunk (CSR-scalar)

// ---------------------------------------------------------------------------
// Row-blocked kernels process row groups g = b, b+G, b+2G, ... with
// G = min(groups, kRowBlocks) logical blocks: at every step the 8 XCDs each
// cover one contiguous slice of rows, and no launch needs more workgroups
// than the dispatcher can issue in a few microseconds.
//
// Fused CG step: every block adds q_i * p_i over its rows (x = p, y = q) and
// stores its partial; the CG "sigma" finish kernel sums them in block order
// and sets alpha = rho / sigma (or flags a breakdown when sigma <= 0).
template <typename T, bool DOT>
__device__ __forceinline__ void cg_sigma_epilogue(T mine, ck::CgDev<T> *cg, T *partials,
                                                  int64_t b, int64_t G) {
    if constexpr (DOT) {
        __shared__ T lds[4];
        const T d = ck::block_sum(mine, lds);
        if (threadIdx.x == 0)
            partials[b] = d;
    }
}

__device__ __forceinline__ bool skipped(const int *skip) { return skip != nullptr && *skip != 0; }

template <int L, typename T, bool BETA, bool DOT>
__global__ __launch_bounds__(256) void spmv_csr_vector(int n, int64_t G,
                                                       const int *__restrict__ rp,
                                                       const int *__restrict__ col,
                                                       const T *__restrict__ val, T alpha,
                                                       const T *__restrict__ x, T beta,
                                                       T *__restrict__ y,
                                                       const int *__restrict__ skip,
                                                       ck::CgDev<T> *cg,
                                                       T *__restrict__ partials) {
    if (skipped(skip))
        return;
    const int64_t b = ck::xcd_block(G);
    if (b < 0)
        return;
    constexpr int R = 256 / L;
    const int lane = threadIdx.x & (L - 1);
    const int64_t groups = ((int64_t)n + R - 1) / R;
    T mine = 0;
    for (int64_t g = b; g < groups; g += G) {
        const int64_t row = g * R + threadIdx.x / L;
        T sum = 0;
        if (row < n) {
            const int k0 = rp[row], k1 = rp[row + 1];
            T s0 = 0, s1 = 0;
            int k = k0 + lane;
            for (; k + L < k1; k += 2 * L) {
                s0 += ld_stream(&val[k]) * x[ld_stream(&col[k])];
                s1 += ld_stream(&val[k + L]) * x[ld_stream(&col[k + L])];
            }
            if (k < k1)
                s0 += ld_stream(&val[k]) * x[ld_stream(&col[k])];
            sum = s0 + s1;
        }
        sum = ck::group_sum_last<L>(sum);   // valid in lane L - 1
        if (lane == L - 1 && row < n) {
            T out = alpha * sum;
            if (BETA)
                out += beta * y[row];
            y[row] = out;
            if (DOT)
                mine += out * x[row];
        }
    }
    cg_sigma_epilogue<T, DOT>(mine, cg, partials, b, G);
}

template <typename T, bool BETA, bool DOT>
__global__ __launch_bounds__(256) void spmv_csr_scalar(int n, int64_t G,
                                                       const int *__restrict__ rp,
                                                       const int *__restrict__ col,
                                                       const T *__restrict__ val, T alpha,
                                                       const T *__restrict__ x, T beta,
                                                       T *__restrict__ y,
                                                       const int *__restrict__ skip,
                                                       ck::CgDev<T> *cg,
                                                       T *__restrict__ partials) {
    __shared__ T prod[kScalarCap];
    __shared__ int srp[257];
    if (skipped(skip))
        return;
    const int64_t b = ck::xcd_block(G);
    if (b < 0)
        return;
    const int tid = threadIdx.x;
    const int64_t groups = ((int64_t)n + 255) / 256;
    T mine = 0;
    for (int64_t g = b; g < groups; g += G) {
        const int64_t r0 = g * 256;
        const int rows = (int)min<int64_t>(256, n - r0);
        __syncthreads();   // srp/prod of the previous group are no longer read
        for (int t = tid; t <= rows; t += 256)
            srp[t] = rp[r0 + t];
        __syncthreads();
        const int k0 = srp[0], k1 = srp[rows];
        const int my_lo = tid < rows ? srp[tid] : 0;
        const int my_hi = tid < rows ? srp[tid + 1] : 0;
        T acc = 0;
        for (int base = k0; base < k1; base += kScalarCap) {
            const int cnt = min(kScalarCap, k1 - base);
            // eight products per thread per step, their loads and gathers in
            // flight together (index clamped, store masked)
            for (int t0 = 0; t0 < cnt; t0 += 8 * 256) {
                int cc[8];
                T vv[8], xv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int t = min(t0 + u * 256 + tid, cnt - 1);
                    cc[u] = ld_stream(&col[base + t]);
                    vv[u] = ld_stream(&val[base + t]);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    xv[u] = x[cc[u]];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (t0 + u * 256 + tid < cnt)
                        prod[t0 + u * 256 + tid] = vv[u] * xv[u];
            }
            __syncthreads();
            const int lo = max(my_lo, base), hi = min(my_hi, base + cnt);
            for (int k = lo; k < hi; ++k)
                acc += prod[k - base];
            __syncthreads();
        }
        if (tid < rows) {
            const int64_t row = r0 + tid;
            T out = alpha * acc;
            if (BETA)
                out += beta * y[row];
            y[row] = out;
            if (DOT)
                mine += out * x[row];
        }
    }
    cg_sigma_epilogue<T, DOT>(mine, cg, partials, b, G);
}

template <typename T, bool BETA, bool DOT>
__device__ __forceinline__ void ell_rows(int n, int64_t G, int K, int64_t pitch,
                                         const int *__restrict__ ecol,
                                         const T *__restrict__ evl, T alpha,
                                         const T *__restrict__ x, T beta, T *__restrict__ y,
                                         ck::CgDev<T> *cg, T *__restrict__ partials) {
    const int64_t b = ck::xcd_block(G);
    if (b < 0)
        return;
    const int64_t groups = ((int64_t)n + 255) / 256;
    T mine = 0;
    for (int64_t g = b; g < groups; g += G) {
        const int64_t row = g * 256 + threadIdx.x;
        if (row < n) {
            // four slots per step: their column and value loads, then their x
            // gathers, are each in flight together.  Padding (column -1) only
            // trails a row, so masking it equals stopping at the first one;
            // x[0] stands in for a masked gather (K > 0 implies ncols > 0).
            constexpr int S = 4;
            T sum = 0;
            for (int s0 = 0; s0 < K; s0 += S) {
                int c[S];
                T v[S], xv[S];
#pragma unroll
                for (int u = 0; u < S; ++u) {
                    const int64_t s = min(s0 + u, K - 1);
                    c[u] = s0 + u < K ? ld_stream(&ecol[s * pitch + row]) : -1;
                    v[u] = ld_stream(&evl[s * pitch + row]);
                }
#pragma unroll
                for (int u = 0; u < S; ++u)
                    xv[u] = x[c[u] >= 0 ? c[u] : 0];
#pragma unroll
                for (int u = 0; u < S; ++u)
                    if (c[u] >= 0)
                        sum += v[u] * xv[u];
                if (c[S - 1] < 0)
                    break;
            }
            T out = alpha * sum;
            if (BETA)
                out += beta * y[row];
            y[row] = out;
            if (DOT)
                mine += out * x[row];
        }
    }
    cg_sigma_epilogue<T, DOT>(mine, cg, partials, b, G);
}

template <typename T, bool BETA, bool DOT>
__global__ __launch_bounds__(256) void spmv_ell(int n, int64_t G, int K, int64_t pitch,
                                                const int *__restrict__ ecol,
                                                const T *__restrict__ evl, T alpha,
                                                const T *__restrict__ x, T beta,
                                                T *__restrict__ y, const int *__restrict__ skip,
                                                ck::CgDev<T> *cg, T *__restrict__ partials) {
    if (skipped(skip))
        return;
    ell_rows<T, BETA, DOT>(n, G, K, pitch, ecol, evl, alpha, x, beta, y, cg, partials);
}

// The ELL part of a HYB product (its own symbol, so profiles tell it apart).
template <typename T, bool BETA>
__global__ __launch_bounds__(256) void spmv_hyb_ell(int n, int64_t G, int K, int64_t pitch,
                                                    const int *__restrict__ ecol,
                                                    const T *__restrict__ evl, T alpha,
                                                    const T *__restrict__ x, T beta,
                                                    T *__restrict__ y,
                                                    const int *__restrict__ skip) {
    if (skipped(skip))
        return;
    ell_rows<T, BETA, false>(n, G, K, pitch, ecol, evl, alpha, x, beta, y, nullptr, nullptr);
}

// ---- carry completion shared by merge-path and COO -------------------------
// Every thread passes the row it ended inside (crow, -1 if none) with its
// partial (cval), and the first row it completed (frow, -1 if none) with its
// own part of that row (fval).  Across the workgroup, equal crow values form
// one contiguous run of threads (rows only grow with the thread index).  The
// first completed row of a thread started in the run just before it: add
// that run's partials.  Thread 0 then records the block's own carry-out (the
// run ending at the last active thread) for carry_fixup.  The run sums come
// from a segmented scan: within each wave by DPP moves, then across the four
// waves through LDS, so a row spanning the whole workgroup costs a few steps
// instead of one LDS round trip per thread.
template <typename T, bool BETA>
__device__ __forceinline__ void finish_carries(int *s_crow, T *s_cval, int crow, T cval,
                                               int frow, T fval, int last_active, int64_t b,
                                               T alpha, T beta, T *__restrict__ y,
                                               int *__restrict__ crow_g,
                                               T *__restrict__ cval_g) {
    const int tid = threadIdx.x;
    s_crow[tid] = crow;
    s_cval[tid] = ck::wave_seg_scan(cval, crow);
    __syncthreads();
    // sum of the partials of the run ending at thread p: its wave's part,
    // then the runs ending each earlier wave while the run goes on
    auto run_to = [&](int p) {
        const int key = s_crow[p];
        T tot = s_cval[p];
        for (int u = (p >> 6) - 1; u >= 0; --u) {
            if (s_crow[64 * u + 63] != key)
                break;
            tot += s_cval[64 * u + 63];
            if (s_crow[64 * u] != key)
                break;
        }
        return tot;
    };
    if (frow >= 0) {
        T tot = tid > 0 && s_crow[tid - 1] == frow ? run_to(tid - 1) : T(0);
        tot += fval;
        T out = alpha * tot;
        if (BETA)
            out += beta * y[frow];
        y[frow] = out;
    }
    if (tid == 0) {
        const int R = last_active >= 0 ? s_crow[last_active] : -1;
        crow_g[b] = R;
        cval_g[b] = R >= 0 ? run_to(last_active) : T(0);
    }
}

// part[q] = merge-path row coordinate of item min(2048 q, n + nnz): the
// number of row ends among those first items (binary search on the row ends).
__global__ __launch_bounds__(256) void merge_partition(int n, int nnz, int64_t Q,
                                                       const int *__restrict__ rp,
                                                       int *__restrict__ part) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= Q)
        return;
    const int64_t d = min<int64_t>(q * 256 * kMergeIPT, (int64_t)n + nnz);
    int lo = (int)max<int64_t>(0, d - nnz), hi = (int)min<int64_t>(d, n);
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)rp[mid + 1] <= d - mid - 1)
            lo = mid + 1;
        else
            hi = mid;
    }
    part[q] = lo;
}

// Merge-path CSR.  Workgroup b owns merged items [2048 b, 2048 (b+1)) of the
// merge of the row ends rp[1..n] with the entries 0..nnz-1.  Its start and
// end coordinates come from the matrix's cached partition (built by the
// conversion to CSR-merge), else two threads search them; it then stages the
// row ends it crosses and the products val[j] * x[col[j]] of the entries it
// covers in LDS with coalesced loads (eight gathers per thread in flight), and
// every thread walks its eight items from LDS after a local merge-path search.
// Rows cut by thread boundaries are completed in LDS, rows cut by workgroup
// boundaries by carry_fixup.
template <typename T, bool BETA>
__device__ __forceinline__ void merge_rows(int n, int nnz, int64_t G, const int *__restrict__ rp,
                                           const int *__restrict__ col,
                                           const T *__restrict__ val, T alpha,
                                           const T *__restrict__ x, T beta, T *__restrict__ y,
                                           int *__restrict__ crow_g, T *__restrict__ cval_g,
                                           const int *__restrict__ part) {
    constexpr int ITEMS = 256 * kMergeIPT;
    __shared__ int s_crow[256];
    __shared__ T s_cval[256];
    __shared__ int s_rend[ITEMS + 1];   // ends of rows i0 .. i1 (local entry index + j0)
    __shared__ T s_prod[ITEMS];         // products of entries j0 .. j1-1
    __shared__ int s_coord[4];
    const int64_t b = ck::xcd_block(G);
    if (b < 0)
        return;
    const int tid = threadIdx.x;
    const int64_t P = (int64_t)n + nnz;
    const int64_t D0 = b * ITEMS;
    const int64_t D1 = min(D0 + ITEMS, P);
    if (tid < 2) {   // merge-path coordinates of D0 (thread 0) and D1 (thread 1)
        const int64_t d = tid == 0 ? D0 : D1;
        int i;
        if (part != nullptr) {   // the matrix's cached partition
            i = part[b + tid];
        } else {
            int lo = (int)max<int64_t>(0, d - nnz), hi = (int)min<int64_t>(d, n);
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if ((int64_t)rp[mid + 1] <= d - mid - 1)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            i = lo;
        }
        s_coord[2 * tid] = i;
        s_coord[2 * tid + 1] = (int)(d - i);
    }
    __syncthreads();
    const int i0 = s_coord[0], j0 = s_coord[1], i1 = s_coord[2], j1 = s_coord[3];
    const int nrows = i1 - i0 + 1;   // rows i0 .. i1 (i1 may be n)
    const int nents = j1 - j0;
    for (int t = tid; t < nrows; t += 256)
        s_rend[t] = i0 + t < n ? rp[i0 + t + 1] : nnz;
    for (int t0 = 0; t0 < nents; t0 += 256 * kMergeIPT) {
        int cc[kMergeIPT];
        T vv[kMergeIPT], xv[kMergeIPT];
#pragma unroll
        for (int u = 0; u < kMergeIPT; ++u) {
            const int t = min(t0 + u * 256 + tid, nents - 1);
            cc[u] = ld_stream(&col[j0 + t]);
            vv[u] = ld_stream(&val[j0 + t]);
        }
#pragma unroll
        for (int u = 0; u < kMergeIPT; ++u)
            xv[u] = x[cc[u]];
        __builtin_amdgcn_sched_barrier(0);   // all gathers in flight before the first use
#pragma unroll
        for (int u = 0; u < kMergeIPT; ++u)
            if (t0 + u * 256 + tid < nents)
                s_prod[t0 + u * 256 + tid] = vv[u] * xv[u];
    }
    __syncthreads();
    int crow = -1, frow = -1;
    T cval = 0, fval = 0;
    const int dl = tid * kMergeIPT;   // this thread's first local item
    if (D0 + dl < D1) {
        const int dle = (int)min<int64_t>(dl + kMergeIPT, D1 - D0);
        // local merge-path search: a = row ends among the block's first dl items
        int lo = max(0, dl - nents), hi = min(dl, nrows - 1);
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_rend[mid] - j0 <= dl - mid - 1)
                lo = mid + 1;
            else
                hi = mid;
        }
        int a = lo;
        int e = dl - lo;
        int rend = s_rend[a] - j0;
        T acc = 0;
        bool first = true;
        for (int d = dl; d < dle; ++d) {
            if (e < rend) {
                acc += s_prod[e];
                ++e;
            } else {
                const int i = i0 + a;
                if (first) {
                    frow = i;
                    fval = acc;
                    first = false;
                } else {
                    T out = alpha * acc;
                    if (BETA)
                        out += beta * y[i];
                    y[i] = out;
                }
                acc = 0;
                ++a;
                rend = s_rend[a] - j0;
            }
        }
        crow = i0 + a < n ? i0 + a : -1;
        cval = acc;
    }
    const int64_t first_d = b * 256 * kMergeIPT;
    const int last_active =
        (int)min<int64_t>(255, (P - first_d + kMergeIPT - 1) / kMergeIPT - 1);
    finish_carries<T, BETA>(s_crow, s_cval, crow, cval, frow, fval, last_active, b, alpha, beta,
                            y, crow_g, cval_g);
}

template <typename T, bool BETA>
__global__ __launch_bounds__(256) void spmv_merge(int n, int nnz, int64_t G,
                                                  const int *__restrict__ rp,
                                                  const int *__restrict__ col,
                                                  const T *__restrict__ val, T alpha,
                                                  const T *__restrict__ x, T beta,
                                                  T *__restrict__ y, int *__restrict__ crow_g,
                                                  T *__restrict__ cval_g,
                                                  const int *__restrict__ part,
                                                  const int *__restrict__ skip) {
    if (skipped(skip))
        return;
    merge_rows<T, BETA>(n, nnz, G, rp, col, val, alpha, x, beta, y, crow_g, cval_g, part);
}

// CSR-panel products: the merge path over the panel-major arrays read as one
// CSR of P*n rows, into the partial vectors (its own symbol, so profiles tell
// it apart from CSR-merge).
template <typename T>
__global__ __launch_bounds__(256) void spmv_panel_merge(int rows, int nnz, int64_t G,
                                                        const int *__restrict__ prp,
                                                        const int *__restrict__ pcol,
                                                        const T *__restrict__ pval,
                                                        const T *__restrict__ x,
                                                        T *__restrict__ ypart,
                                                        int *__restrict__ crow_g,
                                                        T *__restrict__ cval_g,
                                                        const int *__restrict__ part,
                                                        const int *__restrict__ skip) {
    if (skipped(skip))
        return;
    merge_rows<T, false>(rows, nnz, G, prp, pcol, pval, T(1), x, T(0), ypart, crow_g, cval_g,
                         part);
}

template <typename T, bool BETA>
__global__ __launch_bounds__(256) void spmv_coo(int n, int nnz, int64_t G,
                                                const int *__restrict__ row,
                                                const int *__restrict__ col,
                                                const T *__restrict__ val, T alpha,
                                                const T *__restrict__ x, T beta,
                                                T *__restrict__ y, int *__restrict__ crow_g,
                                                T *__restrict__ cval_g,
                                                const int *__restrict__ skip) {
    constexpr int ITEMS = 256 * kCooIPT;
    __shared__ int s_crow[256];
    __shared__ T s_cval[256];
    __shared__ int s_row[ITEMS + 1];   // row of entries K0 .. K0+cnt (the last: next row or n)
    __shared__ T s_prod[ITEMS];
    if (skipped(skip))
        return;
    const int64_t b = ck::xcd_block(G);
    if (b < 0)
        return;
    const int tid = threadIdx.x;
    // stage this workgroup's entries: rows and products, coalesced, with the
    // eight gathers of a thread in flight together
    const int64_t K0 = b * ITEMS;
    const int cnt = (int)min<int64_t>(ITEMS, nnz - K0);
    {
        int cc[kCooIPT];
        T vv[kCooIPT], xv[kCooIPT];
#pragma unroll
        for (int u = 0; u < kCooIPT; ++u) {
            const int t = min(u * 256 + tid, cnt - 1);
            cc[u] = ld_stream(&col[K0 + t]);
            vv[u] = ld_stream(&val[K0 + t]);
        }
#pragma unroll
        for (int u = 0; u < kCooIPT; ++u)
            xv[u] = x[cc[u]];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < kCooIPT; ++u)
            if (u * 256 + tid < cnt)
                s_prod[u * 256 + tid] = vv[u] * xv[u];
    }
    for (int t = tid; t <= cnt; t += 256)
        s_row[t] = K0 + t < nnz ? ld_stream(&row[K0 + t]) : n;
    __syncthreads();
    const int k0 = tid * kCooIPT;   // this thread's first local entry
    int crow = -1, frow = -1;
    T cval = 0, fval = 0;
    if (k0 < cnt) {
        const int k1 = min(k0 + kCooIPT, cnt);
        if (K0 + k0 == 0) {   // rows before the first stored entry are empty
            const int r_first = s_row[0];
            for (int r = 0; r < r_first; ++r)
                y[r] = BETA ? beta * y[r] : T(0);
        }
        int cur = s_row[k0];
        T acc = 0;
        bool first = true;
        for (int k = k0; k < k1; ++k) {
            acc += s_prod[k];
            const int nxt = s_row[k + 1];
            if (nxt != cur) {
                if (first) {
                    frow = cur;
                    fval = acc;
                    first = false;
                } else {
                    T out = alpha * acc;
                    if (BETA)
                        out += beta * y[cur];
                    y[cur] = out;
                }
                for (int r = cur + 1; r < nxt; ++r)   // empty rows in the gap
                    y[r] = BETA ? beta * y[r] : T(0);
                acc = 0;
                cur = nxt;
            }
        }
        if (s_row[k1] == s_row[k1 - 1]) {   // the thread ends inside a row
            crow = s_row[k1 - 1];
            cval = acc;
        }
    }
    const int64_t first_k = b * 256 * kCooIPT;
    const int last_active = (int)min<int64_t>(255, (nnz - first_k + kCooIPT - 1) / kCooIPT - 1);
    finish_carries<T, BETA>(s_crow, s_cval, crow, cval, frow, fval, last_active, b, alpha, beta,
                            y, crow_g, cval_g);
}

// Rows cut by a workgroup boundary: each run of equal carry rows is summed in
// block order by the run's first entry and added once.  The carries are read
// eight at a time (loads issued together, indexes clamped to the array), so a
// row spanning many workgroups does not wait one load latency per workgroup.
template <typename T>
__global__ __launch_bounds__(256) void carry_fixup(int64_t G, const int *__restrict__ crow,
                                                   const T *__restrict__ cval, T alpha,
                                                   T *__restrict__ y,
                                                   const int *__restrict__ skip) {
    if (skipped(skip))
        return;
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= G)
        return;
    const int R = crow[b];
    if (R < 0 || (b > 0 && crow[b - 1] == R))
        return;
    T tot = 0;
    for (int64_t e0 = b; e0 < G; e0 += 8) {
        int r[8];
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t e = min<int64_t>(e0 + u, G - 1);
            r[u] = crow[e];
            v[u] = cval[e];
        }
        bool more = true;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            more = more && e0 + u < G && r[u] == R;
            if (more)
                tot += v[u];
        }
        if (!more)
            break;
    }
    y[R] += alpha * tot;
}

template <typename T, bool BETA>
__global__ __launch_bounds__(256) void scale_rows(int64_t n, T beta, T *__restrict__ y,
                                                  const int *__restrict__ skip) {
    if (skipped(skip))
        return;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        y[i] = BETA ? beta * y[i] : T(0);
}

// ---------------------------------------------------------------------------
namespace ck {

bool config_valid(const ck_config &c) {
    if (c.format == CK_FMT_ELL || c.format == CK_FMT_COO || c.format == CK_FMT_DIA ||
        c.format == CK_FMT_HYB)
        return true;
    if (c.format != CK_FMT_CSR)
        return false;
    if (c.algorithm == CK_ALG_SCALAR || c.algorithm == CK_ALG_MERGE ||
        c.algorithm == CK_ALG_PANEL)
        return true;
    if (c.algorithm != CK_ALG_VECTOR)
        return false;
    return c.lanes >= 1 && c.lanes <= 64 && (c.lanes & (c.lanes - 1)) == 0;
}

bool spmv_fuses_dot(const ck_config &c) {
    return c.format == CK_FMT_ELL || c.format == CK_FMT_DIA ||
           (c.format == CK_FMT_CSR && (c.algorithm == CK_ALG_VECTOR ||
                                       c.algorithm == CK_ALG_SCALAR ||
                                       c.algorithm == CK_ALG_PANEL));
}

static int64_t row_groups(const ck_matrix &M, const ck_config &c) {
    if (c.format == CK_FMT_CSR && c.algorithm == CK_ALG_VECTOR)
        return ceil_div(M.n, 256 / c.lanes);
    return ceil_div(M.n, 256);
}

int64_t spmv_dot_blocks(const ck_matrix &M, const ck_config &c) {
    if (!spmv_fuses_dot(c))
        return 0;
    const int64_t g = row_groups(M, c);
    return g < kMaxPartials ? (g > 0 ? g : 1) : kMaxPartials;
}

static int64_t carry_blocks(const ck_matrix &M, const ck_config &c) {
    if (c.format == CK_FMT_COO)
        return ceil_div(M.nnz, 256 * kCooIPT);
    if (c.format == CK_FMT_CSR && c.algorithm == CK_ALG_MERGE)
        return ceil_div(M.n + M.nnz, 256 * kMergeIPT);
    return 0;
}

int64_t spmv_carry_bytes(const ck_matrix &M, const ck_config &c, bool fp32) {
    if (c.format == CK_FMT_CSR && c.algorithm == CK_ALG_PANEL) {
        // per-panel partial sums, then (merge-path panels) the carries of the
        // merge over the panel rows; sized for the dense P*n layout (an upper
        // bound: the row-list layout has fewer rows, and the size is also
        // needed before the conversion decides)
        const int64_t rows = (int64_t)panel_count_for(M.ncols, 8) * M.n;
        const int64_t Gt = ceil_div(rows + M.nnz, 256 * kMergeIPT);
        return ((rows * (fp32 ? 4 : 8) + 255) / 256) * 256 +
               ((Gt * (int64_t)sizeof(int) + 255) / 256) * 256 + Gt * (fp32 ? 4 : 8) + 256;
    }
    const int64_t G = carry_blocks(M, c);
    return ((G * (int64_t)sizeof(int) + 255) / 256) * 256 + G * (fp32 ? 4 : 8) + 256;
}

int64_t merge_part_entries_rows(int64_t rows, int64_t nnz) {
    return ceil_div(rows + nnz, 256 * kMergeIPT) + 1;
}

int64_t merge_part_entries(const ck_matrix &M) { return merge_part_entries_rows(M.n, M.nnz); }

ck_status launch_merge_partition_rows(int64_t rows, int64_t nnz, const int32_t *rp,
                                      int32_t *part, hipStream_t s) {
    const int64_t Q = merge_part_entries_rows(rows, nnz);
    hipLaunchKernelGGL(merge_partition, dim3(ceil_div(Q, 256)), dim3(256), 0, s, (int)rows,
                       (int)nnz, Q, rp, part);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

ck_status launch_merge_partition(const ck_matrix &M, int32_t *part, hipStream_t s) {
    return launch_merge_partition_rows(M.n, M.nnz, M.rp, part, s);
}

ck_config default_config(int64_t n, int64_t nnz) {
    const int64_t mean = n > 0 ? nnz / n : 0;   // floor(nnz/n) has the same floor(log2)
    int L = 1;
    while ((int64_t)L * 2 <= mean && L < 64)
        L *= 2;
    if (L < 2)
        L = 2;
    return ck_config{CK_FMT_CSR, CK_ALG_VECTOR, L, 0};
}

const char *kernel_name(const ck_config &c, bool fp32) {
    static const char *vec64[7] = {
        "spmv_csr_vector<1, double, false, false>", "spmv_csr_vector<2, double, false, false>",
        "spmv_csr_vector<4, double, false, false>", "spmv_csr_vector<8, double, false, false>",
        "spmv_csr_vector<16, double, false, false>", "spmv_csr_vector<32, double, false, false>",
        "spmv_csr_vector<64, double, false, false>"};
    static const char *vec32[7] = {
        "spmv_csr_vector<1, float, false, false>", "spmv_csr_vector<2, float, false, false>",
        "spmv_csr_vector<4, float, false, false>", "spmv_csr_vector<8, float, false, false>",
        "spmv_csr_vector<16, float, false, false>", "spmv_csr_vector<32, float, false, false>",
        "spmv_csr_vector<64, float, false, false>"};
    if (c.format == CK_FMT_ELL)
        return fp32 ? "spmv_ell<float, false, false>" : "spmv_ell<double, false, false>";
    if (c.format == CK_FMT_DIA)
        return fp32 ? "spmv_dia<float, false, false, ND>" : "spmv_dia<double, false, false, ND>";
    if (c.format == CK_FMT_HYB)
        return fp32 ? "spmv_hyb_ell<float, false>" : "spmv_hyb_ell<double, false>";
    if (c.format == CK_FMT_COO)
        return fp32 ? "spmv_coo<float, false>" : "spmv_coo<double, false>";
    if (c.algorithm == CK_ALG_SCALAR)
        return fp32 ? "spmv_csr_scalar<float, false, false>" : "spmv_csr_scalar<double, false, false>";
    if (c.algorithm == CK_ALG_MERGE)
        return fp32 ? "spmv_merge<float, false>" : "spmv_merge<double, false>";
    if (c.algorithm == CK_ALG_PANEL)
        return fp32 ? "spmv_panel_merge<float>" : "spmv_panel_merge<double>";
    int idx = 0;
    while ((1 << idx) < c.lanes)
        ++idx;
    return fp32 ? vec32[idx] : vec64[idx];
}

template <typename T>
static const T *values(const ck_matrix &M) {
    if constexpr (sizeof(T) == 4)
        return M.val32;
    else
        return M.val;
}

template <typename T>
static const T *ell_values(const ck_matrix &M) {
    if constexpr (sizeof(T) == 4)
        return M.ell_val32;
    else
        return M.ell_val;
}

template <typename T>
static const T *dia_values(const ck_matrix &M) {
    if constexpr (sizeof(T) == 4)
        return M.dia_val32;
    else
        return M.dia_val;
}

template <typename T>
static const T *hyb_values(const ck_matrix &M) {
    if constexpr (sizeof(T) == 4)
        return M.hyb_val32;
    else
        return M.hyb_val;
}

template <int L, typename T, bool BETA, bool DOT>
static void go_vector(const ck_matrix &M, int64_t G, const SpmvArgs<T> &a, hipStream_t s) {
    hipLaunchKernelGGL((spmv_csr_vector<L, T, BETA, DOT>), dim3(xcd_grid(G)), dim3(256), 0, s,
                       (int)M.n, G, M.rp, M.col, values<T>(M), a.alpha, a.x, a.beta, a.y, a.skip,
                       a.cg, a.dot_partials);
}

template <typename T, bool BETA, bool DOT>
static ck_status dispatch_rows(const ck_matrix &M, const ck_config &c, const SpmvArgs<T> &a,
                               hipStream_t s) {
    const int64_t G = std::min<int64_t>(std::max<int64_t>(row_groups(M, c), 1), kRowBlocks);
    if (c.format == CK_FMT_DIA) {
        launch_dia_spmv<T, BETA, DOT>(M, G, dia_values<T>(M), a, s);
        return CK_OK;
    }
    if (c.format == CK_FMT_HYB) {   // ELL part for every row, then the long rows' remainder
        if constexpr (DOT)
            return fail(CK_E_INVALID, "HYB does not fuse the CG dot product");
        hipLaunchKernelGGL((spmv_hyb_ell<T, BETA>), dim3(xcd_grid(G)), dim3(256), 0, s,
                           (int)M.n, G, (int)M.hyb_K, M.hyb_pitch, M.hyb_col, hyb_values<T>(M),
                           a.alpha, a.x, a.beta, a.y, a.skip);
        launch_hyb_tail<T>(M, values<T>(M), a, s);
        return CK_OK;
    }
    if (c.format == CK_FMT_ELL) {
        hipLaunchKernelGGL((spmv_ell<T, BETA, DOT>), dim3(xcd_grid(G)), dim3(256), 0, s,
                           (int)M.n, G, (int)M.ell_K, M.ell_pitch, M.ell_col, ell_values<T>(M),
                           a.alpha, a.x, a.beta, a.y, a.skip, a.cg, a.dot_partials);
        return CK_OK;
    }
    if (c.algorithm == CK_ALG_SCALAR) {
        hipLaunchKernelGGL((spmv_csr_scalar<T, BETA, DOT>), dim3(xcd_grid(G)), dim3(256), 0, s,
                           (int)M.n, G, M.rp, M.col, values<T>(M), a.alpha, a.x, a.beta, a.y,
                           a.skip, a.cg, a.dot_partials);
        return CK_OK;
    }
    switch (c.lanes) {
    case 1: go_vector<1, T, BETA, DOT>(M, G, a, s); break;
    case 2: go_vector<2, T, BETA, DOT>(M, G, a, s); break;
    case 4: go_vector<4, T, BETA, DOT>(M, G, a, s); break;
    case 8: go_vector<8, T, BETA, DOT>(M, G, a, s); break;
    case 16: go_vector<16, T, BETA, DOT>(M, G, a, s); break;
    case 32: go_vector<32, T, BETA, DOT>(M, G, a, s); break;
    case 64: go_vector<64, T, BETA, DOT>(M, G, a, s); break;
    default: return fail(CK_E_INVALID, "lanes must be a power of two in [1, 64]");
    }
    return CK_OK;
}

template <typename T, bool BETA>
static ck_status dispatch_carry(const ck_matrix &M, const ck_config &c, const SpmvArgs<T> &a,
                                hipStream_t s) {
    const int64_t G = carry_blocks(M, c);
    void *ws = a.carry;
    bool own = false;
    if (ws == nullptr) {
        CK_HIP(hipMallocAsync(&ws, (size_t)spmv_carry_bytes(M, c, sizeof(T) == 4), s));
        own = true;
    }
    int *crow = (int *)ws;
    T *cval = (T *)((char *)ws + ((G * (int64_t)sizeof(int) + 255) / 256) * 256);
    if (c.format == CK_FMT_COO)
        hipLaunchKernelGGL((spmv_coo<T, BETA>), dim3(xcd_grid(G)), dim3(256), 0, s, (int)M.n,
                           (int)M.nnz, G, M.coo_row, M.col, values<T>(M), a.alpha, a.x, a.beta,
                           a.y, crow, cval, a.skip);
    else
        hipLaunchKernelGGL((spmv_merge<T, BETA>), dim3(xcd_grid(G)), dim3(256), 0, s, (int)M.n,
                           (int)M.nnz, G, M.rp, M.col, values<T>(M), a.alpha, a.x, a.beta, a.y,
                           crow, cval, M.has_merge_part.load() ? M.merge_part : nullptr,
                           a.skip);
    hipLaunchKernelGGL((carry_fixup<T>), dim3(ceil_div(G, 256)), dim3(256), 0, s, G, crow, cval,
                       a.alpha, a.y, a.skip);
    if (own)
        CK_HIP(hipFreeAsync(ws, s));
    return CK_OK;
}

// CSR-panel: the panel-major arrays are one CSR of P*n rows (panel p's row i
// is row p*n + i), whose merge-path product writes the P partial vectors;
// panel_combine then sums them in panel order.  Logical block ranges are
// contiguous per XCD and a panel's rows are contiguous in the merged
// sequence, so each XCD works through its own consecutive panels and their x
// slices stay in its L2, while the merge balances hub rows.  (One to four
// lanes per panel row instead measured 1.3-2.7x slower: the short panel rows
// left the loads of a wave mostly idle and hub rows serialised.)
template <typename T>
static ck_status panel_merge_spmv(const ck_matrix &M, const SpmvArgs<T> &a, void *ws,
                                  int64_t G_dot, hipStream_t s) {
    const T *pv;
    if constexpr (sizeof(T) == 4)
        pv = M.panel_val32;
    else
        pv = M.panel_val;
    const int64_t rows = M.panel_rows;   // P*n, or the non-empty panel rows
    const int64_t Gt = ceil_div(rows + M.nnz, 256 * kMergeIPT);
    T *ypart = (T *)ws;
    int *crow = (int *)((char *)ws + ((rows * (int64_t)sizeof(T) + 255) / 256) * 256);
    T *cval = (T *)((char *)crow + ((Gt * (int64_t)sizeof(int) + 255) / 256) * 256);
    if (Gt > 0) {   // no panel rows at all (no entries, row-list layout): combine only
        hipLaunchKernelGGL((spmv_panel_merge<T>), dim3(xcd_grid(Gt)), dim3(256), 0, s, (int)rows,
                           (int)M.nnz, Gt, M.panel_rp, M.panel_col, pv, a.x, ypart, crow, cval,
                           M.panel_part, a.skip);
        hipLaunchKernelGGL((carry_fixup<T>), dim3(ceil_div(Gt, 256)), dim3(256), 0, s, Gt, crow,
                           cval, T(1), ypart, a.skip);
    }
    CK_HIP(hipGetLastError());
    return launch_panel_combine<T>(M, a, ypart, G_dot, s);
}

template <typename T>
ck_status launch_spmv(const ck_matrix &M, const ck_config &c, const SpmvArgs<T> &a,
                      hipStream_t s) {
    if (!config_valid(c))
        return fail(CK_E_INVALID, "invalid SpMV configuration");
    if constexpr (sizeof(T) == 4) {
        if (!M.val32)
            return fail(CK_E_INVALID, "FP32 product needs a handle created with CK_KEEP_FP32");
    }
    if (c.format == CK_FMT_ELL && !M.has_ell.load())
        return fail(CK_E_INVALID, "ELL requested but the matrix has not been converted");
    if (c.format == CK_FMT_COO && !M.has_coo.load())
        return fail(CK_E_INVALID, "COO requested but the matrix has not been converted");
    if (c.format == CK_FMT_DIA && !M.has_dia.load())
        return fail(CK_E_INVALID, "DIA requested but the matrix has not been converted");
    if (c.format == CK_FMT_HYB && !M.has_hyb.load())
        return fail(CK_E_INVALID, "HYB requested but the matrix has not been converted");
    const bool panel = c.format == CK_FMT_CSR && c.algorithm == CK_ALG_PANEL;
    if (panel && !M.has_panel.load())
        return fail(CK_E_INVALID, "CSR-panel requested but the matrix has not been converted");
    const bool beta = a.beta != T(0);
    const bool dot = a.cg != nullptr;
    if (dot && (!spmv_fuses_dot(c) || a.dot_partials == nullptr))
        return fail(CK_E_INVALID, "this configuration does not fuse the CG dot product");
    if (M.n == 0)
        return CK_OK;
    ck_status st;
    if (panel) {
        void *ws = a.carry;
        if (ws == nullptr)
            CK_HIP(hipMallocAsync(&ws, (size_t)spmv_carry_bytes(M, c, sizeof(T) == 4), s));
        st = panel_merge_spmv<T>(M, a, ws, spmv_dot_blocks(M, c), s);
        if (a.carry == nullptr)
            CK_HIP(hipFreeAsync(ws, s));
    } else if (M.nnz == 0 && !dot) {
        if (beta)
            hipLaunchKernelGGL((scale_rows<T, true>), dim3(ceil_div(M.n, 256)), dim3(256), 0, s,
                               M.n, a.beta, a.y, a.skip);
        else
            hipLaunchKernelGGL((scale_rows<T, false>), dim3(ceil_div(M.n, 256)), dim3(256), 0, s,
                               M.n, a.beta, a.y, a.skip);
        st = CK_OK;
    } else if (c.format == CK_FMT_COO || (c.format == CK_FMT_CSR && c.algorithm == CK_ALG_MERGE)) {
        st = beta ? dispatch_carry<T, true>(M, c, a, s) : dispatch_carry<T, false>(M, c, a, s);
    } else if (beta) {
        st = dot ? dispatch_rows<T, true, true>(M, c, a, s) : dispatch_rows<T, true, false>(M, c, a, s);
    } else {
        st = dot ? dispatch_rows<T, false, true>(M, c, a, s) : dispatch_rows<T, false, false>(M, c, a, s);
    }
    CK_TRY(st);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

template ck_status launch_spmv<double>(const ck_matrix &, const ck_config &,
                                       const SpmvArgs<double> &, hipStream_t);
template ck_status launch_spmv<float>(const ck_matrix &, const ck_config &,
                                      const SpmvArgs<float> &, hipStream_t);

}  // namespace ck
