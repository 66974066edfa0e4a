// Matrix-side kernels: CSR validation, feature extraction (feature table,
// Section III-B-1) and format conversion (Section III-C-1).
//
// Features are computed on the GPU as exact integer accumulators (integer
// atomics are associative, so the result is deterministic); the host derives
// the floating-point features from them.  Passes:
//   feat_rows : one lane per row  -> sum r, sum r^2, max r, min r, span,
//               row-length histogram                           (reads rowptr, 2 cols/row)
//   feat_nnz  : rows of at most kLongRow entries, 8 lanes per row striding
//               the row (coalesced) -> longest run of consecutive columns,
//               diagonal flags, main-diagonal count, symmetry  (reads col [+ val])
//   feat_long : the same for longer rows (listed by feat_rows), one
//               workgroup per row
//   feat_ndiag: count set diagonal flags
#include <algorithm>

#include "matrix.hpp"

namespace {

struct FeatAcc {
    unsigned long long sum_r, sum_r2, max_r, min_r, span, cluster, diag_nnz, ndiag, asym;
    unsigned long long hist[16];
    unsigned long long nlong;   // rows longer than kLongRow, listed by feat_rows
};

__device__ __forceinline__ int hist_bin(long long r) {
    if (r <= 0)
        return 0;
    int b = 64 - __clzll((unsigned long long)r);   // floor(log2 r) + 1
    return b < 15 ? b : 15;
}

}  // namespace

// Clears n16 16-byte words.
__global__ __launch_bounds__(256) void fill_u128(int64_t n16, uint4 *__restrict__ f) {
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < n16;
         d += (int64_t)gridDim.x * 256)
        f[d] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void feat_init(FeatAcc *acc) {
    if (threadIdx.x == 0) {
        acc->sum_r = acc->sum_r2 = acc->max_r = acc->span = acc->cluster = 0;
        acc->diag_nnz = acc->ndiag = acc->asym = acc->nlong = 0;
        acc->min_r = ~0ull;
        for (int b = 0; b < 16; ++b)
            acc->hist[b] = 0;
    }
}

// Every pass folds its block's share in registers and LDS and writes one
// slot of partial counts per block; feat_finish sums the slots (thousands of
// blocks adding to the same global counters serialised at the memory side).
// Slots are field-major (field f of block b at f * grid + b), so the finish
// reads each field coalesced.
constexpr int kRowFields = 21;   // sum r, sum r^2, span, max r, min r, histogram[16]
// Rows longer than this go to the whole-workgroup passes (feat_long,
// csr_validate_long), which take them from a list; at most nnz / 513 of them.
constexpr int kLongRow = 512;
__host__ __device__ constexpr int64_t long_list_cap(int64_t nnz) { return nnz / (kLongRow + 1) + 1; }
constexpr int kNnzFields = 2;    // longest-run sum, main-diagonal count

// Grid-stride over rows.
// The row-length histogram is counted in registers (16 counters per lane,
// summed once at the end): LDS atomics on the one bin that most rows share
// serialised every wave.
__global__ __launch_bounds__(256) void feat_rows(int64_t n, int64_t nnz,
                                                 const int *__restrict__ rp,
                                                 const int *__restrict__ col,
                                                 unsigned long long *__restrict__ part_rows,
                                                 FeatAcc *acc, int *__restrict__ long_list) {
    unsigned long long *slot = part_rows + blockIdx.x;   // field f at slot[f * gridDim.x]
    __shared__ unsigned long long h[16];
    __shared__ unsigned long long part[5][4];
    if (threadIdx.x < 16)
        h[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long r = 0, r2 = 0, mx = 0, mn = ~0ull, span = 0;
    unsigned hc[16];
#pragma unroll
    for (int b = 0; b < 16; ++b)
        hc[b] = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const int k0 = rp[i], k1 = rp[i + 1];
        const unsigned long long ri = (unsigned long long)(k1 - k0);
        r += ri;
        r2 += ri * ri;
        mx = ri > mx ? ri : mx;
        mn = ri < mn ? ri : mn;
        if (k1 > k0)
            span += (unsigned long long)(col[k1 - 1] - col[k0]);
        if (ri > (unsigned long long)kLongRow) {   // a validated CSR has at most the cap
            const unsigned long long at = atomicAdd(&acc->nlong, 1ull);
            if ((int64_t)at < long_list_cap(nnz))
                long_list[at] = (int)i;
        }
        const int bin = hist_bin((long long)ri);
#pragma unroll
        for (int b = 0; b < 16; ++b)
            hc[b] += bin == b ? 1u : 0u;
    }
#pragma unroll
    for (int b = 0; b < 16; ++b) {
        const unsigned long long t = ck::wave_sum_last((unsigned long long)hc[b]);
        if ((threadIdx.x & 63) == 63 && t)
            atomicAdd(&h[b], t);
    }
    // wave totals in lane 63 (DPP moves; integer sums, max and min are exact)
    r = ck::wave_sum_last(r);
    r2 = ck::wave_sum_last(r2);
    span = ck::wave_sum_last(span);
    mx = ck::wave_max_last(mx);
    mn = ck::wave_min_last(mn);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) {
        part[0][w] = r;
        part[1][w] = r2;
        part[2][w] = span;
        part[3][w] = mx;
        part[4][w] = mn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t[5] = {0, 0, 0, 0, ~0ull};
        for (int v = 0; v < 4; ++v) {
            t[0] += part[0][v];
            t[1] += part[1][v];
            t[2] += part[2][v];
            t[3] = part[3][v] > t[3] ? part[3][v] : t[3];
            t[4] = part[4][v] < t[4] ? part[4][v] : t[4];
        }
        for (int f = 0; f < 5; ++f)
            slot[(int64_t)f * gridDim.x] = t[f];
    }
    if (threadIdx.x < 16)
        slot[(int64_t)(5 + threadIdx.x) * gridDim.x] = h[threadIdx.x];
}

// Longest run of consecutive column indices in a row.  Entry k of a row
// "continues" when it is not the row's first and col[k] = col[k-1] + 1; the
// longest run of columns is 1 + the longest stretch of continuing entries.
// The lanes that read a step of W consecutive entries hand their continue
// bits to a wave ballot, and the stretch state (cur: continuing entries
// ending at the previous step's last entry, best: longest so far) is folded
// over the W-bit mask in entry order.
struct Stretch {
    int cur, best;
};

// longest run of set bits in x
__device__ __forceinline__ int longest_ones(unsigned long long x) {
    int len = 0;
    while (x) {
        x &= x >> 1;
        ++len;
    }
    return len;
}

// fold a step of W (<= 64) continue bits, bit j = the step's entry j
template <int W>
__device__ __forceinline__ void fold_step(Stretch &st, unsigned long long m) {
    constexpr unsigned long long full = W == 64 ? ~0ull : ((1ull << W) - 1);
    m &= full;
    if (m == full) {
        st.cur += W;
        st.best = max(st.best, st.cur);
        return;
    }
    const unsigned long long z = ~m & full;            // positions that break a stretch
    const int pre = __ffsll((long long)z) - 1;        // set bits below the first break
    const int top = 63 - __clzll(z);                   // last break
    st.best = max(st.best, st.cur + pre);
    st.best = max(st.best, longest_ones(m));
    st.cur = W - 1 - top;                              // set bits above the last break
}

// Diagonal flags: a thread remembers the last kDiagMemo diagonals it set, so
// a banded matrix (whose entries at one position of every row lie on the
// same diagonal) writes its few flag bytes once per thread instead of once
// per entry.  Other entries store their flag without reading it first (the
// value only ever goes from 0 to 1, so racing stores agree).
constexpr int kDiagMemo = 4;

struct DiagMemo {
    int64_t d[kDiagMemo];
    int slot;
    __device__ void init() {
#pragma unroll
        for (int m = 0; m < kDiagMemo; ++m)
            d[m] = -1;
        slot = 0;
    }
    __device__ __forceinline__ void mark(int64_t dg, unsigned char *__restrict__ flag) {
        bool seen = false;
#pragma unroll
        for (int m = 0; m < kDiagMemo; ++m)
            seen |= d[m] == dg;
        if (!seen) {
            flag[dg] = 1;
#pragma unroll
            for (int m = 0; m < kDiagMemo; ++m)
                if (m == slot)
                    d[m] = dg;
            slot = slot + 1 == kDiagMemo ? 0 : slot + 1;
        }
    }
};

// The stored transposed entry (c, i) with the same value, else asymmetric.
template <bool SYM>
__device__ __forceinline__ bool unmatched(int64_t i, int c, double v, const int *__restrict__ rp,
                                          const int *__restrict__ col,
                                          const double *__restrict__ val) {
    int lo = rp[c], hi = rp[c + 1];
    const int end = hi;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (col[mid] < (int)i)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo >= end || col[lo] != (int)i || val[lo] != v;
}

// The block's slot of partial counts; an unmatched transposed entry is
// flagged at once in the global accumulator (later blocks then skip the
// searches), which happens at most once per block.
__device__ __forceinline__ void add_block_counts(unsigned long long cl, unsigned long long dcount,
                                                 unsigned long long asym, FeatAcc *acc,
                                                 unsigned long long *__restrict__ slot) {
    __shared__ unsigned long long part[3][4];
    cl = ck::wave_sum_last(cl);   // wave totals in lane 63
    dcount = ck::wave_sum_last(dcount);
    asym = ck::wave_sum_last(asym);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) {
        part[0][w] = cl;
        part[1][w] = dcount;
        part[2][w] = asym;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        slot[0] = part[0][0] + part[0][1] + part[0][2] + part[0][3];
        slot[gridDim.x] = part[1][0] + part[1][1] + part[1][2] + part[1][3];
        if (part[2][0] + part[2][1] + part[2][2] + part[2][3])
            atomicAdd(&acc->asym, 1ull);
    }
}

// Rows of at most kLongRow entries: L = 8 lanes per row, lane l reading
// entries l, l + 8, ... of the row (eight consecutive columns per step,
// coalesced); the wave steps together up to its longest row.
template <bool SYM>
__global__ __launch_bounds__(256) void feat_nnz(int64_t n, const int *__restrict__ rp,
                                                const int *__restrict__ col,
                                                const double *__restrict__ val,
                                                unsigned char *__restrict__ diag_flag,
                                                FeatAcc *acc,
                                                unsigned long long *__restrict__ part_nnz) {
    constexpr int L = 8;
    const int lane = threadIdx.x & (L - 1);
    const int gbase = (threadIdx.x & 63) & ~(L - 1);   // the group's first lane in the wave
    unsigned long long dcount = 0, asym = 0, cl = 0;
    DiagMemo memo;
    memo.init();
    // once any block has found an unmatched entry the answer is fixed, so
    // later blocks skip the transposed-entry searches
    const bool search = SYM && __builtin_nontemporal_load(&acc->asym) == 0;
    const int64_t groups = (n + 256 / L - 1) / (256 / L);
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {   // uniform per block
        const int64_t i = g * (256 / L) + threadIdx.x / L;
        int k0 = 0, r = 0;
        if (i < n) {
            k0 = rp[i];
            r = rp[i + 1] - k0;
            if (r > kLongRow)
                r = 0;                      // feat_long's row
        }
        // the wave's longest row (every lane runs the steps below together,
        // so the DPP moves always read active lanes)
        const int rmax = (int)__builtin_amdgcn_readlane(
            (int)ck::wave_max_last((unsigned long long)r), 63);
        Stretch st{0, 0};
        int prev_last = 0;
        for (int t = 0; t < rmax; t += L) {
            const bool in = t + lane < r;
            const int k = k0 + t + lane;
            const int c = in ? col[k] : 0;
            // previous lane's column (row shift by 1; a group's first lane
            // takes the previous step's last column instead)
            int cprev = __builtin_amdgcn_update_dpp(0, c, 0x111, 0xf, 0xf, true);
            if (lane == 0)
                cprev = prev_last;
            const bool cont = in && t + lane > 0 && c == cprev + 1;
            const unsigned long long bal = __ballot(cont);
            fold_step<L>(st, bal >> gbase);
            // the group's last column, for its first lane (half-row mirror:
            // lane 0 of each eight reads lane 7)
            prev_last = __builtin_amdgcn_update_dpp(0, c, 0x141, 0xf, 0xf, true);
            if (in) {
                memo.mark((int64_t)c - i + (n - 1), diag_flag);
                if (c == i)
                    dcount += 1;
                if (search && asym == 0 && unmatched<SYM>(i, c, val[k], rp, col, val))
                    asym = 1;
            }
        }
        if (lane == 0 && r > 0)
            cl += (unsigned long long)(st.best + 1);
    }
    add_block_counts(cl, dcount, asym, acc, part_nnz + blockIdx.x);
}

// Rows longer than kLongRow (listed by feat_rows): a block runs each with
// all 256 lanes, lane t reading entry t of each 256-entry step; the four
// waves' continue masks are folded in wave order.

template <bool SYM>
__global__ __launch_bounds__(256) void feat_long(int64_t n, const int *__restrict__ rp,
                                                 const int *__restrict__ col,
                                                 const double *__restrict__ val,
                                                 unsigned char *__restrict__ diag_flag,
                                                 FeatAcc *acc, const int *__restrict__ long_list,
                                                 unsigned long long *__restrict__ part_long) {
    __shared__ int s_col[256];
    __shared__ unsigned long long s_mask[4];
    const int tid = threadIdx.x;
    unsigned long long dcount = 0, asym = 0, cl = 0;
    DiagMemo memo;
    memo.init();
    const bool search = SYM && __builtin_nontemporal_load(&acc->asym) == 0;
    const int64_t cnt =
        min((int64_t)__builtin_nontemporal_load(&acc->nlong), long_list_cap(rp[n]));
    for (int64_t q = blockIdx.x; q < cnt; q += gridDim.x) {
        const int64_t i = long_list[q];
        const int k0 = rp[i], r = rp[i + 1] - k0;
        Stretch st{0, 0};
        int prev_last = 0;
        for (int t = 0; t < r; t += 256) {
            const bool in = t + tid < r;
            const int k = k0 + t + tid;
            const int c = in ? col[k] : 0;
            s_col[tid] = c;
            __syncthreads();
            const int cprev = tid > 0 ? s_col[tid - 1] : prev_last;
            const bool cont = in && t + tid > 0 && c == cprev + 1;
            const unsigned long long bal = __ballot(cont);
            if ((tid & 63) == 0)
                s_mask[tid >> 6] = bal;
            if (in) {
                memo.mark((int64_t)c - i + (n - 1), diag_flag);
                if (c == i)
                    dcount += 1;
                if (search && asym == 0 && unmatched<SYM>(i, c, val[k], rp, col, val))
                    asym = 1;
            }
            __syncthreads();
            if (tid == 0)
                for (int w = 0; w < 4; ++w)
                    fold_step<64>(st, s_mask[w]);
            prev_last = s_col[255];
            __syncthreads();   // s_col and s_mask are rewritten by the next step
        }
        if (tid == 0)
            cl += (unsigned long long)(st.best + 1);
    }
    add_block_counts(cl, dcount, asym, acc, part_long + blockIdx.x);
}

// Counts the set flags, 16 bytes per lane (each byte is 0 or 1; bytes past
// the n + ncols - 1 diagonals were cleared and stay 0).
__global__ __launch_bounds__(256) void feat_ndiag(int64_t n16, const uint4 *__restrict__ f,
                                                  unsigned long long *__restrict__ part_diag) {
    unsigned long long c = 0;
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < n16;
         d += (int64_t)gridDim.x * 256) {
        const uint4 w = f[d];
        // bytes are 0/1: multiplying by 0x01010101 sums a word's four bytes into its top byte
        c += ((w.x * 0x01010101u) >> 24) + ((w.y * 0x01010101u) >> 24) +
             ((w.z * 0x01010101u) >> 24) + ((w.w * 0x01010101u) >> 24);
    }
    __shared__ unsigned long long part[4];
    c = ck::wave_sum_last(c);   // valid in lane 63
    if ((threadIdx.x & 63) == 63)
        part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0)
        part_diag[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// Sums the partial slots of every pass (integer sums, max and min: exact
// and order-free) into the accumulators.  One block of 1024 threads.
__global__ __launch_bounds__(1024) void feat_finish(FeatAcc *acc, const unsigned long long *pr,
                                                   int Gr, const unsigned long long *pn, int Gn,
                                                   const unsigned long long *pl, int Gl,
                                                   const unsigned long long *pd, int Gd) {
    constexpr int F = kRowFields + kNnzFields + 1;   // + diagonals
    unsigned long long v[F];
#pragma unroll
    for (int f = 0; f < F; ++f)
        v[f] = f == 4 ? ~0ull : 0ull;
    for (int b = threadIdx.x; b < Gr; b += 1024) {
        const unsigned long long *q = pr + b;   // field f at q[f * Gr]
        v[0] += q[0];
        v[1] += q[Gr];
        v[2] += q[2 * Gr];
        v[3] = q[3 * Gr] > v[3] ? q[3 * Gr] : v[3];
        v[4] = q[4 * Gr] < v[4] ? q[4 * Gr] : v[4];
#pragma unroll
        for (int h = 0; h < 16; ++h)
            v[5 + h] += q[(int64_t)(5 + h) * Gr];
    }
    for (int b = threadIdx.x; b < Gn; b += 1024) {
        v[21] += pn[b];
        v[22] += pn[Gn + b];
    }
    for (int b = threadIdx.x; b < Gl; b += 1024) {
        v[21] += pl[b];
        v[22] += pl[Gl + b];
    }
    for (int b = threadIdx.x; b < Gd; b += 1024)
        v[23] += pd[b];
    __shared__ unsigned long long part[F][16];
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int f = 0; f < F; ++f) {
        unsigned long long t;
        if (f == 3)   // wave results in lane 63
            t = ck::wave_max_last(v[f]);
        else if (f == 4)
            t = ck::wave_min_last(v[f]);
        else
            t = ck::wave_sum_last(v[f]);
        if ((threadIdx.x & 63) == 63)
            part[f][w] = t;
    }
    __syncthreads();
    if (threadIdx.x < F) {
        const int f = threadIdx.x;
        unsigned long long t = part[f][0];
        for (int u = 1; u < 16; ++u) {
            const unsigned long long o = part[f][u];
            t = f == 3 ? (o > t ? o : t) : f == 4 ? (o < t ? o : t) : t + o;
        }
        if (f == 0)
            acc->sum_r = t;
        else if (f == 1)
            acc->sum_r2 = t;
        else if (f == 2)
            acc->span = t;
        else if (f == 3)
            acc->max_r = t;
        else if (f == 4)
            acc->min_r = t;
        else if (f < 21)
            acc->hist[f - 5] = t;
        else if (f == 21)
            acc->cluster = t;
        else if (f == 22)
            acc->diag_nnz = t;
        else
            acc->ndiag = t;
    }
}

// ---- validation ---------------------------------------------------------------
// Row pointers (each row's bounds checked before any of its columns is
// read), then the columns of rows of at most kLongRow entries with 8 lanes
// per row; longer rows with valid bounds go to a list (valid bounds make
// the rows disjoint, so at most long_list_cap(nnz) of them) for
// csr_validate_long.  state[0] = error bits, state[1] = listed rows.
__global__ __launch_bounds__(256) void csr_validate(int64_t n, int64_t ncols, int64_t nnz,
                                                    const int *__restrict__ rp,
                                                    const int *__restrict__ col,
                                                    unsigned *state, int *__restrict__ long_list) {
    constexpr int L = 8;
    unsigned *bad = state;
    const int lane = threadIdx.x & (L - 1);
    const int64_t i = (int64_t)blockIdx.x * (256 / L) + threadIdx.x / L;
    if (i > n)
        return;
    if (i == 0 && lane == 0 && rp[0] != 0)
        atomicOr(bad, 1u);
    if (i == n) {
        if (lane == 0 && (int64_t)rp[n] != nnz)
            atomicOr(bad, 2u);
        return;
    }
    const int64_t k0 = rp[i], k1 = rp[i + 1];
    if (k1 < k0 || k0 < 0 || k1 > nnz) {
        if (lane == 0)
            atomicOr(bad, 4u);
        return;
    }
    if (k1 - k0 > kLongRow) {
        if (lane == 0) {
            // rows with valid bounds may still overlap when other rows are
            // malformed: never write past the list (those rows are flagged)
            const unsigned at = atomicAdd(&state[1], 1u);
            if ((int64_t)at < long_list_cap(nnz))
                long_list[at] = (int)i;
            else
                atomicOr(bad, 16u);
        }
        return;
    }
    for (int64_t k = k0 + lane; k < k1; k += L) {
        const int c = col[k];
        if (c < 0 || c >= ncols || (k > k0 && c <= col[k - 1])) {
            atomicOr(bad, 8u);
            return;
        }
    }
}

// Columns of the listed long rows, each with all 256 lanes of a block.
__global__ __launch_bounds__(256) void csr_validate_long(int64_t ncols, int64_t nnz,
                                                         const int *__restrict__ rp,
                                                         const int *__restrict__ col,
                                                         unsigned *state,
                                                         const int *__restrict__ long_list) {
    const int64_t cnt =
        min((int64_t)__builtin_nontemporal_load(&state[1]), long_list_cap(nnz));
    for (int64_t q = blockIdx.x; q < cnt; q += gridDim.x) {
        const int64_t i = long_list[q];
        const int64_t k0 = rp[i], k1 = rp[i + 1];
        for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) {
            const int c = col[k];
            if (c < 0 || c >= ncols || (k > k0 && c <= col[k - 1])) {
                atomicOr(&state[0], 8u);
                break;
            }
        }
    }
}

// ---- conversions ----------------------------------------------------------------
// ELL: element (s, i) at s*pitch + i; rows past n and slots past a row's
// length hold column -1, value +0.0.
template <bool F32>
__global__ __launch_bounds__(256) void csr_to_ell(int64_t n, int64_t K, int64_t pitch,
                                                  const int *__restrict__ rp,
                                                  const int *__restrict__ col,
                                                  const double *__restrict__ val,
                                                  int *__restrict__ ecol,
                                                  double *__restrict__ evl,
                                                  float *__restrict__ evl32) {
    const int64_t total = K * pitch;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        const int64_t s = idx / pitch, i = idx - s * pitch;
        int c = -1;
        double v = 0.0;
        if (i < n) {
            const int k0 = rp[i];
            if (s < rp[i + 1] - k0) {
                c = col[k0 + s];
                v = val[k0 + s];
            }
        }
        ecol[idx] = c;
        evl[idx] = v;
        if (F32)
            evl32[idx] = (float)v;
    }
}

// COO row array: row[k] = i for rowptr[i] <= k < rowptr[i+1]; 8 lanes per row.
__global__ __launch_bounds__(256) void csr_to_coo(int64_t n, const int *__restrict__ rp,
                                                  int *__restrict__ row) {
    constexpr int L = 8;
    const int lane = threadIdx.x & (L - 1);
    const int64_t i = (int64_t)blockIdx.x * (256 / L) + threadIdx.x / L;
    if (i >= n)
        return;
    const int k1 = rp[i + 1];
    for (int k = rp[i] + lane; k < k1; k += L)
        row[k] = (int)i;
}

__global__ __launch_bounds__(256) void row_max(int64_t n, const int *__restrict__ rp,
                                               unsigned long long *out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    unsigned long long r = i < n ? (unsigned long long)(rp[i + 1] - rp[i]) : 0ull;
    r = ck::wave_max_last(r);   // valid in lane 63
    if ((threadIdx.x & 63) == 63)
        atomicMax(out, r);
}

// ---------------------------------------------------------------------------
namespace ck {

// Ints of the validation state: error bits, list length, the long-row list.
int64_t validate_state_elems(int64_t nnz) { return 2 + long_list_cap(nnz); }

// `state` (validate_state_elems ints, the first two cleared) gets the error bits in state[0].
ck_status launch_validate(int64_t n, int64_t ncols, int64_t nnz, const int *rp, const int *col,
                          unsigned *state, hipStream_t s) {
    const int64_t G = ceil_div(n + 1, 256 / 8);
    int *list = (int *)(state + 2);
    hipLaunchKernelGGL(csr_validate, dim3(G), dim3(256), 0, s, n, ncols, nnz, rp, col, state, list);
    hipLaunchKernelGGL(csr_validate_long, dim3(1024), dim3(256), 0, s, ncols, nnz, rp, col, state,
                       list);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

int64_t features_acc_offset(int64_t n, int64_t ncols);

// Scratch of the feature pass: the diagonal flags (n + ncols - 1 bytes,
// rounded up to 256), the accumulators (512 bytes), then the partial slots
// of the passes (grids of at most kGridRows, kGridNnz, kGridLong and
// kGridDiag blocks).
constexpr int64_t kGridRows = 1024, kGridNnz = 2048, kGridLong = 1024, kGridDiag = 1024;
constexpr int64_t kPartialWords =
    kGridRows * kRowFields + (kGridNnz + kGridLong) * kNnzFields + kGridDiag;

int64_t features_scratch_bytes(int64_t n, int64_t ncols, int64_t nnz) {
    return ((n + ncols + 255) / 256) * 256 + 512 + 8 * kPartialWords + 4 * long_list_cap(nnz);
}

ck_status launch_features(const ck_matrix &M, void *scratch, bool symmetry, hipStream_t s) {
    // the flag bytes occupy the first features_acc_offset() bytes (a multiple
    // of 256 covering the n + ncols - 1 diagonals), all cleared and all counted
    const int64_t n16 = features_acc_offset(M.n, M.ncols) / 16;
    unsigned char *flags = (unsigned char *)scratch;
    FeatAcc *acc = (FeatAcc *)((char *)scratch + features_acc_offset(M.n, M.ncols));
    unsigned long long *pr = (unsigned long long *)((char *)acc + 512);
    unsigned long long *pn = pr + kGridRows * kRowFields;
    unsigned long long *pl = pn + kGridNnz * kNnzFields;
    unsigned long long *pd = pl + kGridLong * kNnzFields;
    int *long_list = (int *)(pd + kGridDiag);
    hipLaunchKernelGGL(feat_init, dim3(1), dim3(64), 0, s, acc);
    if (n16 > 0)
        hipLaunchKernelGGL(fill_u128, dim3(std::min<int64_t>(ceil_div(n16, 256), 4096)), dim3(256),
                           0, s, n16, (uint4 *)flags);
    if (M.n > 0) {
        const int64_t Gr = std::min<int64_t>(ceil_div(M.n, 256), kGridRows);
        const int64_t G = std::min<int64_t>(ceil_div(M.n, 256 / 8), kGridNnz);
        const int64_t GL = kGridLong;
        const int64_t Gd = std::min<int64_t>(ceil_div(n16, 256), kGridDiag);
        hipLaunchKernelGGL(feat_rows, dim3(Gr), dim3(256), 0, s, M.n, M.nnz, M.rp, M.col, pr, acc,
                           long_list);
        if (symmetry && M.n == M.ncols) {
            hipLaunchKernelGGL((feat_nnz<true>), dim3(G), dim3(256), 0, s, M.n, M.rp, M.col,
                               M.val, flags, acc, pn);
            hipLaunchKernelGGL((feat_long<true>), dim3(GL), dim3(256), 0, s, M.n, M.rp, M.col,
                               M.val, flags, acc, long_list, pl);
        } else {
            hipLaunchKernelGGL((feat_nnz<false>), dim3(G), dim3(256), 0, s, M.n, M.rp, M.col,
                               M.val, flags, acc, pn);
            hipLaunchKernelGGL((feat_long<false>), dim3(GL), dim3(256), 0, s, M.n, M.rp, M.col,
                               M.val, flags, acc, long_list, pl);
        }
        hipLaunchKernelGGL(feat_ndiag, dim3(Gd), dim3(256), 0, s, n16, (const uint4 *)flags, pd);
        hipLaunchKernelGGL(feat_finish, dim3(1), dim3(1024), 0, s, acc, pr, (int)Gr, pn, (int)G, pl,
                           (int)GL, pd, (int)Gd);
    }
    CK_HIP(hipGetLastError());
    return CK_OK;
}

// The 28 integer fields on the device (layout of ck_features' integer part;
// is_symmetric from the accumulators only when the symmetry search ran).
__global__ void feat_to_ints(const FeatAcc *acc, int64_t n, int64_t ncols, int64_t nnz,
                             int symmetry, int64_t *out) {
    if (threadIdx.x != 0)
        return;
    out[0] = n;
    out[1] = ncols;
    out[2] = nnz;
    out[3] = (int64_t)acc->sum_r;
    out[4] = (int64_t)acc->sum_r2;
    out[5] = n > 0 ? (int64_t)acc->max_r : 0;
    out[6] = n > 0 ? (int64_t)acc->min_r : 0;
    out[7] = (int64_t)acc->span;
    out[8] = (int64_t)acc->cluster;
    out[9] = (int64_t)acc->ndiag;
    out[10] = (int64_t)acc->diag_nnz;
    for (int b = 0; b < 16; ++b)
        out[11 + b] = (int64_t)acc->hist[b];
    out[27] = symmetry ? ((n == ncols && acc->asym == 0) ? 1 : 0) : -1;
}

ck_status launch_feature_ints(const ck_matrix &M, const void *scratch, bool symmetry,
                              int64_t *out28, hipStream_t s) {
    const FeatAcc *acc =
        (const FeatAcc *)((const char *)scratch + features_acc_offset(M.n, M.ncols));
    hipLaunchKernelGGL(feat_to_ints, dim3(1), dim3(64), 0, s, acc, M.n, M.ncols, M.nnz,
                       symmetry ? 1 : 0, out28);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

// Copies the accumulators into the 28 int64 of ck_features' integer part.
void features_from_acc(const void *acc_host, const ck_matrix &M, int64_t *out28) {
    const FeatAcc *a = (const FeatAcc *)acc_host;
    out28[0] = M.n;
    out28[1] = M.ncols;
    out28[2] = M.nnz;
    out28[3] = (int64_t)a->sum_r;
    out28[4] = (int64_t)a->sum_r2;
    out28[5] = M.n > 0 ? (int64_t)a->max_r : 0;
    out28[6] = M.n > 0 ? (int64_t)a->min_r : 0;
    out28[7] = (int64_t)a->span;
    out28[8] = (int64_t)a->cluster;
    out28[9] = (int64_t)a->ndiag;
    out28[10] = (int64_t)a->diag_nnz;
    for (int b = 0; b < 16; ++b)
        out28[11 + b] = (int64_t)a->hist[b];
    out28[27] = (M.n == M.ncols && a->asym == 0) ? 1 : 0;
}

int64_t features_acc_offset(int64_t n, int64_t ncols) { return ((n + ncols + 255) / 256) * 256; }
size_t features_acc_size() { return sizeof(FeatAcc); }

ck_status launch_row_max(int64_t n, const int *rp, unsigned long long *out, hipStream_t s) {
    hipLaunchKernelGGL(row_max, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, rp, out);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

ck_status launch_to_ell(const ck_matrix &M, int64_t K, int64_t pitch, int *ecol, double *evl,
                        float *evl32, hipStream_t s) {
    const int64_t total = K * pitch;
    if (total == 0)
        return CK_OK;
    const int64_t g = std::min<int64_t>(ceil_div(total, 256), 65536);
    if (evl32)
        hipLaunchKernelGGL((csr_to_ell<true>), dim3(g), dim3(256), 0, s, M.n, K, pitch, M.rp,
                           M.col, M.val, ecol, evl, evl32);
    else
        hipLaunchKernelGGL((csr_to_ell<false>), dim3(g), dim3(256), 0, s, M.n, K, pitch, M.rp,
                           M.col, M.val, ecol, evl, evl32);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

ck_status launch_to_coo(const ck_matrix &M, int *row, hipStream_t s) {
    if (M.n == 0)
        return CK_OK;
    hipLaunchKernelGGL(csr_to_coo, dim3(ceil_div(M.n, 256 / 8)), dim3(256), 0, s, M.n, M.rp, row);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

}  // namespace ck
