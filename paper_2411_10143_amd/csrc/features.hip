// Matrix-side kernels: CSR validation, feature extraction (feature table,
// Section III-B-1) and format conversion (Section III-C-1).
//
// Features are computed on the GPU as exact integer accumulators (integer
// atomics are associative, so the result is deterministic); the host derives
// the floating-point features from them.  Passes:
//   feat_rows : one lane per row  -> sum r, sum r^2, max r, min r, span,
//               row-length histogram                           (reads rowptr, 2 cols/row)
//   feat_nnz  : 8 lanes per row   -> longest run of consecutive columns,
//               diagonal flags, main-diagonal count, symmetry  (reads col [+ val])
//   feat_ndiag: count set diagonal flags
#include <algorithm>

#include "matrix.hpp"

namespace {

struct FeatAcc {
    unsigned long long sum_r, sum_r2, max_r, min_r, span, cluster, diag_nnz, ndiag, asym;
    unsigned long long hist[16];
};

__device__ __forceinline__ int hist_bin(long long r) {
    if (r <= 0)
        return 0;
    int b = 64 - __clzll((unsigned long long)r);   // floor(log2 r) + 1
    return b < 15 ? b : 15;
}

template <typename T>
__device__ __forceinline__ T wave_max_u64(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const T o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_min_u64(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const T o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

}  // namespace

__global__ __launch_bounds__(256) void fill_u8(int64_t n, unsigned char *__restrict__ f) {
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < n;
         d += (int64_t)gridDim.x * 256)
        f[d] = 0;
}

__global__ void feat_init(FeatAcc *acc) {
    if (threadIdx.x == 0) {
        acc->sum_r = acc->sum_r2 = acc->max_r = acc->span = acc->cluster = 0;
        acc->diag_nnz = acc->ndiag = acc->asym = 0;
        acc->min_r = ~0ull;
        for (int b = 0; b < 16; ++b)
            acc->hist[b] = 0;
    }
}

// Grid-stride over rows; each block folds its rows in registers and LDS and
// adds one value per field to the global accumulators, so no address sees
// more atomics than there are blocks.
__global__ __launch_bounds__(256) void feat_rows(int64_t n, const int *__restrict__ rp,
                                                 const int *__restrict__ col, FeatAcc *acc) {
    __shared__ unsigned long long h[16];
    __shared__ unsigned long long part[5][4];
    if (threadIdx.x < 16)
        h[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long r = 0, r2 = 0, mx = 0, mn = ~0ull, span = 0;
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
        atomicAdd(&h[hist_bin((long long)ri)], 1ull);
    }
    r = ck::wave_sum(r);
    r2 = ck::wave_sum(r2);
    span = ck::wave_sum(span);
    mx = wave_max_u64(mx);
    mn = wave_min_u64(mn);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
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
        atomicAdd(&acc->sum_r, t[0]);
        atomicAdd(&acc->sum_r2, t[1]);
        atomicAdd(&acc->span, t[2]);
        atomicMax(&acc->max_r, t[3]);
        atomicMin(&acc->min_r, t[4]);
    }
    if (threadIdx.x < 16 && h[threadIdx.x])
        atomicAdd(&acc->hist[threadIdx.x], h[threadIdx.x]);
}

// Longest run of consecutive column indices in a row, as a fold over
// contiguous chunks.  Chunk summary: len, pre (run at the chunk start),
// suf (run at the chunk end), best, first and last column.
struct Run {
    int len, pre, suf, best, first, last;
};

__device__ __forceinline__ Run run_join(const Run &A, const Run &B) {
    if (A.len == 0)
        return B;
    if (B.len == 0)
        return A;
    const bool join = B.first == A.last + 1;
    Run R;
    R.len = A.len + B.len;
    R.best = max(A.best, B.best);
    if (join)
        R.best = max(R.best, A.suf + B.pre);
    R.pre = (join && A.pre == A.len) ? A.len + B.pre : A.pre;
    R.suf = (join && B.suf == B.len) ? B.len + A.suf : B.suf;
    R.first = A.first;
    R.last = B.last;
    return R;
}

// Diagonal flags: a thread remembers the last kDiagMemo diagonals it set, so
// a banded matrix (whose k-th entry of every row lies on the same diagonal)
// touches its few flag bytes once per thread instead of once per entry; every
// other entry reads its flag before setting it.  Without this, all entries of
// a stencil matrix hammer the same few cache lines.
constexpr int kDiagMemo = 4;

template <bool SYM>
__global__ __launch_bounds__(256) void feat_nnz(int64_t n, const int *__restrict__ rp,
                                                const int *__restrict__ col,
                                                const double *__restrict__ val,
                                                unsigned char *__restrict__ diag_flag,
                                                FeatAcc *acc) {
    constexpr int L = 8;
    __shared__ unsigned long long part[3][4];
    const int lane = threadIdx.x & (L - 1);
    const int base = (threadIdx.x & 63) & ~(L - 1);
    unsigned long long dcount = 0, asym = 0, cl = 0;
    int64_t memo[kDiagMemo];
#pragma unroll
    for (int m = 0; m < kDiagMemo; ++m)
        memo[m] = -1;
    int slot = 0;
    // once any block has found an unmatched entry the answer is fixed, so
    // later blocks skip the transposed-entry searches
    const bool search = SYM && __builtin_nontemporal_load(&acc->asym) == 0;
    const int64_t groups = (n + 256 / L - 1) / (256 / L);
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int64_t i = g * (256 / L) + threadIdx.x / L;
        Run mine{0, 0, 0, 0, 0, 0};
        if (i < n) {
            const int k0 = rp[i], k1 = rp[i + 1];
            const int r = k1 - k0;
            const int chunk = (r + L - 1) / L;
            const int a = k0 + lane * chunk;
            const int e = min(k1, a + chunk);
            for (int k = a; k < e; ++k) {
                const int c = col[k];
                if (k == a) {
                    mine = Run{1, 1, 1, 1, c, c};
                } else {
                    const bool cont = c == mine.last + 1;
                    mine.suf = cont ? mine.suf + 1 : 1;
                    if (cont && mine.pre == mine.len)
                        mine.pre += 1;
                    mine.len += 1;
                    mine.best = max(mine.best, mine.suf);
                    mine.last = c;
                }
                const int64_t d = (int64_t)c - i + (n - 1);
                bool seen = false;
#pragma unroll
                for (int m = 0; m < kDiagMemo; ++m)
                    seen |= memo[m] == d;
                if (!seen) {
                    if (diag_flag[d] == 0)
                        diag_flag[d] = 1;
#pragma unroll
                    for (int m = 0; m < kDiagMemo; ++m)
                        if (m == slot)
                            memo[m] = d;
                    slot = slot + 1 == kDiagMemo ? 0 : slot + 1;
                }
                if (c == i)
                    dcount += 1;
                if (search && asym == 0) {
                    // transposed entry (c, i) must be stored with the same value
                    int lo = rp[c], hi = rp[c + 1];
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (col[mid] < (int)i)
                            lo = mid + 1;
                        else
                            hi = mid;
                    }
                    if (lo >= rp[c + 1] || col[lo] != (int)i || val[lo] != val[k])
                        asym = 1;
                }
            }
        }
        // fold the L chunk summaries of a row in lane order (lane 0 of the group)
        Run tot = mine;
#pragma unroll
        for (int t = 1; t < L; ++t) {
            Run o;
            o.len = __shfl(mine.len, base + t, 64);
            o.pre = __shfl(mine.pre, base + t, 64);
            o.suf = __shfl(mine.suf, base + t, 64);
            o.best = __shfl(mine.best, base + t, 64);
            o.first = __shfl(mine.first, base + t, 64);
            o.last = __shfl(mine.last, base + t, 64);
            tot = run_join(tot, o);
        }
        if (lane == 0 && i < n)
            cl += (unsigned long long)tot.best;
    }
    // one atomic per block and counter
    cl = ck::wave_sum(cl);
    dcount = ck::wave_sum(dcount);
    asym = ck::wave_sum(asym);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        part[0][w] = cl;
        part[1][w] = dcount;
        part[2][w] = asym;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t0 = part[0][0] + part[0][1] + part[0][2] + part[0][3];
        const unsigned long long t1 = part[1][0] + part[1][1] + part[1][2] + part[1][3];
        const unsigned long long t2 = part[2][0] + part[2][1] + part[2][2] + part[2][3];
        if (t0)
            atomicAdd(&acc->cluster, t0);
        if (t1)
            atomicAdd(&acc->diag_nnz, t1);
        if (t2)
            atomicAdd(&acc->asym, t2);
    }
}

__global__ __launch_bounds__(256) void feat_ndiag(int64_t nd, const unsigned char *__restrict__ f,
                                                  FeatAcc *acc) {
    unsigned long long c = 0;
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < nd;
         d += (int64_t)gridDim.x * 256)
        c += f[d];
    c = ck::wave_sum(c);
    if ((threadIdx.x & 63) == 0 && c)
        atomicAdd(&acc->ndiag, c);
}

// ---- validation ---------------------------------------------------------------
__global__ __launch_bounds__(256) void csr_validate(int64_t n, int64_t ncols, int64_t nnz,
                                                    const int *__restrict__ rp,
                                                    const int *__restrict__ col,
                                                    unsigned *bad) {
    constexpr int L = 8;
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
    for (int64_t k = k0 + lane; k < k1; k += L) {
        const int c = col[k];
        if (c < 0 || c >= ncols || (k > k0 && c <= col[k - 1])) {
            atomicOr(bad, 8u);
            return;
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
    r = wave_max_u64(r);
    if ((threadIdx.x & 63) == 0)
        atomicMax(out, r);
}

// ---------------------------------------------------------------------------
namespace ck {

ck_status launch_validate(int64_t n, int64_t ncols, int64_t nnz, const int *rp, const int *col,
                          unsigned *bad, hipStream_t s) {
    const int64_t G = ceil_div(n + 1, 256 / 8);
    hipLaunchKernelGGL(csr_validate, dim3(G), dim3(256), 0, s, n, ncols, nnz, rp, col, bad);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

// Fills out[0..27] with the integer accumulators in the feature layout;
// `scratch` must hold n + ncols - 1 bytes plus sizeof(FeatAcc) (+256).
int64_t features_scratch_bytes(int64_t n, int64_t ncols) {
    return ((n + ncols + 255) / 256) * 256 + 512;
}

ck_status launch_features(const ck_matrix &M, void *scratch, bool symmetry, hipStream_t s) {
    const int64_t nd = M.n + M.ncols - 1;
    unsigned char *flags = (unsigned char *)scratch;
    FeatAcc *acc = (FeatAcc *)((char *)scratch + ((M.n + M.ncols + 255) / 256) * 256);
    hipLaunchKernelGGL(feat_init, dim3(1), dim3(64), 0, s, acc);
    if (nd > 0) {
        const int64_t g = std::min<int64_t>(ceil_div(nd, 256), 8192);
        hipLaunchKernelGGL((fill_u8), dim3(g), dim3(256), 0, s, nd, flags);
    }
    if (M.n > 0) {
        hipLaunchKernelGGL(feat_rows, dim3(std::min<int64_t>(ceil_div(M.n, 256), 2048)), dim3(256),
                           0, s, M.n, M.rp, M.col, acc);
        const int64_t G = std::min<int64_t>(ceil_div(M.n, 256 / 8), 8192);
        if (symmetry && M.n == M.ncols)
            hipLaunchKernelGGL((feat_nnz<true>), dim3(G), dim3(256), 0, s, M.n, M.rp, M.col,
                               M.val, flags, acc);
        else
            hipLaunchKernelGGL((feat_nnz<false>), dim3(G), dim3(256), 0, s, M.n, M.rp, M.col,
                               M.val, flags, acc);
        const int64_t g = std::min<int64_t>(ceil_div(nd, 256), 4096);
        hipLaunchKernelGGL(feat_ndiag, dim3(g), dim3(256), 0, s, nd, flags, acc);
    }
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
