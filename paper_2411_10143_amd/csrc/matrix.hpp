// Device-resident matrix store and the internal launch interface of the SpMV
// kernel family.
#pragma once

#include <atomic>
#include <map>
#include <mutex>

#include "devcache.hpp"
#include "krylov.hpp"

struct ck_matrix {
    int64_t n = 0, ncols = 0, nnz = 0;
    int device = 0;
    uint32_t flags = 0;
    // CSR (always present)
    int32_t *rp = nullptr;
    int32_t *col = nullptr;
    double *val = nullptr;
    float *val32 = nullptr;           // CK_KEEP_FP32
    // ELL (after conversion): column-major, slot s of row i at s*pitch + i
    int32_t *ell_col = nullptr;
    double *ell_val = nullptr;
    float *ell_val32 = nullptr;
    int64_t ell_K = 0, ell_pitch = 0;
    std::atomic<bool> has_ell{false};
    // COO (after conversion): row index per stored entry; col/val shared with CSR
    int32_t *coo_row = nullptr;
    std::atomic<bool> has_coo{false};
    // CSR-panel (after conversion): P column panels of width W, panel-major.
    // Dense layout (panel_row == nullptr): panel_rows = P*n, panel_rp[p*n + i]
    // = start of row i in panel p.  Row-list layout: only the panel_rows
    // non-empty panel rows, in panel-major order; panel_row[k] = the matrix
    // row of panel row k, panel_rp[k] its start, and panel_boff[p*(B+1) + j]
    // = the first panel row of panel p whose row is >= 256 j (B = ceil(n/256))
    int panel_P = 0;
    int64_t panel_W = 0;
    int64_t panel_rows = 0;
    int64_t panel_B = 0;
    int32_t *panel_row = nullptr;
    int32_t *panel_boff = nullptr;
    int32_t *panel_rp = nullptr;
    int32_t *panel_col = nullptr;
    double *panel_val = nullptr;
    float *panel_val32 = nullptr;
    std::atomic<bool> has_panel{false};
    // merge-path partition of the panel-major arrays read as one CSR of P*n rows
    int32_t *panel_part = nullptr;
    // merge-path partition (after conversion to CSR-merge): merge_part[q] =
    // rows whose end lies among the first min(2048 q, n + nnz) merged items
    int32_t *merge_part = nullptr;
    std::atomic<bool> has_merge_part{false};
    // DIA (after conversion): dia_nd offsets (col - row, ascending), values
    // diagonal-major: diagonal k of row i at k*dia_pitch + i, absent = +0.0
    int32_t *dia_off = nullptr;
    double *dia_val = nullptr;
    float *dia_val32 = nullptr;
    int64_t dia_nd = 0, dia_pitch = 0;
    std::atomic<bool> has_dia{false};
    // HYB (after conversion): ELL part of width hyb_K (layout as ELL) and the
    // hyb_nt rows longer than hyb_K, ascending; their entries hyb_K.. stay in
    // the CSR arrays and are summed with hyb_L lanes per row
    int32_t *hyb_col = nullptr;
    double *hyb_val = nullptr;
    float *hyb_val32 = nullptr;
    int32_t *hyb_rows = nullptr;
    int64_t hyb_K = 0, hyb_pitch = 0, hyb_nt = 0;
    int hyb_L = 1;
    std::atomic<bool> has_hyb{false};
    int64_t max_row = -1;             // longest row, once known
    // feature scratch of the device-resident cascade (kept with the handle)
    char *devsel_scratch = nullptr;
    int64_t *devsel_ints = nullptr;
    ck_config active{};
    std::mutex mu;                    // guards conversions, `active` and `carry`
    ck::MemSource mem;                // where every device block of the handle comes from
    // merge-path / COO carry workspace of spmv_apply, one per stream (work on
    // one stream is ordered, so reuse on that stream is safe)
    std::map<hipStream_t, void *> carry;
};

namespace ck {

// A block of `count` T for handle M, allocated for use on stream s.
template <typename T>
ck_status mat_alloc(ck_matrix &M, T **p, int64_t count, hipStream_t s) {
    void *q = nullptr;
    const ck_status st = mem_alloc(M.mem, &q, (size_t)(count > 0 ? count : 1) * sizeof(T), s);
    *p = (T *)q;
    return st;
}
inline void mat_free(ck_matrix &M, void *p) { mem_free(M.mem, p); }

// Arguments of one product y = alpha*A*x + beta*y.
//  skip   : if non-null and *skip != 0 when the launch starts, it does nothing
//           (lets a solver enqueue iterations ahead of its convergence test).
//  cg     : fused CG step (only where spmv_fuses_dot() holds): the launch also
//           forms sigma = y.x (x = p, y = q = A p) and its last block sets
//           alpha = rho/sigma, or state = BREAKDOWN when sigma <= 0.
//           dot_partials needs spmv_dot_blocks() entries.
//  carry  : workspace of spmv_carry_bytes() for merge-path and COO carries
//           and CSR-panel partial sums; when null the launch allocates it
//           stream-ordered.
template <typename T>
struct SpmvArgs {
    T alpha = 1, beta = 0;
    const T *x = nullptr;
    T *y = nullptr;
    const int *skip = nullptr;
    CgDev<T> *cg = nullptr;
    T *dot_partials = nullptr;
    void *carry = nullptr;
};

bool config_valid(const ck_config &c);
bool spmv_fuses_dot(const ck_config &c);
// Number of dot partials a fused launch writes (0 if not fused; <= kMaxPartials).
int64_t spmv_dot_blocks(const ck_matrix &M, const ck_config &c);
// Bytes of carry workspace a launch needs (0 if none).
int64_t spmv_carry_bytes(const ck_matrix &M, const ck_config &c, bool fp32);
// Merge-path partition: entries of merge_part, and its launch (stream-ordered).
int64_t merge_part_entries(const ck_matrix &M);
ck_status launch_merge_partition(const ck_matrix &M, int32_t *part, hipStream_t s);
// The same for any CSR of `rows` rows (used for the panel-major arrays).
int64_t merge_part_entries_rows(int64_t rows, int64_t nnz);
ck_status launch_merge_partition_rows(int64_t rows, int64_t nnz, const int32_t *rp,
                                      int32_t *part, hipStream_t s);

template <typename T>
ck_status launch_spmv(const ck_matrix &M, const ck_config &c, const SpmvArgs<T> &a,
                      hipStream_t s);

// Deterministic two-stage reductions (vecops.hip)
template <typename T>
int64_t dot_blocks(int64_t n);
template <typename T>
ck_status launch_dot_partials(int64_t n, const T *x, const T *y, T *partials, hipStream_t s);

const char *kernel_name(const ck_config &c, bool fp32);
ck_config default_config(int64_t n, int64_t nnz);

}  // namespace ck
