// Slot record of the batched small-system solver (device memory, one per slot).
#pragma once

#include "krylov.hpp"

namespace ck {

constexpr int kBMaxM = 32;            // largest GMRES restart in the batched path
enum : int { B_CG = 0, B_GMRES = 1 };
enum : int { B_OUTER = 0, B_INNER = 1, B_UPDATE = 2, B_DONE = 3 };

struct BSlot {
    // problem, set at admission
    int kind, n, lanes, m;
    const int *rp;
    const int *col;
    const double *val64;
    const float *val32;
    const double *b;
    double *x;            // caller's solution vector (holds x0 on admission)
    double *r64;          // FP64 residual
    void *work;           // inner vectors: CG r,p,q,d; GMRES basis (m+1 columns)
    int64_t ld;           // length of one inner vector (n rounded up to 64)
    double bnorm, tol;
    int max_iter, inner_cap;
    int keep_x0;          // 1: start from the x given; 0: start from x = 0
    int pad0;
    // state
    int phase, status, iter, outer, inner_iter, j, launches, pad;
    double beta, relres, inner_tol, rho;
    // Hessenberg least squares (values held in the inner precision)
    double H[(kBMaxM + 1) * kBMaxM];
    double cs[kBMaxM], sn[kBMaxM], g[kBMaxM + 1], y[kBMaxM];
};

// Compact per-slot status written at the end of every launch (read by the host)
struct BStat {
    int phase, status, iter, outer;
    double relres;
};

// Single-workgroup FP64 CG (one launch per solve) for at most kWgCgMaxN rows.
constexpr int kWgCgMaxN = 4096;
struct WgCgOut {
    int status, iter, restarts, pad;
    double relres;   // true relative residual at exit
};
// When the longest row has 6 to this many entries (even), the matrix is
// copied column-major once per solve into cm_col / cm_val: kWgCgColMajorK *
// kWgCgMaxN ints and doubles, 16-byte aligned (rows of at most 5 entries are
// held in registers instead, and longer ones read in place).
constexpr int kWgCgColMajorK = 16;
ck_status launch_cg_wg(int n, const int *rp, const int *col, const double *val, const double *b,
                       double *x, double tol, int max_iter, void *cm_col, void *cm_val,
                       WgCgOut *out, hipStream_t s);

// elements (of the inner type) of a slot's `work`
int64_t bslot_work_elems(int kind, int64_t n, int m);
// wide = 1024 threads per slot (single-system path), else 256
ck_status launch_batched_chunk(BSlot *slots, BStat *stat, const int *active, int nactive,
                               int budget, bool fp32, hipStream_t s, bool wide = false);

}  // namespace ck
