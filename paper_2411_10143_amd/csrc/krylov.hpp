// Device-resident solver state and the reduction helpers the fused Krylov
// kernels share.  All scalar algebra of CG and GMRES stays on the GPU; the
// host only enqueues work and polls a small status record.
#pragma once

#include "common.hpp"

namespace ck {

constexpr int kMaxRestart = 64;    // largest GMRES restart length m
// Row-blocked kernels launch at most this many workgroups (32 per CU) and
// loop over row groups inside each one: the dispatcher issues roughly one
// workgroup per nanosecond, so a workgroup per short row group would make
// the launch, not memory, the bound.  Also the most partials one reduction
// ever finishes.
constexpr int kMaxPartials = 8192;
constexpr int kRowBlocks = kMaxPartials;
// GMRES Gram-Schmidt passes: at most this many blocks, one partial per
// block and basis column.
constexpr int kGmMaxBlocks = 2048;

// Run states shared by the solvers
enum : int { RUN = 0, CONVERGED = 1, BREAKDOWN = 2, BUDGET = 3 };

// CG (Hestenes-Stiefel) scalars.  `state` != RUN makes every iteration
// kernel a no-op, so the host may enqueue ahead of convergence.
template <typename T>
struct CgDev {
    T rho;            // r.r of the current residual
    T rho_prev;       // rho as the sigma finish saw it (read by the x/p
                      // update while its block 0 replaces rho)
    T sigma;          // p.Ap
    T alpha, beta;
    double bnorm;     // ||rhs|| of this (inner) solve
    double tol;       // stop when sqrt(rho)/bnorm <= tol
    double relres;    // last sqrt(rho)/bnorm
    int state;
    int iter;         // iterations completed
    int max_iter;
    int go;           // set by the sigma finish: 1 when this iteration's
                      // x/p update runs (state RUN and sigma > 0)
};

// GMRES(m) cycle scalars (Givens form of the Hessenberg least squares).
// cycle_stop ends the current cycle's Arnoldi steps; final_state ends the
// whole solve.  H is column-major (m+1) x m.
template <typename T>
struct GmDev {
    T H[(kMaxRestart + 1) * kMaxRestart];
    T cs[kMaxRestart], sn[kMaxRestart];
    T g[kMaxRestart + 1];
    T y[kMaxRestart];
    T Hraw[(kMaxRestart + 1) * kMaxRestart];   // H before the rotations
    T h1[kMaxRestart + 1];      // first Gram-Schmidt pass
    T h2[kMaxRestart + 1];      // second pass
    T u[kMaxRestart + 2];       // Hbar_j h2: A (V_j h2) = V_{j+1} u
    T inv;                      // 1 / h_{j+1,j}
    double beta;                // ||r|| at the cycle start (FP64 true residual)
    double inv_beta;            // 1 / beta
    double bnorm, tol, relres;  // relres: last estimate or true value
    int m;
    int j;                      // Arnoldi steps done in this cycle
    int iter;                   // total Arnoldi steps
    int max_iter;
    int cycle_stop;             // RUN, CONVERGED (estimate), BREAKDOWN (happy), BUDGET
    int final_state;            // RUN, CONVERGED, BREAKDOWN (singular), BUDGET
    int cycles;
    int halt;                   // 1 when cycle_stop or final_state is not RUN
};

constexpr int FULL = 4;         // cycle_stop value: m steps done

// ---- two-stage reductions ----------------------------------------------------
// Every reduction writes one partial per block; a separate one-block
// "finish" kernel then sums the partials in block order and does the scalar
// algebra.  The kernel boundary makes the partials visible across XCDs, so no
// device-scope fence (an L2 write-back on this chip) is issued per block.

// Fixed-order sum of n partials by the 256 threads of one block (valid in
// thread 0 only).  Thread t adds p[t], p[t + 256], ... in order; the loads of
// eight consecutive terms are issued together (index clamped, term masked).
template <typename T>
__device__ __forceinline__ T sum_partials(const T *p, int64_t n, T *lds4) {
    constexpr int U = 8;
    T s = 0;
    for (int64_t i0 = threadIdx.x; i0 < n; i0 += U * 256) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * 256;
            v[u] = __builtin_nontemporal_load(&p[i < n ? i : n - 1]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 + u * 256 < n)
                s += v[u];
    }
    return block_sum(s, lds4);
}

}  // namespace ck
