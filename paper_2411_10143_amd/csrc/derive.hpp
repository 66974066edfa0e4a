// The cascade's floating-point inputs from the exact integer features
// (feature table, Section III-B-1).  One definition, compiled for the host
// cascade and for the device-resident one, so both see the same bits: every
// value is a single correctly rounded IEEE operation (or a chain of them)
// with no contraction into fused multiply-adds, and the one 128-bit integer
// is converted with an explicit round-to-nearest-even.
#pragma once

#include <cmath>
#include <cstdint>

#if defined(__HIPCC__)
#define CK_HD __host__ __device__
#else
#define CK_HD
#endif

namespace ck {

// Nearest double to v (ties to even), by integer operations only.
CK_HD inline double u128_to_double(unsigned __int128 v) {
    if ((v >> 53) == 0)
        return (double)(unsigned long long)v;   // fits the significand: exact
    int top = 127;                               // index of the leading set bit
    while (((v >> top) & 1) == 0)
        --top;
    const int shift = top - 52;                  // low bits dropped
    unsigned long long mant = (unsigned long long)(v >> shift);
    const unsigned __int128 rem = v & (((unsigned __int128)1 << shift) - 1);
    const unsigned __int128 half = (unsigned __int128)1 << (shift - 1);
    int e = shift;
    if (rem > half || (rem == half && (mant & 1))) {
        ++mant;
        if (mant >> 53) {                        // carried into a new bit
            mant >>= 1;
            ++e;
        }
    }
    return std::ldexp((double)mant, e);          // mant < 2^53 and a power of two: exact
}

// I: the 28 integer fields of ck_features in struct order (nrows, ncols,
// nnz, sum_r, sum_r2, max_r, min_r, span_sum, cluster_sum, ndiag, diag_nnz,
// hist[16], is_symmetric).  out: density, mean, sd, cov, maxavg, distavg,
// clusteravg, fill, diagfill (all 0 for a matrix without rows).
CK_HD inline void derive_inputs(const int64_t *I, double *out) {
#pragma clang fp contract(off)
    for (int k = 0; k < 9; ++k)
        out[k] = 0.0;
    const int64_t nrows = I[0], ncols = I[1], nnz = I[2], sum_r = I[3], sum_r2 = I[4];
    const int64_t max_r = I[5], span = I[7], cluster = I[8], ndiag = I[9];
    if (nrows <= 0)
        return;
    const double n = (double)nrows;
    out[0] = ncols > 0 ? (double)nnz / (n * (double)ncols) : 0.0;
    out[1] = (double)nnz / n;
    const unsigned __int128 var =
        (unsigned __int128)nrows * (unsigned __int128)sum_r2 -
        (unsigned __int128)sum_r * (unsigned __int128)sum_r;   // >= 0 (Cauchy-Schwarz)
    out[2] = std::sqrt(u128_to_double(var)) / n;
    out[3] = out[1] > 0.0 ? out[2] / out[1] : 0.0;
    out[4] = (double)max_r - out[1];
    out[5] = (double)span / n;
    out[6] = (double)cluster / n;
    out[7] = nnz > 0 ? (n * (double)max_r) / (double)nnz : 0.0;
    out[8] = nnz > 0 ? (n * (double)ndiag) / (double)nnz : 0.0;
}

// The 15 model inputs in feature-table order.
CK_HD inline void model_inputs_from(const int64_t *I, const double *d, double *f) {
    f[0] = (double)I[0];
    f[1] = (double)I[1];
    f[2] = (double)I[2];
    f[3] = d[0];
    f[4] = d[1];
    f[5] = d[2];
    f[6] = d[3];
    f[7] = (double)I[5];
    f[8] = (double)I[6];
    f[9] = d[4];
    f[10] = d[5];
    f[11] = d[6];
    f[12] = d[7];
    f[13] = (double)I[9];
    f[14] = d[8];
}

}  // namespace ck
