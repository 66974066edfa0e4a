// Internal helpers shared by the HIP translation units of libcaskrylov.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>

#include "../../include/caskrylov.h"

namespace ck {

// ---- error plumbing --------------------------------------------------------
void set_error(const std::string &msg);
ck_status fail(ck_status st, const char *fmt, ...);

#define CK_HIP(...)                                                                    \
    do {                                                                               \
        hipError_t e_ = (__VA_ARGS__);                                                 \
        if (e_ != hipSuccess)                                                          \
            return ::ck::fail(CK_E_HIP, "%s failed: %s (%s:%d)", #__VA_ARGS__,         \
                              hipGetErrorString(e_), __FILE__, __LINE__);              \
    } while (0)

#define CK_TRY(...)                                                                    \
    do {                                                                               \
        ck_status s_ = (__VA_ARGS__);                                                  \
        if (s_ != CK_OK)                                                               \
            return s_;                                                                 \
    } while (0)

// ---- launch geometry --------------------------------------------------------
constexpr int kBlock = 256;   // 4 wave64 per workgroup
constexpr int kWave = 64;
constexpr int kXcds = 8;      // MI355X: workgroups are dealt round-robin over 8 XCDs

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// A grid padded to a multiple of the XCD count, so that xcd_block() can give
// every XCD one contiguous range of logical blocks.
inline int64_t xcd_grid(int64_t blocks) { return ceil_div(blocks, kXcds) * kXcds; }

// Logical block for hardware block b of a grid built with xcd_grid(G):
// XCD x = b % 8 receives logical blocks [x*G/8, (x+1)*G/8), so neighbouring
// row blocks share one XCD's L2.  Returns -1 for padding blocks.
__device__ __forceinline__ int64_t xcd_block(int64_t G) {
    const int64_t Gp = (int64_t)gridDim.x;
    const int64_t b = (int64_t)blockIdx.x;
    const int64_t logical = (b % kXcds) * (Gp / kXcds) + b / kXcds;
    return logical < G ? logical : -1;
}

// ---- wave64 reductions ---------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v += __shfl_xor(v, off, kWave);
    return v;
}

// Sum over groups of L consecutive lanes (L a power of two <= 64); every lane
// of a group ends with the group total.  Fixed butterfly order: deterministic.
template <int L, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1)
        v += __shfl_xor(v, off, L);
    return v;
}

// Block (256 threads) sum, result valid in thread 0.  Fixed order.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *lds4) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0)
        lds4[w] = v;
    __syncthreads();
    T r = 0;
    if (threadIdx.x == 0)
        r = (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
    __syncthreads();
    return r;
}

// Streaming loads of matrix arrays: touched once per product, so they are
// marked non-temporal to leave cache capacity to the gathered vector.
template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) {
    return __builtin_nontemporal_load(p);
}

}  // namespace ck
