// Internal helpers shared by the HIP translation units of libcaskrylov.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>
#include <type_traits>

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

// v moved across lanes by the DPP control CTRL (row_mask RM, bank_mask BM);
// lanes with no source, or masked out, read 0.  A double moves as its two
// 32-bit halves.
template <int CTRL, int RM, int BM>
__device__ __forceinline__ double dpp_read(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int l = __builtin_amdgcn_update_dpp(0, lo, CTRL, RM, BM, true);
    const int h = __builtin_amdgcn_update_dpp(0, hi, CTRL, RM, BM, true);
    return __hiloint2double(h, l);
}
template <int CTRL, int RM, int BM>
__device__ __forceinline__ float dpp_read(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, RM, BM, true));
}

template <int CTRL, int RM, int BM>
__device__ __forceinline__ unsigned long long dpp_read(unsigned long long v) {
    const unsigned l = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, RM, BM,
                                                             true);
    const unsigned h = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL,
                                                             RM, BM, true);
    return ((unsigned long long)h << 32) | l;
}

// Sum over the 64 lanes of a wave, valid in lane 63 only, by data-parallel-
// primitive moves between registers (no LDS permute, so a step costs a few
// cycles instead of an LDS round trip): within each row of 16 lanes, lane i
// adds lanes i-1, i-2, i-3 (row_shr 1..3), then lane i-4 (row_shr 4, lanes
// 4..15) and lane i-8 (row_shr 8, lanes 8..15), so lane 15 of each row holds
// the row's sum; rows 1 and 3 then add lane 15 of the row before (row_bcast
// 15), and rows 2 and 3 add lane 31 (row_bcast 31).  Fixed order:
// deterministic.
template <typename T>
__device__ __forceinline__ T wave_sum_last(T v) {
    T t = v + dpp_read<0x111, 0xf, 0xf>(v);
    t += dpp_read<0x112, 0xf, 0xf>(v);
    t += dpp_read<0x113, 0xf, 0xf>(v);
    t += dpp_read<0x114, 0xf, 0xe>(t);
    t += dpp_read<0x118, 0xf, 0xc>(t);
    t += dpp_read<0x142, 0xa, 0xf>(t);
    t += dpp_read<0x143, 0xc, 0xf>(t);
    return t;
}

// Maximum over the 64 lanes of a wave (unsigned: lanes without a source
// read 0, the identity), valid in lane 63, in the steps of wave_sum_last.
__device__ __forceinline__ unsigned long long wave_max_last(unsigned long long v) {
    auto mx = [](unsigned long long a, unsigned long long b) { return a > b ? a : b; };
    unsigned long long t = mx(v, dpp_read<0x111, 0xf, 0xf>(v));
    t = mx(t, dpp_read<0x112, 0xf, 0xf>(v));
    t = mx(t, dpp_read<0x113, 0xf, 0xf>(v));
    t = mx(t, dpp_read<0x114, 0xf, 0xe>(t));
    t = mx(t, dpp_read<0x118, 0xf, 0xc>(t));
    t = mx(t, dpp_read<0x142, 0xa, 0xf>(t));
    t = mx(t, dpp_read<0x143, 0xc, 0xf>(t));
    return t;
}
// Minimum: the maximum of the complements, complemented.
__device__ __forceinline__ unsigned long long wave_min_last(unsigned long long v) {
    return ~wave_max_last(~v);
}

// Inclusive scan of v over the lanes of a wave, restarted wherever key
// changes: a lane gets the sum of v over the lanes of its run up to itself.
// Lanes with equal keys must form one contiguous run, except key -1, whose
// lanes may get any value.  DPP moves only: within each row of 16 lanes,
// lane i adds lane i-1, then i-2, i-4, i-8 (row_shr, each only if that
// lane has the same key), so every lane holds its run's sum within its row;
// rows 1 and 3 then add lane 15 of the row before (row_bcast 15) and rows 2
// and 3 lane 31 (row_bcast 31), again only on equal keys.  Keys move as
// key + 2, so a lane with no source (which reads 0) never matches.  Fixed
// order: deterministic.
template <int CTRL, int RM, typename T>
__device__ __forceinline__ void seg_scan_step(T &v, int k) {
    const int ku = __builtin_amdgcn_update_dpp(0, k, CTRL, RM, 0xf, true);
    const T vu = dpp_read<CTRL, RM, 0xf>(v);
    v = ku == k ? v + vu : v;
}
template <typename T>
__device__ __forceinline__ T wave_seg_scan(T v, int key) {
    const int k = key + 2;
    seg_scan_step<0x111, 0xf>(v, k);
    seg_scan_step<0x112, 0xf>(v, k);
    seg_scan_step<0x114, 0xf>(v, k);
    seg_scan_step<0x118, 0xf>(v, k);
    seg_scan_step<0x142, 0xa>(v, k);
    seg_scan_step<0x143, 0xc>(v, k);
    return v;
}

// Sum over groups of L consecutive lanes (L a power of two <= 64) by DPP
// register moves, valid in lane L - 1 of each group (for L <= 16 in every
// lane of the group): lanes exchange with lane ^ 1 and lane ^ 2 (quad
// permutes), then add the mirrored half row (8) and the mirrored row (16);
// rows 1 and 3 add lane 15 of the row before (32), rows 2 and 3 add lane 31
// (64).  Fixed order: deterministic.
template <int L, typename T>
__device__ __forceinline__ T group_sum_last(T v) {
    if constexpr (L >= 2)
        v += dpp_read<0xb1, 0xf, 0xf>(v);    // quad_perm [1, 0, 3, 2]
    if constexpr (L >= 4)
        v += dpp_read<0x4e, 0xf, 0xf>(v);    // quad_perm [2, 3, 0, 1]
    if constexpr (L >= 8)
        v += dpp_read<0x141, 0xf, 0xf>(v);   // row_half_mirror
    if constexpr (L >= 16)
        v += dpp_read<0x140, 0xf, 0xf>(v);   // row_mirror
    if constexpr (L >= 32)
        v += dpp_read<0x142, 0xa, 0xf>(v);   // row_bcast 15 into rows 1, 3
    if constexpr (L >= 64)
        v += dpp_read<0x143, 0xc, 0xf>(v);   // row_bcast 31 into rows 2, 3
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
// Floating-point sums use the DPP wave sum (its total sits in lane 63).
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *lds4) {
    constexpr bool fp = std::is_same<T, double>::value || std::is_same<T, float>::value;
    int src = 0;
    if constexpr (fp) {
        v = wave_sum_last(v);
        src = kWave - 1;
    } else {
        v = wave_sum(v);
    }
    const int w = threadIdx.x / kWave;
    if ((int)(threadIdx.x & (kWave - 1)) == src)
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
