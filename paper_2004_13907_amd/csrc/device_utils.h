// Wavefront-level helpers for gfx950 (CDNA4, 64-lane wavefronts).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace reap {

constexpr int kWave = 64;
constexpr int kNumXcd = 8;  // MI355X: 8 accelerator complex dies, each with its own L2
// Word 3 of a raw buffer descriptor on CDNA (gfx9 family): 32-bit data
// format, no swizzle, no index stride.  Reads past the descriptor's
// num_records bytes return 0.
constexpr int kBufferWord3 = 0x00020000;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Orders this wavefront's LDS accesses across lanes (no cross-wave effect).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Number of set bits of m in lanes strictly below this lane.
__device__ __forceinline__ int mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Marks a value that is equal on all lanes as wave-uniform (scalar register).
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int32_t uniform(int32_t v) { return uniform_i32(v); }
__device__ __forceinline__ int64_t uniform(int64_t v) { return uniform_i64(v); }

template <typename T>
__device__ __forceinline__ T shfl(T v, int src) { return __shfl(v, src, kWave); }

__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ long long wave_sum_i64(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}

// Inclusive prefix sum across the wavefront.
__device__ __forceinline__ int wave_incl_scan_i32(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
    }
    return v;
}

__device__ __forceinline__ long long wave_incl_scan_i64(long long v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        long long u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
    }
    return v;
}

// --- DPP (data-parallel primitive) wavefront scans and reductions ----------
// Lanes are grouped in 4 rows of 16.  row_shr:n moves values n lanes up inside
// a row; row_bcast:15 / row_bcast:31 broadcast lane 15 / 31 into the following
// rows.  Out-of-range sources read 0 (or the identity passed as `old`).
constexpr int kDppRowShr = 0x110;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

template <int N>
__device__ __forceinline__ int dpp_shr(int v, int id) {
    return __builtin_amdgcn_update_dpp(id, v, kDppRowShr + N, 0xf, 0xf, false);
}

// Inclusive prefix sum over the wavefront.
__device__ __forceinline__ int dpp_incl_scan(int v) {
    v += dpp_shr<1>(v, 0);
    v += dpp_shr<2>(v, 0);
    v += dpp_shr<4>(v, 0);
    v += dpp_shr<8>(v, 0);
    v += __builtin_amdgcn_update_dpp(0, v, kDppRowBcast15, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kDppRowBcast31, 0xc, 0xf, false);
    return v;
}

// Reductions whose result is returned to every lane (read from lane 63).
__device__ __forceinline__ int dpp_reduce_sum(int v) {
    return __builtin_amdgcn_readlane(dpp_incl_scan(v), kWave - 1);
}

__device__ __forceinline__ int dpp_reduce_max(int v) {  // for v >= INT32_MIN + 1
    constexpr int id = INT32_MIN;
    v = max(v, dpp_shr<1>(v, id));
    v = max(v, dpp_shr<2>(v, id));
    v = max(v, dpp_shr<4>(v, id));
    v = max(v, dpp_shr<8>(v, id));
    v = max(v, __builtin_amdgcn_update_dpp(id, v, kDppRowBcast15, 0xa, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(id, v, kDppRowBcast31, 0xc, 0xf, false));
    return __builtin_amdgcn_readlane(v, kWave - 1);
}

__device__ __forceinline__ int dpp_reduce_min(int v) {
    return -dpp_reduce_max(-v);  // v > INT32_MIN
}

// Exclusive scan over a workgroup of NT threads; returns this thread's
// exclusive prefix and writes the block total to *total.
template <int NT>
__device__ __forceinline__ long long block_excl_scan_i64(long long v, long long* s_red, long long* total) {
    const int w = threadIdx.x / kWave, lane = lane_id();
    const long long incl = wave_incl_scan_i64(v);
    __syncthreads();
    if (lane == kWave - 1) s_red[w] = incl;
    __syncthreads();
    long long before = 0, all = 0;
    // partially unrolled: sixteen 64-bit partials loaded at once would take
    // 32 registers at a point where the long-row kernels have none to spare
#pragma unroll 4
    for (int x = 0; x < NT / kWave; ++x) {
        const long long t = s_red[x];
        before += (x < w) ? t : 0;
        all += t;
    }
    *total = all;
    return before + incl - v;
}

// The same scan with one barrier: the partials go to `buf`, which no thread
// may still be reading from an earlier call (the caller places a workgroup
// barrier between two calls on one buffer).
template <int NT>
__device__ __forceinline__ long long block_excl_scan1_i64(long long v, long long* buf, long long* total) {
    const int w = threadIdx.x / kWave, lane = lane_id();
    const long long incl = wave_incl_scan_i64(v);
    if (lane == kWave - 1) buf[w] = incl;
    __syncthreads();
    long long before = 0, all = 0;
    // partially unrolled: sixteen 64-bit partials loaded at once would take
    // 32 registers at a point where the long-row kernels have none to spare
#pragma unroll 4
    for (int x = 0; x < NT / kWave; ++x) {
        const long long t = buf[x];
        before += (x < w) ? t : 0;
        all += t;
    }
    *total = all;
    return before + incl - v;
}

// Maps hardware workgroup ids (dispatched round-robin over the XCDs) to
// logical ids so that each XCD processes one contiguous range of logical ids;
// neighbouring rows then share that XCD's L2.  A bijection on [0, n).
__device__ __forceinline__ int xcd_contiguous_block(int b, int n) {
    const int q = n / kNumXcd, r = n % kNumXcd;
    const int xcd = b % kNumXcd, idx = b / kNumXcd;
    return (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Index q of the product that owns workgroup b: start[q] <= b < start[q + 1]
// (start is non-decreasing, start[0] = 0).  Uniform across the workgroup.
__device__ __forceinline__ int find_product(const int32_t* start, int nprod, int b) {
    int lo = 0, hi = nprod;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// Multiplicative hash for LDS open-addressing tables (Knuth's constant).
__device__ __forceinline__ uint32_t hash_col(int32_t c) { return (uint32_t)c * 2654435761u; }

}  // namespace reap
