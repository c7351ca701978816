// Exclusive prefix scan of the per-row entry counts of C into C's row pointer
// (the allocation step that the row-by-row product needs before any value is
// written), plus the reduction of the symbolic pass's statistics.
#pragma once
#include "device_utils.h"
#include "spgemm_common.h"

namespace reap {

// Per-product view of the scan.
struct ScanArgs {
    const int32_t* rnnz;   // [m] nnz of each row of C
    int64_t m;
    long long* tiles;      // [ntiles] tile sums, then tile offsets
    int32_t ntiles;
    int32_t nparts;
    const WGPart* parts;   // [nparts] statistics of the wavefront symbolic kernel
    Counters* ctr;
    void* c_rp;            // [m + 1] C row pointer (IdxC)
    Counters* h_ctr;       // the product's counters in pinned host memory (device-mapped), or null
    const unsigned int* n_long;   // long-row counter block of the batch ...
    unsigned int* h_nlong;        // ... and the host copy of its counts (written by product 0), or null
    TileStat* h_tiles;     // [ntiles] the product's tile statistics in pinned host memory (one-launch scan)
};

// Host copy of the long-row counts: all long rows, medium rows, large rows.
__device__ __forceinline__ void copy_long_counts(unsigned int* h, const unsigned int* n_long) {
    h[0] = n_long[kLongCtrCount];
    h[1] = n_long[kLongCtrSplit];
    h[2] = n_long[kLongCtrSplit + 1];
}

// Tile t of product q: tile_start[q] <= blockIdx.x < tile_start[q + 1].
struct ScanMap {
    const int32_t* tile_start;  // [nprod + 1]
    int32_t nprod;
};

__device__ __forceinline__ void scan_tile_of(const ScanArgs& s0, const ScanArgs* S, ScanMap sm, ScanArgs& s, int& t) {
    const int q = sm.nprod > 1 ? find_product(sm.tile_start, sm.nprod, (int)blockIdx.x) : 0;
    t = (int)blockIdx.x - (sm.nprod > 1 ? sm.tile_start[q] : 0);
    s = S ? S[q] : s0;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(ScanArgs s0, const ScanArgs* __restrict__ S, ScanMap sm) {
    __shared__ long long s_red[kScanThreads / kWave];
    ScanArgs sa;
    int t;
    scan_tile_of(s0, S, sm, sa, t);
    const int64_t base = (int64_t)t * kScanTile + (int64_t)threadIdx.x * kScanItems;
    long long s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j)
        if (base + j < sa.m) s += sa.rnnz[base + j];
    long long total;
    block_excl_scan_i64<kScanThreads>(s, s_red, &total);
    if (threadIdx.x == 0) sa.tiles[t] = total;
}

// One workgroup per product: scans the product's tile sums in place
// (exclusive), folds the per-workgroup statistics of the symbolic kernel into
// its counters, and writes C.row_ptr[m] = nnz(C).
template <typename IdxC>
__global__ void __launch_bounds__(1024) k_scan_spine(ScanArgs s0, const ScanArgs* __restrict__ S) {
    __shared__ long long s_red[1024 / kWave];
    __shared__ unsigned long long s_prod[1024 / kWave];
    __shared__ unsigned int s_cls[1024 / kWave][kNumClasses];
    __shared__ unsigned int s_max[1024 / kWave][2];
    const ScanArgs sa = S ? S[blockIdx.x] : s0;
    long long* __restrict__ tile_sums = sa.tiles;
    const int ntiles = sa.ntiles;
    const WGPart* __restrict__ parts = sa.parts;
    const int nparts = sa.nparts;
    Counters* ctr = sa.ctr;
    IdxC* c_rp = static_cast<IdxC*>(sa.c_rp);
    const int64_t m = sa.m;
    long long carry = 0;
    for (int b0 = 0; b0 < ntiles; b0 += 1024) {
        const int b = b0 + threadIdx.x;
        const long long v = (b < ntiles) ? tile_sums[b] : 0;
        long long total;
        const long long ex = block_excl_scan_i64<1024>(v, s_red, &total);
        if (b < ntiles) tile_sums[b] = carry + ex;
        carry += total;
    }
    unsigned long long prod = 0;
    unsigned int cls[kNumClasses] = {0, 0, 0, 0, 0};
    unsigned int mp = 0, mn = 0;
    for (int x = threadIdx.x; x < nparts; x += 1024) {
        const WGPart& q = parts[x];
        prod += q.products;
#pragma unroll
        for (int c = 0; c < kNumClasses; ++c) cls[c] += q.cls[c];
        mp = max(mp, q.max_prod);
        mn = max(mn, q.max_nnz);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        prod += __shfl_xor(prod, o, kWave);
#pragma unroll
        for (int c = 0; c < kNumClasses; ++c) cls[c] += __shfl_xor(cls[c], o, kWave);
        mp = max(mp, __shfl_xor(mp, o, kWave));
        mn = max(mn, __shfl_xor(mn, o, kWave));
    }
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
        s_prod[w] = prod;
#pragma unroll
        for (int c = 0; c < kNumClasses; ++c) s_cls[w][c] = cls[c];
        s_max[w][0] = mp;
        s_max[w][1] = mn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int x = 1; x < 1024 / kWave; ++x) {
            prod += s_prod[x];
            for (int c = 0; c < kNumClasses; ++c) cls[c] += s_cls[x][c];
            mp = max(mp, s_max[x][0]);
            mn = max(mn, s_max[x][1]);
        }
        ctr->products += prod;   // the long-row kernel has already added its rows
        for (int c = 0; c < kNumClasses; ++c) ctr->cls[c] = cls[c];
        ctr->max_prod = max(ctr->max_prod, mp);
        ctr->max_nnz = max(ctr->max_nnz, mn);
        ctr->nnz = (unsigned long long)carry;
        c_rp[m] = (IdxC)carry;
        // the host reads the counters straight from its pinned mirror once
        // the stream is synchronised (no device-to-host copy is enqueued)
        if (sa.h_ctr) *sa.h_ctr = *ctr;
        if (sa.h_nlong && blockIdx.x == 0) copy_long_counts(sa.h_nlong, sa.n_long);
        __threadfence_system();
    }
}

template <typename IdxC>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(ScanArgs s0, const ScanArgs* __restrict__ S, ScanMap sm) {
    __shared__ long long s_red[kScanThreads / kWave];
    ScanArgs sa;
    int t;
    scan_tile_of(s0, S, sm, sa, t);
    IdxC* __restrict__ c_rp = static_cast<IdxC*>(sa.c_rp);
    const int64_t base = (int64_t)t * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    long long s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = (base + j < sa.m) ? sa.rnnz[base + j] : 0;
        s += v[j];
    }
    long long total;
    long long run = sa.tiles[t] + block_excl_scan_i64<kScanThreads>(s, s_red, &total);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < sa.m) c_rp[base + j] = (IdxC)run;
        run += v[j];
    }
}

// One-launch scan, used when no product has more than kScanOnePassTiles
// tiles.  The symbolic kernels have already added every row's count into its
// tile's sum, so tile t of a product learns its offset by summing the sums of
// tiles 0..t-1 itself (a few loads per thread) and no workgroup waits for
// another or synchronises with another.  Wavefront 0 of each tile's workgroup
// folds the statistics of the wavefront workgroups that covered the tile's
// rows and writes them, with the tile's entry count, to the pinned host
// mirror; the host adds the tiles up after the pass.  The extra workgroup
// b == total_tiles copies every product's counters (what the long-row kernel
// accumulated) and the long-row count to the host mirror and writes
// row_ptr[0] = 0 of products without rows.
constexpr int kScanOnePassTiles = 1024;

template <typename IdxC>
__global__ void __launch_bounds__(kScanThreads)
k_scan_onepass(ScanArgs s0, const ScanArgs* __restrict__ S, ScanMap sm, int total_tiles) {
    __shared__ long long s_red[kScanThreads / kWave];
    const int b = (int)blockIdx.x;
    if (b == total_tiles) {
        const int nprod = sm.nprod;
        constexpr int words = (int)(sizeof(Counters) / 4);
        for (int x = threadIdx.x; x < nprod * words; x += kScanThreads) {
            const ScanArgs& sa = S ? S[x / words] : s0;
            reinterpret_cast<uint32_t*>(sa.h_ctr)[x % words] = reinterpret_cast<const uint32_t*>(sa.ctr)[x % words];
        }
        for (int q = threadIdx.x; q < nprod; q += kScanThreads) {
            const ScanArgs& sa = S ? S[q] : s0;
            if (sa.m == 0) static_cast<IdxC*>(sa.c_rp)[0] = (IdxC)0;
        }
        if (threadIdx.x == 0) copy_long_counts(s0.h_nlong, s0.n_long);
        return;
    }
    ScanArgs sa;
    int t;
    scan_tile_of(s0, S, sm, sa, t);
    const long long* __restrict__ tile_sums = sa.tiles;
    long long pre = 0;
    for (int x = threadIdx.x; x < t; x += kScanThreads) pre += tile_sums[x];
    block_excl_scan_i64<kScanThreads>(pre, s_red, &pre);

    IdxC* __restrict__ c_rp = static_cast<IdxC*>(sa.c_rp);
    const int64_t base = (int64_t)t * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    long long sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = (base + j < sa.m) ? sa.rnnz[base + j] : 0;
        sum += v[j];
    }
    long long total;
    long long run = pre + block_excl_scan_i64<kScanThreads>(sum, s_red, &total);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < sa.m) c_rp[base + j] = (IdxC)run;
        run += v[j];
    }
    if (t == sa.ntiles - 1 && threadIdx.x == 0) c_rp[sa.m] = (IdxC)(pre + total);

    if (threadIdx.x < kWave) {
        constexpr int per_tile = kScanTile / kRowsPerBlock;
        const int x0 = t * per_tile, x1 = min(sa.nparts, x0 + per_tile);
        unsigned long long prod = 0;
        unsigned int cls[kNumClasses] = {0, 0, 0, 0, 0};
        unsigned int mp = 0, mn = 0;
        for (int x = x0 + (int)threadIdx.x; x < x1; x += kWave) {
            const WGPart& q = sa.parts[x];
            prod += q.products;
#pragma unroll
            for (int c = 0; c < kNumClasses; ++c) cls[c] += q.cls[c];
            mp = max(mp, q.max_prod);
            mn = max(mn, q.max_nnz);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            prod += __shfl_xor(prod, o, kWave);
#pragma unroll
            for (int c = 0; c < kNumClasses; ++c) cls[c] += __shfl_xor(cls[c], o, kWave);
            mp = max(mp, __shfl_xor(mp, o, kWave));
            mn = max(mn, __shfl_xor(mn, o, kWave));
        }
        // lanes write the record's words in parallel
        uint32_t w[sizeof(TileStat) / 4] = {(uint32_t)total, (uint32_t)((unsigned long long)total >> 32),
                                            (uint32_t)prod, (uint32_t)(prod >> 32),
                                            cls[0], cls[1], cls[2], cls[3], cls[4], mp, mn, 0u};
        static_assert(sizeof(TileStat) == 48 && kNumClasses == 5, "tile record layout");
        const int l = (int)threadIdx.x;
        uint32_t mine = 0;
#pragma unroll
        for (int x = 0; x < 12; ++x) mine = (l == x) ? w[x] : mine;
        if (l < 12) reinterpret_cast<uint32_t*>(sa.h_tiles + t)[l] = mine;
    }
}

// Zeroes the counters, the long-row count and queue words, and the scan
// tiles' sums (a kernel rather than a memset, so the sequence can be
// captured in a graph).
__global__ void k_zero_counters(Counters* ctr, int nprod, unsigned int* n_long, long long* tiles, int ntiles) {
    uint32_t* p = reinterpret_cast<uint32_t*>(ctr);
    const int64_t words = (int64_t)nprod * (int64_t)(sizeof(Counters) / 4);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t x0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t x = x0; x < words; x += stride) p[x] = 0u;
    for (int64_t x = x0; x < ntiles; x += stride) tiles[x] = 0;
    if (blockIdx.x == 0 && threadIdx.x < kLongCtrWords) n_long[threadIdx.x] = 0u;  // counts and queue counters
}

}  // namespace reap
