// Device transpose of a CSR matrix (equivalently its CSC form): the entries
// are sorted by column with a stable least-significant-digit radix sort
// (8-bit digits), so inside each row of the transpose the entries keep A's
// row order, which is ascending -- the transpose is canonical CSR whenever A
// is.  Rows of the transpose are counted with a column histogram and an
// exclusive scan (the scan kernels of the product).
#pragma once
#include "device_utils.h"
#include "spgemm_common.h"

namespace reap {

constexpr int kRsThreads = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;  // keys per workgroup
constexpr int kRsBins = 256;

// rowid[q] = i for every entry q of row i (one wavefront per row).
template <typename IdxT>
__global__ void __launch_bounds__(256) k_tr_rowid(const IdxT* __restrict__ rp, int64_t m, int32_t* __restrict__ rowid) {
    const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) / kWave;
    if (i >= m) return;
    const int64_t b = (int64_t)rp[i], e = (int64_t)rp[i + 1];
    for (int64_t q = b + lane_id(); q < e; q += kWave) rowid[q] = (int32_t)i;
}

// cnt[j] = entries of column j.
__global__ void __launch_bounds__(256) k_tr_colcount(const int32_t* __restrict__ col, int64_t nnz,
                                                     int32_t* __restrict__ cnt) {
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * 256)
        atomicAdd(&cnt[col[q]], 1);
}

// Digit histogram of one tile of keys: hist[d * ntiles + tile].
__global__ void __launch_bounds__(kRsThreads) k_rs_count(const int32_t* __restrict__ keys, int64_t n, int shift,
                                                         int32_t* __restrict__ hist) {
    __shared__ int32_t s_h[kRsBins];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        const int64_t e = base + (int64_t)r * kRsThreads + threadIdx.x;
        if (e < n) atomicAdd(&s_h[((uint32_t)keys[e] >> shift) & (kRsBins - 1)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = s_h[threadIdx.x];
}

// Stable scatter of one tile: element e of the tile goes to
// offs[d * ntiles + tile] + (number of earlier elements of the tile with digit d).
// Elements are taken in rounds of 256 in index order; inside a round the
// rank among equal digits comes from ballots over the digit bits (lanes of
// one wavefront) and per-wavefront digit counts (wavefronts of the round).
__global__ void __launch_bounds__(kRsThreads) k_rs_scatter(const int32_t* __restrict__ keys_in,
                                                           const int32_t* __restrict__ vals_in, int64_t n,
                                                           int shift, const int32_t* __restrict__ offs,
                                                           int32_t* __restrict__ keys_out,
                                                           int32_t* __restrict__ vals_out) {
    constexpr int NW = kRsThreads / kWave;
    __shared__ int32_t s_run[kRsBins];       // elements of each digit placed by earlier rounds
    __shared__ int32_t s_wc[NW][kRsBins];    // digit counts of each wavefront in this round
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    s_run[threadIdx.x] = offs[(int64_t)threadIdx.x * gridDim.x + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kRsItems; ++r) {
        for (int x = threadIdx.x; x < NW * kRsBins; x += kRsThreads) (&s_wc[0][0])[x] = 0;
        __syncthreads();
        const int64_t e = base + (int64_t)r * kRsThreads + threadIdx.x;
        const bool valid = e < n;
        const int32_t key = valid ? keys_in[e] : 0;
        const int32_t val = valid ? vals_in[e] : 0;
        const int d = ((uint32_t)key >> shift) & (kRsBins - 1);
        // lanes of this wavefront holding a valid element with the same digit
        uint64_t same = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = ballot(((d >> b) & 1) != 0);
            same &= ((d >> b) & 1) ? m : ~m;
        }
        const int rank_w = __popcll(same & below);
        const int cnt_w = __popcll(same);
        // the lowest lane of each digit group records the group's count
        if (valid && rank_w == 0) s_wc[w][d] = cnt_w;
        __syncthreads();
        if (valid) {
            int before = 0;
            for (int v = 0; v < w; ++v) before += s_wc[v][d];
            const int pos = s_run[d] + before + rank_w;
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        // advance the running offsets by this round's totals
        {
            int tot = 0;
#pragma unroll
            for (int v = 0; v < NW; ++v) tot += s_wc[v][threadIdx.x];
            s_run[threadIdx.x] += tot;
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_tr_gather(const int32_t* __restrict__ order, int64_t nnz,
                                                   const int32_t* __restrict__ rowid, const T* __restrict__ a_val,
                                                   int32_t* __restrict__ t_col, T* __restrict__ t_val) {
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * 256) {
        const int32_t e = order[q];
        t_col[q] = rowid[e];
        t_val[q] = a_val[e];
    }
}

__global__ void __launch_bounds__(256) k_tr_iota(int32_t* __restrict__ v, int64_t n) {
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
        v[q] = (int32_t)q;
}

__global__ void __launch_bounds__(256) k_tr_zero(int32_t* __restrict__ v, int64_t n) {
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256) v[q] = 0;
}

}  // namespace reap
