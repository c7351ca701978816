// Symbolic pass: partial-product count per row (P_i), binning of rows by P_i,
// and the number of distinct columns of each row of C (the column set COLB of
// the paper's Algorithm 1), without any value arithmetic.
#pragma once
#include "device_utils.h"
#include "spgemm_common.h"

namespace reap {

template <typename IdxT>
struct SymArgs {
    int64_t m;                 // rows of A
    int64_t n;                 // columns of B
    int64_t k;                 // rows of B (B's row pointer has k + 1 entries)
    gptr<const IdxT> a_rp;
    gptr<const int32_t> a_col;
    gptr<const IdxT> b_rp;
    gptr<const int32_t> b_col;
    gptr<uint8_t> cls;         // [m] row class
    gptr<int32_t> rnnz;        // [m] nnz of each row of C
    gptr<int2> win;            // [m] {lo, words} bitmap window of wavefront rows; {lo, span} of long rows
    gptr<Counters> ctr;        // this product's counters
    gptr<WGPart> parts;        // per-workgroup statistics of the wavefront symbolic kernel
    gptr<unsigned long long> tiles;  // [ceil(m / kScanTile)] sum of rnnz over each scan tile (zeroed before)
    Thresholds th;
};

// Block-wide sum over a workgroup of NT threads.
template <int NT>
__device__ __forceinline__ long long block_sum_i64(long long v, long long* s_red) {
    v = wave_sum_i64(v);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if (lane_id() == 0) s_red[w] = v;
    __syncthreads();
    long long t = 0;
#pragma unroll
    for (int x = 0; x < NT / kWave; ++x) t += s_red[x];
    return t;
}

template <int NT>
__device__ __forceinline__ int block_min_i32(int v, int* s_red) {
    v = wave_min_i32(v);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if (lane_id() == 0) s_red[w] = v;
    __syncthreads();
    int t = INT32_MAX;
#pragma unroll
    for (int x = 0; x < NT / kWave; ++x) t = min(t, s_red[x]);
    return t;
}

template <int NT>
__device__ __forceinline__ int block_max_i32(int v, int* s_red) {
    v = wave_max_i32(v);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if (lane_id() == 0) s_red[w] = v;
    __syncthreads();
    int t = -1;
#pragma unroll
    for (int x = 0; x < NT / kWave; ++x) t = max(t, s_red[x]);
    return t;
}

// ---------------------------------------------------------------------------
// Optional operand check: row_ptr[0] = 0, non-decreasing, row_ptr[rows] = nnz,
// every column index in [0, cols).  Sets `flag_bit` in ctr->bad_csr.
template <typename IdxT>
__global__ void __launch_bounds__(256) k_validate(const IdxT* rp, const int32_t* col, int64_t rows,
                                                  int64_t cols, int64_t nnz, Counters* ctr,
                                                  unsigned flag_bit) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > rows) return;
    bool bad = false;
    const int64_t r = (int64_t)rp[i];
    if (i == 0 && r != 0) bad = true;
    if (i == rows && r != nnz) bad = true;
    if (i < rows) {
        const int64_t r1 = (int64_t)rp[i + 1];
        if (r1 < r || r < 0 || r1 > nnz) {
            bad = true;
        } else {
            for (int64_t q = r; q < r1; ++q) {
                const int32_t c = col[q];
                if (c < 0 || (int64_t)c >= cols) { bad = true; break; }
            }
        }
    }
    if (bad) atomicOr(&ctr->bad_csr, flag_bit);
}

}  // namespace reap
