// Numeric pass: partial products a_ik * b_kj, their accumulation by column and
// the ascending-column write of each row of C (the multiply, sort and merge
// steps of the paper's Algorithm 1).  Sorting is replaced by ranking: a bitmap
// over the row's column window, with a prefix count per 32-bit word, gives
// every column its position in the sorted row directly.  This file holds the
// argument block and the long-row kernel; the wavefront kernels are in
// kernels_wave.h.
#pragma once
#include "device_utils.h"
#include "kernels_symbolic.h"
#include "spgemm_common.h"

namespace reap {

template <typename T, typename IdxT, typename IdxC>
struct NumArgs {
    int64_t m;
    int64_t n;
    const IdxT* a_rp;
    const int32_t* a_col;
    const T* a_val;
    const IdxT* b_rp;
    const int32_t* b_col;
    const T* b_val;
    const IdxC* c_rp;
    int32_t* c_col;
    T* c_val;
    const uint8_t* cls;
    const int2* win;
    const int32_t* group_rows;
    Counters* ctr;
    double* gvals;          // per-workgroup FP64 accumulators for long rows with FP32 output
    int64_t gvals_stride;   // doubles per workgroup slot
    Thresholds th;
};

// ---------------------------------------------------------------------------
// Long rows: one workgroup per row (atomic work counter over the long-row
// list).  The column window is processed in segments of th.group_lds_span
// columns.  Per segment: (1) set the bitmap bit of every product's column,
// (2) prefix-count the bitmap words, (3) re-gather the products and add each
// into the slot given by its column's rank, in LDS when the segment has at
// most th.group_lds_values entries, otherwise in device memory (the row's own
// output for FP64, a per-workgroup FP64 buffer for FP32), (4) write columns
// from the bitmap (already ascending) and the values.
template <typename T, typename IdxT, typename IdxC>
__global__ void __launch_bounds__(1024) k_num_group(NumArgs<T, IdxT, IdxC> p) {
    constexpr int NT = 1024, NW = NT / kWave;
    __shared__ uint32_t s_bits[kGroupBitsWords];
    __shared__ uint32_t s_pfx[kGroupBitsWords];
    __shared__ double s_vals[kGroupLdsValues];
    __shared__ uint32_t s_smask[NW][kGroupMaskWords];
    __shared__ int64_t s_ebase[NW][kWave];
    __shared__ double s_eval[NW][kWave];
    __shared__ long long s_red[NW];
    __shared__ int s_row;

    const int w = threadIdx.x / kWave;
    const int nG = (int)p.ctr->n_group;
    for (;;) {
        if (threadIdx.x == 0) s_row = (int)atomicAdd(&p.ctr->group_next_num, 1u);
        __syncthreads();
        const int j = s_row;
        __syncthreads();
        if (j >= nG) break;
        const int64_t i = p.group_rows[j];
        const IdxT rs = p.a_rp[i];
        const int64_t nA = (int64_t)p.a_rp[i + 1] - (int64_t)rs;
        const int2 wn = p.win[i];
        const int lo = wn.x;
        const int64_t span = wn.y;
        const int64_t cb = (int64_t)p.c_rp[i];
        const int64_t nc_row = (int64_t)p.c_rp[i + 1] - cb;
        int64_t off = 0;
        for (int64_t s0 = 0; s0 < span; s0 += p.th.group_lds_span) {
            const int seg_lo = lo + (int)s0;
            const int seg_w = (int)((min((int64_t)p.th.group_lds_span, span - s0) + 31) >> 5);
            const int seg_hi = seg_lo + seg_w * 32;
            for (int x = threadIdx.x; x < seg_w; x += NT) s_bits[x] = 0u;
            __syncthreads();
            long long dummy = 0;
            wave_row_products<IdxT, T, false>(rs, nA, p.a_col, p.a_val, p.b_rp, p.b_col, w, NW, s_smask[w],
                                              s_ebase[w], s_eval[w], dummy, [&](int col, int64_t, double) {
                                                  if (col >= seg_lo && col < seg_hi) {
                                                      const int d = col - seg_lo;
                                                      atomicOr(&s_bits[d >> 5], 1u << (d & 31));
                                                  }
                                              });
            __syncthreads();
            const int per = (seg_w + NT - 1) / NT;
            const int w0 = min((int)threadIdx.x * per, seg_w), w1 = min(w0 + per, seg_w);
            long long local = 0;
            for (int x = w0; x < w1; ++x) local += __popc(s_bits[x]);
            long long seg_nnz;
            long long run = block_excl_scan_i64<NT>(local, s_red, &seg_nnz);
            for (int x = w0; x < w1; ++x) {
                s_pfx[x] = (uint32_t)run;
                run += __popc(s_bits[x]);
            }
            if (off + seg_nnz > nc_row) {  // pattern differs from the symbolic pass
                if (threadIdx.x == 0) atomicOr(&p.ctr->bad_csr, 4u);
                break;
            }
            const bool in_lds = seg_nnz <= p.th.group_lds_values;
            double* gacc = nullptr;  // device-memory accumulator of a segment too long for LDS
            if (!in_lds) {
                if constexpr (sizeof(T) == sizeof(double)) {
                    gacc = reinterpret_cast<double*>(p.c_val) + cb + off;
                } else {
                    gacc = p.gvals + (int64_t)blockIdx.x * p.gvals_stride;
                }
            }
            if (in_lds) {
                for (long long x = threadIdx.x; x < seg_nnz; x += NT) s_vals[x] = 0.0;
            } else {
                for (long long x = threadIdx.x; x < seg_nnz; x += NT) gacc[x] = 0.0;
            }
            __threadfence_block();
            __syncthreads();
            auto rank_of = [&](int col) {
                const int d = col - seg_lo;
                const int x = d >> 5;
                return (int)s_pfx[x] + __popc(s_bits[x] & ((1u << (d & 31)) - 1u));
            };
            if (in_lds) {
                wave_row_products<IdxT, T, true>(rs, nA, p.a_col, p.a_val, p.b_rp, p.b_col, w, NW, s_smask[w],
                                                 s_ebase[w], s_eval[w], dummy, [&](int col, int64_t bidx, double a) {
                                                     if (col >= seg_lo && col < seg_hi)
                                                         atomicAdd(&s_vals[rank_of(col)], a * (double)p.b_val[bidx]);
                                                 });
            } else {
                wave_row_products<IdxT, T, true>(rs, nA, p.a_col, p.a_val, p.b_rp, p.b_col, w, NW, s_smask[w],
                                                 s_ebase[w], s_eval[w], dummy, [&](int col, int64_t bidx, double a) {
                                                     if (col >= seg_lo && col < seg_hi)
                                                         atomicAdd(&gacc[rank_of(col)], a * (double)p.b_val[bidx]);
                                                 });
            }
            __threadfence_block();
            __syncthreads();
            for (int x = w0; x < w1; ++x) {
                uint32_t bw = s_bits[x];
                int64_t o = cb + off + s_pfx[x];
                while (bw) {
                    const int b = __ffs(bw) - 1;
                    bw &= bw - 1;
                    p.c_col[o++] = seg_lo + x * 32 + b;
                }
            }
            if (in_lds) {
                for (long long x = threadIdx.x; x < seg_nnz; x += NT) p.c_val[cb + off + x] = (T)s_vals[x];
            } else if constexpr (sizeof(T) != sizeof(double)) {
                for (long long x = threadIdx.x; x < seg_nnz; x += NT) p.c_val[cb + off + x] = (T)gacc[x];
            }
            off += seg_nnz;
            __syncthreads();
        }
    }
}

}  // namespace reap
