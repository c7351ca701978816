// Long rows: rows of A with more than 64 entries or more partial products than
// a wavefront row holds (the paper splits such rows into fixed-size pieces so
// that no processing element stalls on one row; here a whole workgroup takes
// the row).  Both passes walk the row's products once per column segment: a
// segment is a window of up to kLongSegWords * 32 columns whose bitmap lives in
// LDS.  The symbolic pass counts set bits; the numeric pass also prefix-counts
// the bitmap words, so that the rank of a column (its position in the sorted
// row) is one LDS read and a popcount, and adds each product into that slot.
//
// Rows are taken from the batch's long-row list of (product, row) pairs with a
// grid-stride loop (entry j goes to workgroup j mod gridDim.x), so every loop
// bound is known when the row starts.
#pragma once
#include "device_utils.h"
#include "kernels_symbolic.h"
#include "kernels_numeric.h"
#include "spgemm_common.h"

namespace reap {

constexpr int kLongThreads = 512;
constexpr int kLongWaves = kLongThreads / kWave;
constexpr int kLongSegWords = 8192;  // 262144 columns per segment

// Per-wavefront table of one chunk of (at most 64) A entries.
template <typename IdxT>
struct LongChunk {
    IdxT b0[kWave];       // first B entry of the named B row
    int32_t len[kWave];   // its length when shorter than 64, else 0
    double a[kWave];      // the A value
};

// Calls fn(col, bidx, a) once for every partial product of the A row
// [rs, rs + nA) that this wavefront owns.  Wavefront w takes the chunks of 64
// entries starting at w*64, (w + nwaves)*64, ...  Entries whose B row has 64
// or more entries are walked by the whole wavefront, 64 consecutive B entries
// per step.  The other entries of the chunk are taken in groups of G lanes
// (G the smallest power of two not below the chunk's longest such B row):
// 64/G entries per step, lane `off` of a group reads B entry b0 + off.
template <typename IdxT, typename T, bool VALS, typename Fn>
__device__ __forceinline__ void long_row_products(IdxT rs, int64_t nA, const int32_t* __restrict__ a_col,
                                                  const T* __restrict__ a_val, const IdxT* __restrict__ b_rp,
                                                  const int32_t* __restrict__ b_col, int wave, int nwaves,
                                                  LongChunk<IdxT>& tb, Fn&& fn) {
    const int lane = lane_id();
    for (int64_t ch = (int64_t)wave * kWave; ch < nA; ch += (int64_t)nwaves * kWave) {
        const int cnt = (int)min((int64_t)kWave, nA - ch);
        IdxT b0 = 0;
        int64_t len = 0;
        double a = 0.0;
        if (lane < cnt) {
            const int k = a_col[rs + ch + lane];
            const IdxT x0 = b_rp[k];
            const IdxT x1 = b_rp[k + 1];
            b0 = x0;
            len = (int64_t)x1 - (int64_t)x0;
            if (VALS) a = (double)a_val[rs + ch + lane];
        }
        const bool lng = len >= kWave;
        const int slen = lng ? 0 : (int)len;
        const int maxs = wave_max_i32(slen);
        if (maxs > 0) {
            tb.b0[lane] = b0;
            tb.len[lane] = slen;
            if (VALS) tb.a[lane] = a;
            wave_sync();
            const int logG = maxs <= 1 ? 0 : 32 - __clz(maxs - 1);
            const int g = lane >> logG;
            const int off = lane & ((1 << logG) - 1);
            const int per = kWave >> logG;
            for (int e0 = 0; e0 < cnt; e0 += per) {
                const int e = e0 + g;
                if (e < cnt && off < tb.len[e]) {
                    const IdxT q = tb.b0[e] + (IdxT)off;
                    fn(b_col[q], (int64_t)q, VALS ? tb.a[e] : 0.0);
                }
            }
            wave_sync();
        }
        uint64_t lm = ballot(lng);
        while (lm) {
            const int e = __ffsll((unsigned long long)lm) - 1;
            lm &= lm - 1;
            const int64_t eb0 = (int64_t)shfl(b0, e);
            const int64_t elen = shfl(len, e);
            const double ea = VALS ? shfl(a, e) : 0.0;
            for (int64_t q = lane; q < elen; q += kWave) fn(b_col[eb0 + q], eb0 + q, ea);
        }
    }
}

// Partial products of the A row [rs, rs + nA): sum of its entries' B-row lengths.
template <typename IdxT>
__device__ __forceinline__ long long long_row_count(IdxT rs, int64_t nA, const int32_t* __restrict__ a_col,
                                                    const IdxT* __restrict__ b_rp, long long* s_red) {
    long long s = 0;
    for (int64_t e = threadIdx.x; e < nA; e += kLongThreads) {
        const int k = a_col[rs + e];
        s += (long long)b_rp[k + 1] - (long long)b_rp[k];
    }
    return block_sum_i64<kLongThreads>(s, s_red);
}

// ---------------------------------------------------------------------------
// Symbolic pass for the long-row list: nnz(C_i) and the column window of each
// long row.  The window is [0, n) when n fits one segment, else the row's
// [min column, max column] (one extra walk of the products).
template <typename IdxT>
__global__ void __launch_bounds__(kLongThreads) k_long_sym(SymArgs<IdxT> p0, const SymArgs<IdxT>* __restrict__ P,
                                                          BatchMap bm) {
    __shared__ uint32_t s_bits[kLongSegWords];
    __shared__ LongChunk<IdxT> s_tb[kLongWaves];
    __shared__ long long s_red[kLongWaves];
    __shared__ int s_redi[kLongWaves];

    const int w = threadIdx.x / kWave;
    const int nL = (int)*bm.n_long;
    for (int j = blockIdx.x; j < nL; j += gridDim.x) {
        const int2 ent = bm.long_list[j];
        const SymArgs<IdxT> p = P ? P[ent.x] : p0;
        const int seg_cols = p.th.group_lds_span;
        const int64_t i = ent.y;
        const IdxT rs = p.a_rp[i];
        const int64_t nA = (int64_t)p.a_rp[i + 1] - (int64_t)rs;
        const long long prods = long_row_count<IdxT>(rs, nA, p.a_col, p.b_rp, s_red);

        int lo = 0;
        int64_t span = p.n;
        if (p.n > seg_cols) {
            int cmin = INT32_MAX, cmax = -1;
            long_row_products<IdxT, float, false>(rs, nA, p.a_col, nullptr, p.b_rp, p.b_col, w, kLongWaves, s_tb[w],
                                                  [&](int col, int64_t, double) {
                                                      cmin = min(cmin, col);
                                                      cmax = max(cmax, col);
                                                  });
            cmin = block_min_i32<kLongThreads>(cmin, s_redi);
            cmax = block_max_i32<kLongThreads>(cmax, s_redi);
            lo = cmin;
            span = (cmax >= cmin) ? (int64_t)cmax - cmin + 1 : 0;
        }
        long long nnz = 0;
        for (int64_t s0 = 0; s0 < span; s0 += seg_cols) {
            const int seg_lo = lo + (int)s0;
            const int seg_w = (int)((min((int64_t)seg_cols, span - s0) + 31) >> 5);
            const int seg_hi = seg_lo + seg_w * 32;
            for (int x = threadIdx.x; x < seg_w; x += kLongThreads) s_bits[x] = 0u;
            __syncthreads();
            long_row_products<IdxT, float, false>(rs, nA, p.a_col, nullptr, p.b_rp, p.b_col, w, kLongWaves, s_tb[w],
                                                  [&](int col, int64_t, double) {
                                                      if (col >= seg_lo && col < seg_hi) {
                                                          const int d = col - seg_lo;
                                                          atomicOr(&s_bits[d >> 5], 1u << (d & 31));
                                                      }
                                                  });
            __syncthreads();
            long long pc = 0;
            for (int x = threadIdx.x; x < seg_w; x += kLongThreads) pc += __popc(s_bits[x]);
            nnz += block_sum_i64<kLongThreads>(pc, s_red);
        }
        if (threadIdx.x == 0) {
            p.rnnz[i] = (int32_t)nnz;
            p.win[i] = make_int2(lo, (int)span);
            atomicAdd(&p.ctr->products, (unsigned long long)prods);
            atomicMax(&p.ctr->max_prod, (unsigned)min(prods, (long long)UINT32_MAX));
            atomicMax(&p.ctr->max_nnz, (unsigned)nnz);
            atomicMax(&p.ctr->max_group_nnz, (unsigned)nnz);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Numeric pass for the long-row list.  Per segment of the row's window:
// (1) bitmap of the segment's columns, (2) prefix count of set bits per word
// (block scan), (3) the segment's slots are cleared and every product is added
// into the slot of its column's rank with a device-memory FP64 atomic (the
// row's own output for FP64; a per-workgroup FP64 buffer for FP32, rounded
// once on the copy out), (4) columns are written from the bitmap in ascending
// order.  Only this workgroup touches the row's slots during the kernel, so
// the atomics are workgroup-scoped.
template <typename T, typename IdxT, typename IdxC>
__global__ void __launch_bounds__(kLongThreads) k_long_num(NumArgs<T, IdxT, IdxC> p0,
                                                          const NumArgs<T, IdxT, IdxC>* __restrict__ P, BatchMap bm) {
    __shared__ uint32_t s_bits[kLongSegWords];
    __shared__ uint32_t s_pfx[kLongSegWords];
    __shared__ LongChunk<IdxT> s_tb[kLongWaves];
    __shared__ long long s_red[kLongWaves];

    const int w = threadIdx.x / kWave;
    const int nL = (int)*bm.n_long;
    for (int j = blockIdx.x; j < nL; j += gridDim.x) {
        const int2 ent = bm.long_list[j];
        const NumArgs<T, IdxT, IdxC> p = P ? P[ent.x] : p0;
        const int seg_cols = p.th.group_lds_span;
        const int64_t i = ent.y;
        const IdxT rs = p.a_rp[i];
        const int64_t nA = (int64_t)p.a_rp[i + 1] - (int64_t)rs;
        const int2 wn = p.win[i];
        const int lo = wn.x;
        const int64_t span = wn.y;
        const int64_t cb = (int64_t)p.c_rp[i];
        const int64_t nc_row = (int64_t)p.c_rp[i + 1] - cb;
        int64_t off = 0;
        for (int64_t s0 = 0; s0 < span; s0 += seg_cols) {
            const int seg_lo = lo + (int)s0;
            const int seg_w = (int)((min((int64_t)seg_cols, span - s0) + 31) >> 5);
            const int seg_hi = seg_lo + seg_w * 32;
            for (int x = threadIdx.x; x < seg_w; x += kLongThreads) s_bits[x] = 0u;
            __syncthreads();
            long_row_products<IdxT, T, false>(rs, nA, p.a_col, p.a_val, p.b_rp, p.b_col, w, kLongWaves, s_tb[w],
                                              [&](int col, int64_t, double) {
                                                  if (col >= seg_lo && col < seg_hi) {
                                                      const int d = col - seg_lo;
                                                      atomicOr(&s_bits[d >> 5], 1u << (d & 31));
                                                  }
                                              });
            __syncthreads();
            // thread t owns words [t*per, t*per + per)
            const int per = (seg_w + kLongThreads - 1) / kLongThreads;
            const int w0 = min((int)threadIdx.x * per, seg_w), w1 = min(w0 + per, seg_w);
            long long local = 0;
            for (int x = w0; x < w1; ++x) local += __popc(s_bits[x]);
            long long seg_nnz;
            long long run = block_excl_scan_i64<kLongThreads>(local, s_red, &seg_nnz);
            for (int x = w0; x < w1; ++x) {
                s_pfx[x] = (uint32_t)run;
                run += __popc(s_bits[x]);
            }
            if (off + seg_nnz > nc_row) {  // pattern differs from the symbolic pass
                if (threadIdx.x == 0) atomicOr(&p.ctr->bad_csr, 4u);
                break;
            }
            double* acc;
            if constexpr (sizeof(T) == sizeof(double)) {
                acc = reinterpret_cast<double*>(p.c_val) + cb + off;
            } else {
                acc = p.gvals + (int64_t)blockIdx.x * p.gvals_stride;
            }
            for (long long x = threadIdx.x; x < seg_nnz; x += kLongThreads) acc[x] = 0.0;
            __threadfence_block();
            __syncthreads();
            long_row_products<IdxT, T, true>(rs, nA, p.a_col, p.a_val, p.b_rp, p.b_col, w, kLongWaves, s_tb[w],
                                             [&](int col, int64_t bidx, double a) {
                                                 if (col >= seg_lo && col < seg_hi) {
                                                     const int d = col - seg_lo;
                                                     const int x = d >> 5;
                                                     const int rk = (int)s_pfx[x] +
                                                                    __popc(s_bits[x] & ((1u << (d & 31)) - 1u));
                                                     __hip_atomic_fetch_add(&acc[rk], a * (double)p.b_val[bidx],
                                                                            __ATOMIC_RELAXED,
                                                                            __HIP_MEMORY_SCOPE_WORKGROUP);
                                                 }
                                             });
            for (int x = w0; x < w1; ++x) {
                uint32_t bw = s_bits[x];
                int64_t o = cb + off + s_pfx[x];
                while (bw) {
                    const int b = __ffs(bw) - 1;
                    bw &= bw - 1;
                    p.c_col[o++] = seg_lo + x * 32 + b;
                }
            }
            if constexpr (sizeof(T) != sizeof(double)) {
                // the adds of every wavefront must be complete and visible
                // before the buffer is read back (and L1 holds no stale copy)
                __threadfence();
                __syncthreads();
                for (long long x = threadIdx.x; x < seg_nnz; x += kLongThreads) p.c_val[cb + off + x] = (T)acc[x];
            }
            off += seg_nnz;
            __threadfence();
            __syncthreads();
        }
    }
}

}  // namespace reap
