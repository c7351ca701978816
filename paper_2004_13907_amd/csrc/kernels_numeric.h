// Numeric pass: partial products a_ik * b_kj, their accumulation by column and
// the ascending-column write of each row of C (the multiply, sort and merge
// steps of the paper's Algorithm 1).  Sorting is replaced by ranking: a bitmap
// over the row's column window, with a prefix count per 32-bit word, gives
// every column its position in the sorted row directly.
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

// Loads the A entries of row i into the lanes of this wavefront and prepares
// the flattened product index space: smask marks where each non-empty B row
// starts, ebase[c] is the B index of product 0 of the c-th non-empty entry,
// aval[c] its A value.  Returns P_i (at most kWaveMaxProducts).
template <typename T, typename IdxT>
__device__ __forceinline__ int wave_row_setup(const IdxT* __restrict__ a_rp, const int32_t* __restrict__ a_col,
                                              const T* __restrict__ a_val, const IdxT* __restrict__ b_rp,
                                              int64_t i, uint32_t* smask, IdxT* ebase, double* aval,
                                              int smask_words) {
    const int lane = lane_id();
    const IdxT rs = a_rp[i];
    const int nA = (int)((int64_t)a_rp[i + 1] - (int64_t)rs);
    int64_t b0 = 0;
    int len = 0;
    double a = 0.0;
    if (lane < nA) {
        const int k = a_col[rs + lane];
        const IdxT x0 = b_rp[k];
        const IdxT x1 = b_rp[k + 1];
        b0 = (int64_t)x0;
        len = (int)((int64_t)x1 - (int64_t)x0);
        a = (double)a_val[rs + lane];
    }
    const int incl = wave_incl_scan_i32(len);
    const int P = uniform_i32(shfl(incl, kWave - 1));
    const int start = incl - len;
    const bool ne = len > 0;
    const int c = mbcnt(ballot(ne));
    if (lane < smask_words) smask[lane] = 0u;
    wave_sync();
    if (ne) {
        ebase[c] = (IdxT)(b0 - start);
        aval[c] = a;
        atomicOr(&smask[start >> 5], 1u << (start & 31));
    }
    wave_sync();
    return P;
}

// Rows of one wavefront class: each wavefront scans kRowsPerWave consecutive
// rows and processes those whose class is CLS, so rows stay in order and
// neighbouring rows (which share B rows) run close together on one XCD.
template <typename Fn>
__device__ __forceinline__ void for_each_class_row(const uint8_t* __restrict__ cls, int64_t m, int W,
                                                   uint8_t want, Fn&& fn) {
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int blk = xcd_contiguous_block(blockIdx.x, gridDim.x);
    const int64_t row0 = ((int64_t)blk * W + w) * kRowsPerWave;
    const bool mine = lane < kRowsPerWave && row0 + lane < m && cls[row0 + lane] == want;
    uint64_t todo = ballot(mine);
    while (todo) {
        const int r = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        fn(row0 + r);
    }
}

// ---------------------------------------------------------------------------
// One wavefront per row, bitmap window of at most WMAX words, at most NCMAX
// entries in the row of C.  Products are held in registers (16 per lane).
template <typename T, typename IdxT, typename IdxC, int NCMAX, int WMAX, int W>
__global__ void __launch_bounds__(W * 64) k_num_wave_bmp(NumArgs<T, IdxT, IdxC> p, uint8_t want) {
    __shared__ uint32_t s_bits[W][WMAX];
    __shared__ uint16_t s_pfx[W][WMAX];
    __shared__ double s_vals[W][NCMAX];
    __shared__ int32_t s_cols[W][NCMAX];
    __shared__ uint32_t s_smask[W][kWaveMaxProducts / 32];
    __shared__ IdxT s_ebase[W][kWave];
    __shared__ double s_aval[W][kWave];

    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    uint32_t* bits = s_bits[w];
    uint16_t* pfx = s_pfx[w];
    double* vals = s_vals[w];
    int32_t* cols_l = s_cols[w];

    for_each_class_row(p.cls, p.m, W, want, [&](int64_t i) {
        const int P = wave_row_setup<T, IdxT>(p.a_rp, p.a_col, p.a_val, p.b_rp, i, s_smask[w], s_ebase[w],
                                              s_aval[w], kWaveMaxProducts / 32);
        const int2 wn = p.win[i];
        const int lo = wn.x, nw = wn.y;
        const IdxC cb = p.c_rp[i];
        const int nc = (int)((int64_t)p.c_rp[i + 1] - (int64_t)cb);
        for (int x = lane; x < nw; x += kWave) bits[x] = 0u;
        for (int x = lane; x < nc; x += kWave) vals[x] = 0.0;
        wave_sync();
        const int nIt = (P + kWave - 1) / kWave;
        int cols[kWaveMaxIt];
        double prod[kWaveMaxIt];
        int seen = 0;
#pragma unroll
        for (int t = 0; t < kWaveMaxIt; ++t) {
            cols[t] = -1;
            prod[t] = 0.0;
            if (t < nIt) {
                const uint64_t M = ((uint64_t)s_smask[w][2 * t + 1] << 32) | s_smask[w][2 * t];
                const int own = seen + mbcnt(M) + (int)((M >> lane) & 1u) - 1;
                seen += __popcll(M);
                const int q = t * kWave + lane;
                if (q < P) {
                    const int64_t bidx = (int64_t)s_ebase[w][own] + q;
                    const int col = p.b_col[bidx];
                    prod[t] = s_aval[w][own] * (double)p.b_val[bidx];
                    cols[t] = col;
                    const int d = col - lo;
                    atomicOr(&bits[d >> 5], 1u << (d & 31));
                }
            }
        }
        wave_sync();
        // prefix count of set bits per word: lane l owns words [l*per, l*per + per)
        const int per = (nw + kWave - 1) / kWave;
        const int w0 = min(lane * per, nw), w1 = min(w0 + per, nw);
        int local = 0;
        for (int x = w0; x < w1; ++x) local += __popc(bits[x]);
        int run = wave_incl_scan_i32(local) - local;
        for (int x = w0; x < w1; ++x) {
            pfx[x] = (uint16_t)run;
            run += __popc(bits[x]);
        }
        wave_sync();
#pragma unroll
        for (int t = 0; t < kWaveMaxIt; ++t) {
            if (cols[t] >= 0) {
                const int d = cols[t] - lo;
                const int x = d >> 5;
                const int r = pfx[x] + __popc(bits[x] & ((1u << (d & 31)) - 1u));
                if (r < nc) {  // always true when the pattern matches the symbolic pass
                    atomicAdd(&vals[r], prod[t]);
                    cols_l[r] = cols[t];
                }
            }
        }
        wave_sync();
        for (int x = lane; x < nc; x += kWave) {
            p.c_col[(int64_t)cb + x] = cols_l[x];
            p.c_val[(int64_t)cb + x] = (T)vals[x];
        }
        wave_sync();
    });
}

// ---------------------------------------------------------------------------
// One wavefront per row whose column window is too wide for a bitmap (at most
// kWaveHashProducts products): LDS hash table keyed by column, then the
// occupied slots are compacted and each entry is placed by counting the
// smaller columns.
template <typename T, typename IdxT, typename IdxC, int W>
__global__ void __launch_bounds__(W * 64) k_num_wave_hash(NumArgs<T, IdxT, IdxC> p, uint8_t want) {
    __shared__ uint32_t s_keys[W][kWaveHashSlots];
    __shared__ double s_hv[W][kWaveHashSlots];
    __shared__ int32_t s_ck[W][kWaveHashProducts];
    __shared__ double s_cv[W][kWaveHashProducts];
    __shared__ uint32_t s_smask[W][kWaveHashProducts / 32];
    __shared__ IdxT s_ebase[W][kWave];
    __shared__ double s_aval[W][kWave];

    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    uint32_t* keys = s_keys[w];
    double* hv = s_hv[w];
    int32_t* ck = s_ck[w];
    double* cv = s_cv[w];
    constexpr uint32_t kEmpty = 0xFFFFFFFFu;

    for_each_class_row(p.cls, p.m, W, want, [&](int64_t i) {
        const int P = wave_row_setup<T, IdxT>(p.a_rp, p.a_col, p.a_val, p.b_rp, i, s_smask[w], s_ebase[w],
                                              s_aval[w], kWaveHashProducts / 32);
        const IdxC cb = p.c_rp[i];
        for (int x = lane; x < kWaveHashSlots; x += kWave) {
            keys[x] = kEmpty;
            hv[x] = 0.0;
        }
        wave_sync();
        const int nIt = (P + kWave - 1) / kWave;
        int seen = 0;
#pragma unroll
        for (int t = 0; t < kWaveHashIt; ++t) {
            if (t < nIt) {
                const uint64_t M = ((uint64_t)s_smask[w][2 * t + 1] << 32) | s_smask[w][2 * t];
                const int own = seen + mbcnt(M) + (int)((M >> lane) & 1u) - 1;
                seen += __popcll(M);
                const int q = t * kWave + lane;
                if (q < P) {
                    const int64_t bidx = (int64_t)s_ebase[w][own] + q;
                    const int col = p.b_col[bidx];
                    const double v = s_aval[w][own] * (double)p.b_val[bidx];
                    const uint32_t key = (uint32_t)col;
                    uint32_t h = hash_col(col) >> (32 - 9);
                    while (true) {
                        const uint32_t old = atomicCAS(&keys[h], kEmpty, key);
                        if (old == kEmpty || old == key) break;
                        h = (h + 1) & (kWaveHashSlots - 1);
                    }
                    atomicAdd(&hv[h], v);
                }
            }
        }
        wave_sync();
        int nc = 0;
        for (int x0 = 0; x0 < kWaveHashSlots; x0 += kWave) {
            const int x = x0 + lane;
            const bool occ = keys[x] != kEmpty;
            const uint64_t bm = ballot(occ);
            if (occ) {
                const int pos = nc + mbcnt(bm);
                ck[pos] = (int32_t)keys[x];
                cv[pos] = hv[x];
            }
            nc += __popcll(bm);
        }
        wave_sync();
        int key[kWaveHashIt];
        int rank[kWaveHashIt];
#pragma unroll
        for (int u = 0; u < kWaveHashIt; ++u) {
            const int e = u * kWave + lane;
            key[u] = (e < nc) ? ck[e] : INT32_MAX;
            rank[u] = 0;
        }
        for (int j = 0; j < nc; ++j) {
            const int kj = ck[j];
#pragma unroll
            for (int u = 0; u < kWaveHashIt; ++u) rank[u] += (kj < key[u]) ? 1 : 0;
        }
#pragma unroll
        for (int u = 0; u < kWaveHashIt; ++u) {
            const int e = u * kWave + lane;
            if (e < nc) {
                p.c_col[(int64_t)cb + rank[u]] = key[u];
                p.c_val[(int64_t)cb + rank[u]] = (T)cv[e];
            }
        }
        wave_sync();
    });
}

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
