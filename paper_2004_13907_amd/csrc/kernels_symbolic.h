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
    const IdxT* a_rp;
    const int32_t* a_col;
    const IdxT* b_rp;
    const int32_t* b_col;
    uint8_t* cls;              // [m] row class
    int32_t* rnnz;             // [m] nnz of each row of C
    int2* win;                 // [m] {lo, words} bitmap window of wavefront rows; {lo, span} of long rows
    int32_t* group_rows;       // [m] list of long rows
    Counters* ctr;
    WGPart* parts;             // [gridDim.x] per-workgroup statistics
    Thresholds th;
};

// ---------------------------------------------------------------------------
// Enumerates the partial products of one row of A for one wavefront of a
// workgroup.  The row's A entries are taken in chunks of 64 (chunk = wave,
// wave + nwaves, ...).  Inside a chunk, entries whose B row is shorter than 64
// are flattened over the lanes (a bit mask of segment starts in LDS gives each
// lane its owner entry); entries with a B row of 64 or more are walked by the
// whole wavefront, 64 consecutive B entries at a time.  fn(col, bidx, a) is
// called once per partial product with the B entry index and, when VALS, the
// A value promoted to double (0 otherwise).  Lane 0 of each wavefront adds the
// wavefront's products to `products` (summed over the block, that is P_i).
template <typename IdxT, typename T, bool VALS, typename Fn>
__device__ __forceinline__ void wave_row_products(const IdxT rs, const int64_t nA,
                                                  const int32_t* __restrict__ a_col,
                                                  const T* __restrict__ a_val,
                                                  const IdxT* __restrict__ b_rp,
                                                  const int32_t* __restrict__ b_col,
                                                  int wave, int nwaves, uint32_t* smask,
                                                  int64_t* ebase, double* eval,
                                                  long long& products, Fn&& fn) {
    const int lane = lane_id();
    for (int64_t ch = (int64_t)wave * kWave; ch < nA; ch += (int64_t)nwaves * kWave) {
        const int cnt = (int)min((int64_t)kWave, nA - ch);
        int64_t b0 = 0, len = 0;
        double a = 0.0;
        if (lane < cnt) {
            const int k = a_col[rs + ch + lane];
            const IdxT x0 = b_rp[k];
            const IdxT x1 = b_rp[k + 1];
            b0 = (int64_t)x0;
            len = (int64_t)x1 - (int64_t)x0;
            if (VALS) a = (double)a_val[rs + ch + lane];
        }
        const long long chunk_products = wave_sum_i64(len);
        if (lane == 0) products += chunk_products;  // one contribution per wavefront
        const bool is_long = len >= kWave;
        const int slen = is_long ? 0 : (int)len;
        const int incl = wave_incl_scan_i32(slen);
        const int Ps = uniform_i32(shfl(incl, kWave - 1));
        if (Ps > 0) {
            const int start = incl - slen;
            const bool ne = slen > 0;
            const int c = mbcnt(ballot(ne));
            const int nmw = 2 * ((Ps + kWave - 1) / kWave);  // <= 126 words
            for (int x = lane; x < nmw; x += kWave) smask[x] = 0u;
            wave_sync();
            if (ne) {
                ebase[c] = b0 - start;
                if (VALS) eval[c] = a;
                atomicOr(&smask[start >> 5], 1u << (start & 31));
            }
            wave_sync();
            int seen = 0;
            for (int base = 0; base < Ps; base += kWave) {
                const int t = base >> 6;
                const uint64_t M = ((uint64_t)smask[2 * t + 1] << 32) | smask[2 * t];
                const int own = seen + mbcnt(M) + (int)((M >> lane) & 1u) - 1;
                seen += __popcll(M);
                const int q = base + lane;
                if (q < Ps) {
                    const int64_t bidx = ebase[own] + q;
                    fn(b_col[bidx], bidx, VALS ? eval[own] : 0.0);
                }
            }
            wave_sync();
        }
        uint64_t lm = ballot(is_long);
        while (lm) {
            const int e = __ffsll((unsigned long long)lm) - 1;
            lm &= lm - 1;
            const int64_t eb0 = shfl(b0, e);
            const int64_t elen = shfl(len, e);
            const double ea = VALS ? shfl(a, e) : 0.0;
            for (int64_t q = lane; q < elen; q += kWave) {
                const int64_t bidx = eb0 + q;
                fn(b_col[bidx], bidx, ea);
            }
        }
    }
}

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
// Long rows: one workgroup per row, rows taken from the long-row list by an
// atomic work counter (their sizes vary by orders of magnitude).  The column
// window [lo, lo + span) is [0, n) when n fits the LDS bitmap, otherwise the
// row's [min, max].  The window is cut into segments of th.group_lds_span
// columns; each segment is counted with an LDS bitmap (products re-gathered
// per segment, so no device scratch is needed).
template <typename IdxT>
__global__ void __launch_bounds__(512) k_sym_group(SymArgs<IdxT> p) {
    constexpr int NT = 512, NW = NT / kWave;
    __shared__ uint32_t s_bits[kGroupBitsWords];
    __shared__ uint32_t s_smask[NW][kGroupMaskWords];
    __shared__ int64_t s_ebase[NW][kWave];
    __shared__ long long s_red[NW];
    __shared__ int s_redi[NW];
    __shared__ int s_row;

    const int w = threadIdx.x / kWave;
    const int nG = (int)p.ctr->n_group;
    for (;;) {
        if (threadIdx.x == 0) s_row = (int)atomicAdd(&p.ctr->group_next, 1u);
        __syncthreads();
        const int j = s_row;
        __syncthreads();
        if (j >= nG) break;
        const int64_t i = p.group_rows[j];
        const IdxT rs = p.a_rp[i];
        const int64_t nA = (int64_t)p.a_rp[i + 1] - (int64_t)rs;

        int lo = 0;
        int64_t span = p.n;
        long long prods = 0;
        if (p.n > p.th.group_lds_span) {
            int cmin = INT32_MAX, cmax = -1;
            wave_row_products<IdxT, float, false>(rs, nA, p.a_col, nullptr, p.b_rp, p.b_col, w, NW,
                                                  s_smask[w], s_ebase[w], nullptr, prods,
                                                  [&](int col, int64_t, double) {
                                        cmin = min(cmin, col);
                                        cmax = max(cmax, col);
                                    });
            cmin = block_min_i32<NT>(cmin, s_redi);
            cmax = block_max_i32<NT>(cmax, s_redi);
            lo = cmin;
            span = (cmax >= cmin) ? (int64_t)cmax - cmin + 1 : 0;
        }
        long long nnz = 0;
        for (int64_t s0 = 0; s0 < span; s0 += p.th.group_lds_span) {
            const int seg_lo = lo + (int)s0;
            const int seg_w = (int)((min((int64_t)p.th.group_lds_span, span - s0) + 31) >> 5);
            const int seg_hi = seg_lo + seg_w * 32;  // exclusive (may exceed the window)
            for (int x = threadIdx.x; x < seg_w; x += NT) s_bits[x] = 0u;
            __syncthreads();
            long long pr = 0;
            wave_row_products<IdxT, float, false>(rs, nA, p.a_col, nullptr, p.b_rp, p.b_col, w, NW,
                                                  s_smask[w], s_ebase[w], nullptr, pr,
                                                  [&](int col, int64_t, double) {
                                        if (col >= seg_lo && col < seg_hi) {
                                            const int d = col - seg_lo;
                                            atomicOr(&s_bits[d >> 5], 1u << (d & 31));
                                        }
                                    });
            if (s0 == 0 && p.n <= p.th.group_lds_span) prods = pr;
            __syncthreads();
            long long pc = 0;
            for (int x = threadIdx.x; x < seg_w; x += NT) pc += __popc(s_bits[x]);
            nnz += block_sum_i64<NT>(pc, s_red);
        }
        const long long tot_prod = block_sum_i64<NT>(prods, s_red);
        if (threadIdx.x == 0) {
            p.rnnz[i] = (int32_t)nnz;
            p.win[i] = make_int2(lo, (int)span);
            atomicAdd(&p.ctr->products, (unsigned long long)tot_prod);
            atomicMax(&p.ctr->max_prod, (unsigned)min(tot_prod, (long long)UINT32_MAX));
            atomicMax(&p.ctr->max_nnz, (unsigned)nnz);
            atomicMax(&p.ctr->max_group_nnz, (unsigned)nnz);
        }
    }
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
