// Long rows: rows of A with more than 64 entries or more partial products than
// a wavefront row holds (the paper splits such rows into fixed-size pieces so
// that no processing element stalls on one row; here a whole workgroup takes
// the row).  Both passes walk the row's products once per column segment: a
// segment is a window of up to kLongSegWords * 32 columns whose bitmap lives in
// LDS.  The symbolic pass counts set bits; the numeric pass also prefix-counts
// the bitmap words, so that the rank of a column (its position in the sorted
// row) is one LDS read and a popcount, and adds each product into that slot.
//
// Rows are taken from the batch's long-row list of (product, row) pairs
// through a device counter (each workgroup takes the next unprocessed entry
// when it finishes one), so a few heavy rows do not hold back the workgroups
// that were handed them together with many others.
#pragma once
#include "device_utils.h"
#include "kernels_symbolic.h"
#include "kernels_numeric.h"
#include "spgemm_common.h"

namespace reap {

constexpr int kLongThreads = 512;       // symbolic pass
constexpr int kLongWaves = kLongThreads / kWave;
constexpr int kLongNumThreads = 1024;   // numeric pass (one workgroup per CU: its LDS is ~150 KB)
constexpr int kLongNumWaves = kLongNumThreads / kWave;
constexpr int kLongSegWords = 8192;     // 262144 columns per window segment
constexpr int kLongVals = 8192;         // numeric: FP64 accumulator slots in LDS
constexpr int kLongMinVals = 256;       // smallest rank chunk accepted
constexpr int kLongMaxChunks = kLongSegWords * 32 / kLongMinVals;
constexpr unsigned kUnsortedB = 8u;     // Counters::bad_csr bit: a B row read by a long row is not in column order

// Per-wavefront table of one chunk of (at most 64) A entries.
template <typename IdxT>
struct LongChunk {
    IdxT b0[kWave];       // first B entry of the named B row
    int32_t len[kWave];   // its length when shorter than 64, else 0
    double a[kWave];      // the A value
};

// Calls fn(col, v) once for every partial product of the A row [rs, rs + nA)
// that this wavefront owns, v = a_ik * b_kj in FP64 (0 when !VALS).
// Wavefront w takes the chunks of 64 entries starting at w*64,
// (w + nwaves)*64, ...  Entries whose B row has 64 or more entries are walked
// by the whole wavefront, 256 consecutive B entries per step (four loads of
// column and value in flight per lane before any is used).  The other
// entries of the chunk are taken in groups of G lanes (G the smallest power
// of two not below the chunk's longest such B row): 64/G entries per step,
// lane `off` of a group reads B entry b0 + off.  CHECK sets *unsorted when a
// B row is not in ascending column order.
template <typename IdxT, typename T, bool VALS, bool CHECK = false, typename Fn>
__device__ __forceinline__ void long_row_products(IdxT rs, int64_t nA, const int32_t* __restrict__ a_col,
                                                  const T* __restrict__ a_val, const IdxT* __restrict__ b_rp,
                                                  const int32_t* __restrict__ b_col, const T* __restrict__ b_val,
                                                  int wave, int nwaves, LongChunk<IdxT>& tb, Fn&& fn,
                                                  bool* unsorted = nullptr) {
    constexpr int U = 4;
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
            // two steps per trip: the loads of both are issued before either is used
            for (int e0 = 0; e0 < cnt; e0 += 2 * per) {
                int c[2];
                T bv[2];
                bool on[2];
                int ei[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int e = e0 + u * per + g;
                    ei[u] = e;
                    on[u] = e < cnt && off < tb.len[e];
                    c[u] = -1;
                    bv[u] = T(0);
                    if (on[u]) {
                        const IdxT q = tb.b0[e] + (IdxT)off;
                        c[u] = b_col[q];
                        if (VALS) bv[u] = b_val[q];
                    }
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    if (CHECK) {
                        // lane - 1 holds the previous entry of the same B row when off > 0
                        const int prev = __shfl_up(c[u], 1, kWave);
                        if (on[u] && off > 0 && prev > c[u]) *unsorted = true;
                    }
                    if (on[u]) fn(c[u], VALS ? tb.a[ei[u]] * (double)bv[u] : 0.0);
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
            int last = INT32_MIN;  // CHECK: column of the entry before this step's first
            for (int64_t q0 = 0; q0 < elen; q0 += U * kWave) {
                int c[U];
                T bv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t q = q0 + u * kWave + lane;
                    c[u] = -1;
                    bv[u] = T(0);
                    if (q < elen) {
                        c[u] = b_col[eb0 + q];
                        if (VALS) bv[u] = b_val[eb0 + q];
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (CHECK) {
                        int prev = __shfl_up(c[u], 1, kWave);
                        if (lane == 0) prev = last;
                        if (c[u] >= 0 && prev > c[u]) *unsorted = true;
                        last = __shfl(c[u], kWave - 1, kWave);
                    }
                    if (c[u] >= 0) fn(c[u], VALS ? ea * (double)bv[u] : 0.0);
                }
            }
        }
    }
}

// Walks a B row stored in column order (entries [0, elen) of col/val) from
// entry qlo, U steps of 64 entries at a time, calling fn(col, a * val) for
// the entries with columns in [clo, chi); stops after the step in which a
// column reaches chi or the row ends.
template <int U, typename T, typename Fn>
__device__ __forceinline__ void chunk_walk(const int32_t* __restrict__ col, const T* __restrict__ val, int64_t qlo,
                                           int64_t elen, int clo, int chi, double a, int lane, Fn&& fn) {
    for (int64_t base = qlo; base < elen; base += U * kWave) {
        int c[U];
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = base + u * kWave + lane;
            c[u] = INT32_MAX;
            v[u] = T(0);
            if (q < elen) {
                c[u] = col[q];
                v[u] = val[q];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (c[u] >= clo && c[u] < chi) fn(c[u], a * (double)v[u]);
        if (ballot(c[U - 1] < chi) != ~0ull) break;
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
    __shared__ int s_next;

    const int w = threadIdx.x / kWave;
    const int nL = (int)*bm.n_long;
    if (nL == 0) return;   // the usual case on regular inputs: leave before touching the queue
    for (;;) {
        if (threadIdx.x == 0) s_next = (int)atomicAdd(&bm.queue[0], 1u);
        __syncthreads();
        const int j = s_next;
        if (j >= nL) break;
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
            long_row_products<IdxT, float, false>(rs, nA, p.a_col, nullptr, p.b_rp, p.b_col, nullptr, w, kLongWaves,
                                                  s_tb[w], [&](int col, double) {
                                                      cmin = min(cmin, col);
                                                      cmax = max(cmax, col);
                                                  });
            cmin = block_min_i32<kLongThreads>(cmin, s_redi);
            cmax = block_max_i32<kLongThreads>(cmax, s_redi);
            lo = cmin;
            span = (cmax >= cmin) ? (int64_t)cmax - cmin + 1 : 0;
        }
        long long nnz = 0;
        bool unsorted = false;
        for (int64_t s0 = 0; s0 < span; s0 += seg_cols) {
            const int seg_lo = lo + (int)s0;
            const int seg_w = (int)((min((int64_t)seg_cols, span - s0) + 31) >> 5);
            const int seg_hi = seg_lo + seg_w * 32;
            for (int x = threadIdx.x; x < seg_w; x += kLongThreads) s_bits[x] = 0u;
            __syncthreads();
            long_row_products<IdxT, float, false, true>(
                rs, nA, p.a_col, nullptr, p.b_rp, p.b_col, nullptr, w, kLongWaves, s_tb[w],
                [&](int col, double) {
                    if (col >= seg_lo && col < seg_hi) {
                        const int d = col - seg_lo;
                        atomicOr(&s_bits[d >> 5], 1u << (d & 31));
                    }
                },
                &unsorted);
            __syncthreads();
            long long pc = 0;
            for (int x = threadIdx.x; x < seg_w; x += kLongThreads) pc += __popc(s_bits[x]);
            nnz += block_sum_i64<kLongThreads>(pc, s_red);
        }
        if (p.n <= seg_cols && span > 0) {
            // one segment from column 0: narrow the window to the set bits
            // (the numeric pass then zeroes, scans and emits fewer words)
            const int seg_w = (int)((span + 31) >> 5);
            int cmin = INT32_MAX, cmax = -1;
            for (int x = threadIdx.x; x < seg_w; x += kLongThreads) {
                const uint32_t bw = s_bits[x];
                if (bw) {
                    cmin = min(cmin, x * 32 + __ffs(bw) - 1);
                    cmax = max(cmax, x * 32 + 31 - __clz(bw));
                }
            }
            cmin = block_min_i32<kLongThreads>(cmin, s_redi);
            cmax = block_max_i32<kLongThreads>(cmax, s_redi);
            lo = cmax >= 0 ? cmin : 0;
            span = cmax >= 0 ? (int64_t)cmax - cmin + 1 : 0;
        }
        // the numeric pass walks the B rows of long rows in column order only
        // when they are stored that way
        if (ballot(unsorted) && lane_id() == 0) atomicOr(&p.ctr->bad_csr, kUnsortedB);
        if (threadIdx.x == 0) {
            p.rnnz[i] = (int32_t)nnz;
            p.win[i] = make_int2(lo, (int)span);
            if (nnz) atomicAdd(&p.tiles[i / kScanTile], (unsigned long long)nnz);
            atomicAdd(&p.ctr->products, (unsigned long long)prods);
            atomicMax(&p.ctr->max_prod, (unsigned)min(prods, (long long)UINT32_MAX));
            atomicMax(&p.ctr->max_nnz, (unsigned)nnz);
            atomicMax(&p.ctr->max_group_nnz, (unsigned)nnz);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Numeric pass for the long-row list, one workgroup of 1024 threads per row.
// Per segment of the row's window (up to 262144 columns): (1) bitmap of the
// segment's columns, (2) prefix count of set bits per word (block scan), so
// the rank of a column -- its position in the sorted row -- is one LDS read
// and a popcount, (3) accumulation by rank, (4) columns written from the
// bitmap in ascending order.  Accumulation:
//  - a segment with at most V = group_lds_values (<= 8192) entries is summed
//    in LDS in one walk of the products;
//  - a larger segment is cut into nch chunks of V consecutive ranks (a column
//    range each).  If the long B rows are in column order (checked by the
//    symbolic pass), each chunk is summed in LDS and written to C: every lane
//    binary-searches where the chunk's column range starts in its A entry's
//    B row; rows averaging fewer than 64 entries per chunk are then walked by
//    their own lane, longer ones by the whole wavefront, until the range ends;
//  - if a long B row is not in column order, every product of the segment is
//    added with FP64 atomics into device memory: C's own values for FP64, a
//    per-workgroup FP64 buffer for FP32 (rounded once on the copy out).  Only
//    this workgroup touches those slots, so the atomics are workgroup-scoped.
template <typename T, typename IdxT, typename IdxC>
__global__ void __launch_bounds__(kLongNumThreads) k_long_num(NumArgs<T, IdxT, IdxC> p0,
                                                             const NumArgs<T, IdxT, IdxC>* __restrict__ P,
                                                             BatchMap bm) {
    constexpr int NT = kLongNumThreads, NW = kLongNumWaves;
    __shared__ uint32_t s_bits[kLongSegWords];
    __shared__ uint32_t s_pfx[kLongSegWords];
    __shared__ double s_vals[kLongVals];
    __shared__ LongChunk<IdxT> s_tb[NW];
    __shared__ long long s_red[NW];
    __shared__ int s_bound[kLongMaxChunks + 1];
    __shared__ int s_next;

    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int nL = (int)*bm.n_long;
    for (;;) {
        if (threadIdx.x == 0) s_next = (int)atomicAdd(&bm.queue[1], 1u);
        __syncthreads();
        const int j = s_next;
        if (j >= nL) break;
        const int2 ent = bm.long_list[j];
        const NumArgs<T, IdxT, IdxC> p = P ? P[ent.x] : p0;
        const int seg_cols = p.th.group_lds_span;
        const int V = min(max(p.th.group_lds_values, kLongMinVals), kLongVals);
        const bool sorted_b = (p.ctr->bad_csr & kUnsortedB) == 0u;
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
            for (int x = threadIdx.x; x < seg_w; x += NT) s_bits[x] = 0u;
            __syncthreads();
            long_row_products<IdxT, T, false>(rs, nA, p.a_col, p.a_val, p.b_rp, p.b_col, p.b_val, w, NW, s_tb[w],
                                              [&](int col, double) {
                                                  if (col >= seg_lo && col < seg_hi) {
                                                      const int d = col - seg_lo;
                                                      atomicOr(&s_bits[d >> 5], 1u << (d & 31));
                                                  }
                                              });
            __syncthreads();
            // thread t owns words [t*per, t*per + per)
            const int per = (seg_w + NT - 1) / NT;
            const int w0 = min((int)threadIdx.x * per, seg_w), w1 = min(w0 + per, seg_w);
            long long local = 0;
            for (int x = w0; x < w1; ++x) local += __popc(s_bits[x]);
            long long seg_nnz_ll;
            long long run = block_excl_scan_i64<NT>(local, s_red, &seg_nnz_ll);
            for (int x = w0; x < w1; ++x) {
                s_pfx[x] = (uint32_t)run;
                run += __popc(s_bits[x]);
            }
            if (off + seg_nnz_ll > nc_row) {  // pattern differs from the symbolic pass
                if (threadIdx.x == 0) atomicOr(&p.ctr->bad_csr, 4u);
                break;
            }
            const int seg_nnz = (int)seg_nnz_ll;
            auto rank_of = [&](int col) {
                const int d = col - seg_lo;
                const int x = d >> 5;
                return (int)s_pfx[x] + __popc(s_bits[x] & ((1u << (d & 31)) - 1u));
            };
            if (threadIdx.x == 0)
                atomicAdd(seg_nnz <= V ? &p.ctr->seg_lds : (sorted_b ? &p.ctr->seg_chunked : &p.ctr->seg_device), 1u);
            if (seg_nnz <= V) {
                // the whole segment in LDS
                for (int x = threadIdx.x; x < seg_nnz; x += NT) s_vals[x] = 0.0;
                __syncthreads();
                long_row_products<IdxT, T, true>(rs, nA, p.a_col, p.a_val, p.b_rp, p.b_col, p.b_val, w, NW, s_tb[w],
                                                 [&](int col, double v) {
                                                     if (col >= seg_lo && col < seg_hi)
                                                         atomicAdd(&s_vals[rank_of(col)], v);
                                                 });
                __syncthreads();
                for (int x = threadIdx.x; x < seg_nnz; x += NT) p.c_val[cb + off + x] = (T)s_vals[x];
            } else if (sorted_b) {
                // rank chunks, each summed in LDS and written to C as it completes
                const int nch = (seg_nnz + V - 1) / V;
                // column boundaries of the chunks: chunk c holds ranks [cV, cV + V),
                // columns [s_bound[c], s_bound[c + 1])
                if (threadIdx.x == 0) {
                    s_bound[0] = seg_lo;
                    s_bound[nch] = seg_hi;
                }
                for (int x = w0; x < w1; ++x) {
                    const int r0 = (int)s_pfx[x];
                    const uint32_t bw = s_bits[x];
                    const int c = __popc(bw);
                    // every multiple of V in [r0, r0 + c) but 0
                    for (int k = max(1, (r0 + V - 1) / V); k * V < r0 + c; ++k) {
                        uint32_t m = bw;
                        for (int t = k * V - r0; t > 0; --t) m &= m - 1;  // drop the lower set bits
                        s_bound[k] = seg_lo + x * 32 + (__ffs(m) - 1);
                    }
                }
                __syncthreads();
                for (int c = 0; c < nch; ++c) {
                    const int clo = s_bound[c], chi = s_bound[c + 1];
                    const int r0 = c * V, rn = min(V, seg_nnz - r0);
                    for (int x = threadIdx.x; x < rn; x += NT) s_vals[x] = 0.0;
                    __syncthreads();
                    auto add = [&](int col, double v) { atomicAdd(&s_vals[rank_of(col) - r0], v); };
                    for (int64_t ch = (int64_t)w * kWave; ch < nA; ch += (int64_t)NW * kWave) {
                        const int cnt = (int)min((int64_t)kWave, nA - ch);
                        int64_t b0 = 0, len = 0;
                        double a = 0.0;
                        if (lane < cnt) {
                            const int k = p.a_col[rs + ch + lane];
                            const IdxT x0 = p.b_rp[k];
                            b0 = (int64_t)x0;
                            len = (int64_t)p.b_rp[k + 1] - (int64_t)x0;
                            a = (double)p.a_val[rs + ch + lane];
                        }
                        // every lane finds where the chunk's column range starts in its
                        // own B row (binary search, the 64 searches side by side)
                        int64_t cur = 0;
                        {
                            int64_t hi = len;
                            while (cur < hi) {
                                const int64_t mid = (cur + hi) >> 1;
                                if (p.b_col[b0 + mid] < clo) cur = mid + 1; else hi = mid;
                            }
                        }
                        // B rows averaging fewer than 64 entries per chunk: each lane
                        // walks its own row until the range ends, four entries per
                        // step (their loads issued together; in a sorted row the
                        // entries below chi are a prefix of the four)
                        const bool heavy = len >= (int64_t)kWave * nch;
                        bool act = !heavy && cur < len;
                        while (ballot(act)) {
                            if (act) {
                                int c4[4];
                                T v4[4];
#pragma unroll
                                for (int u = 0; u < 4; ++u) {
                                    c4[u] = INT32_MAX;
                                    v4[u] = T(0);
                                    if (cur + u < len) {
                                        c4[u] = p.b_col[b0 + cur + u];
                                        v4[u] = p.b_val[b0 + cur + u];
                                    }
                                }
                                int taken = 0;
#pragma unroll
                                for (int u = 0; u < 4; ++u) {
                                    if (c4[u] < chi) {
                                        add(c4[u], a * (double)v4[u]);
                                        ++taken;
                                    }
                                }
                                cur += taken;
                                act = taken == 4 && cur < len;
                            }
                        }
                        // the others: the whole wavefront walks one row at a time, with
                        // four, two or one 64-entry steps of loads in flight as the row
                        // averages >= 256, >= 128 or fewer entries per chunk
                        uint64_t hm = ballot(heavy);
                        while (hm) {
                            const int e = __ffsll((unsigned long long)hm) - 1;
                            hm &= hm - 1;
                            const int64_t eb0 = shfl(b0, e);
                            const int64_t elen = shfl(len, e);
                            const int64_t q0 = shfl(cur, e);
                            const double ea = shfl(a, e);
                            if (elen >= 256 * (int64_t)nch)
                                chunk_walk<4, T>(p.b_col + eb0, p.b_val + eb0, q0, elen, clo, chi, ea, lane, add);
                            else if (elen >= 128 * (int64_t)nch)
                                chunk_walk<2, T>(p.b_col + eb0, p.b_val + eb0, q0, elen, clo, chi, ea, lane, add);
                            else
                                chunk_walk<1, T>(p.b_col + eb0, p.b_val + eb0, q0, elen, clo, chi, ea, lane, add);
                        }
                    }
                    __syncthreads();
                    for (int x = threadIdx.x; x < rn; x += NT) p.c_val[cb + off + r0 + x] = (T)s_vals[x];
                    __syncthreads();
                }
            } else {
                // a long B row out of column order: every product into device memory
                double* acc;
                if constexpr (sizeof(T) == sizeof(double)) {
                    acc = (double*)(p.c_val + cb + off);
                } else {
                    acc = p.gvals + (int64_t)blockIdx.x * p.gvals_stride;
                }
                for (int x = threadIdx.x; x < seg_nnz; x += NT) acc[x] = 0.0;
                __threadfence_block();
                __syncthreads();
                long_row_products<IdxT, T, true>(rs, nA, p.a_col, p.a_val, p.b_rp, p.b_col, p.b_val, w, NW, s_tb[w],
                                                 [&](int col, double v) {
                                                     if (col >= seg_lo && col < seg_hi)
                                                         __hip_atomic_fetch_add(&acc[rank_of(col)], v,
                                                                                __ATOMIC_RELAXED,
                                                                                __HIP_MEMORY_SCOPE_WORKGROUP);
                                                 });
                if constexpr (sizeof(T) != sizeof(double)) {
                    // the adds of every wavefront are complete before the buffer is read
                    // back (all of the workgroup's accesses go through one CU, so a
                    // workgroup-scope fence is enough: an agent-scope one would write
                    // back and invalidate the whole L2 of the XCD, per row)
                    __threadfence_block();
                    __syncthreads();
                    for (int x = threadIdx.x; x < seg_nnz; x += NT) p.c_val[cb + off + x] = (T)acc[x];
                }
            }
            for (int x = w0; x < w1; ++x) {
                uint32_t bw = s_bits[x];
                int64_t o = cb + off + s_pfx[x];
                while (bw) {
                    const int b = __ffs(bw) - 1;
                    bw &= bw - 1;
                    p.c_col[o++] = seg_lo + x * 32 + b;
                }
            }
            off += seg_nnz;
            __syncthreads();
        }
    }
}

// Rewinds the numeric pass's long-row counter (a kernel, so that the
// sequence can be captured in a graph).
__global__ void k_long_rewind(unsigned int* queue) {
    if (threadIdx.x == 0) queue[1] = 0u;
}

}  // namespace reap
