// Long rows: rows of A with more than 64 entries or more partial products than
// a wavefront row holds (the paper splits such rows into fixed-size pieces so
// that no processing element stalls on one row; here a whole workgroup takes
// the row and cuts its products into equal pieces for its wavefronts).  Both
// passes walk the row's products once per column segment: a segment is a
// window of up to kLongSegWords * 32 columns whose bitmap lives in LDS.  The
// symbolic pass counts set bits; the numeric pass also prefix-counts the
// bitmap words, so that the rank of a column (its position in the sorted row)
// is one LDS read and a popcount, and adds each product into that slot.
//
// Flattened walks.  The products of a row form one index space: A entry e
// (thread e of the workgroup holds it) covers the products
// [pre[e], pre[e + 1]), pre being the exclusive prefix sum of the lengths of
// the B rows the entries name.  Each wavefront takes steps of 64 * kFlatU
// consecutive products and each lane kFlatU consecutive ones of a step; a
// lane finds the entry of its first product by a binary search over pre in
// LDS and moves to the next entry when its run crosses one.  Every wavefront
// of the workgroup thus gets the same share of the row whatever the lengths
// of its B rows (a row of A·Aᵀ on a power-law matrix typically has a dozen
// entries, some naming B rows of tens of thousands of entries).  Rows with
// more entries than the workgroup has threads are taken in blocks of that
// many entries.
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
constexpr int kLongNumThreads = 1024;   // numeric pass (one workgroup per CU: its LDS is ~156 KB)
constexpr int kLongNumWaves = kLongNumThreads / kWave;
constexpr int kLongSegWords = 8192;     // 262144 columns per window segment
constexpr int kLongVals = 8192;         // numeric: FP64 accumulator slots in LDS
constexpr int kLongMinVals = 256;       // smallest rank chunk accepted
constexpr int kLongMaxChunks = kLongSegWords * 32 / kLongMinVals;
constexpr int kFlatU = 4;               // consecutive products per lane and step of a flattened walk
constexpr unsigned kUnsortedB = 8u;     // Counters::bad_csr bit: a B row read by a long row is not in column order

// One block of (at most NT) A entries of a long row, published for a
// flattened walk: entry e covers the block's products [pre[e], pre[e + 1]),
// product p of it reads B entry qs[e] + (p - pre[e]) and is scaled by a[e].
template <int NT, bool VALS>
struct FlatStage {
    int64_t pre[NT + 1];
    int64_t qs[NT];
    double a[VALS ? NT : 1];
};

// The A entry a thread holds: the B row it names and the A value.
struct LongEnt {
    int64_t b0;    // first B entry of the named row
    int64_t len;   // its length (0 for threads without an entry)
    double a;
};

// Thread t's entry of block `blk` (entries blk * NT + t of the A row at rs).
template <int NT, typename T, typename IdxT, bool VALS>
__device__ __forceinline__ LongEnt long_entry(IdxT rs, int64_t nA, int blk, const int32_t* __restrict__ a_col,
                                              const T* __restrict__ a_val, const IdxT* __restrict__ b_rp) {
    LongEnt en{0, 0, 0.0};
    const int64_t e = (int64_t)blk * NT + threadIdx.x;
    if (e < nA) {
        const int k = a_col[rs + e];
        const IdxT x0 = b_rp[k];
        const IdxT x1 = b_rp[k + 1];
        en.b0 = (int64_t)x0;
        en.len = (int64_t)x1 - (int64_t)x0;
        if (VALS) en.a = (double)a_val[rs + e];
    }
    return en;
}

// Publishes every thread's range [q, q + len) (scaled by a) for a flattened
// walk and returns the block's product count.  Collective: every thread of
// the workgroup calls it.  The scan's first barrier also ends the walks of
// the previous publication before the stage is overwritten.
template <int NT, bool VALS>
__device__ __forceinline__ int64_t flat_publish(FlatStage<NT, VALS>& st, int64_t q, int64_t len, double a,
                                                long long* s_red) {
    long long tot;
    const long long ex = block_excl_scan_i64<NT>((long long)len, s_red, &tot);
    st.pre[threadIdx.x] = ex;
    st.qs[threadIdx.x] = q;
    if constexpr (VALS) st.a[threadIdx.x] = a;
    if (threadIdx.x == 0) st.pre[NT] = tot;
    __syncthreads();
    return tot;
}

// Calls fn(col, v) for every product of a published block (total products)
// that this wavefront owns; v = a_e * b_kj in FP64 when VALS (else 0).
// CHECK sets *unsorted when two consecutive entries of one B row are in
// descending column order.
template <int NT, typename T, bool VALS, bool SVALS, bool CHECK, typename Fn>
__device__ __forceinline__ void flat_walk(const FlatStage<NT, SVALS>& st, int64_t total,
                                          const int32_t* __restrict__ b_col, const T* __restrict__ b_val,
                                          int wave, int nwaves, Fn&& fn, bool* unsorted = nullptr) {
    constexpr int U = kFlatU;
    const int lane = lane_id();
    for (int64_t s = (int64_t)wave * (kWave * U); s < total; s += (int64_t)nwaves * (kWave * U)) {
        const int64_t p0 = s + (int64_t)lane * U;
        int64_t q[U];
        double a[U];
        bool on[U], first[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            q[u] = 0;
            a[u] = 0.0;
            on[u] = false;
            first[u] = true;
        }
        if (p0 < total) {
            // entry of p0: pre[lo] <= p0 < pre[hi] (pre[0] = 0, pre[NT] = total)
            int lo = 0, hi = NT;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (st.pre[mid] <= p0) lo = mid; else hi = mid;
            }
            int e = lo;
            int64_t eb = st.pre[e], nb = st.pre[e + 1];
            int64_t base = st.qs[e] - eb;
            double ea = 0.0;
            if constexpr (SVALS) ea = st.a[e];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t pp = p0 + u;
                if (pp < total) {
                    // the run crosses into the next non-empty entry (pre[NT] = total > pp bounds it)
                    while (pp >= nb) {
                        ++e;
                        eb = nb;
                        nb = st.pre[e + 1];
                        base = st.qs[e] - eb;
                        if constexpr (SVALS) ea = st.a[e];
                    }
                    on[u] = true;
                    q[u] = base + pp;
                    a[u] = ea;
                    first[u] = pp == eb;
                }
            }
        }
        int c[U];
        T bv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = -1;
            bv[u] = T(0);
            if (on[u]) {
                c[u] = b_col[q[u]];
                if (VALS) bv[u] = b_val[q[u]];
            }
        }
        if (CHECK) {
            // the product before this lane's first is lane - 1's last (for
            // lane 0 it belongs to another step: read it)
            int prev = __shfl_up(c[U - 1], 1, kWave);
            if (lane == 0 && on[0] && !first[0]) prev = b_col[q[0] - 1];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int pc = u == 0 ? prev : c[u - 1];
                if (on[u] && !first[u] && pc > c[u]) *unsorted = true;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (on[u]) fn(c[u], VALS ? a[u] * (double)bv[u] : 0.0);
    }
}

// First position in [lo, hi) of the column-ordered B row at col whose column
// is at least x (hi if none).
__device__ __forceinline__ int64_t lower_col(const int32_t* __restrict__ col, int64_t lo, int64_t hi, int x) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (col[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Partial products of the A row [rs, rs + nA): sum of its entries' B-row lengths.
template <int NT, typename IdxT>
__device__ __forceinline__ long long long_row_count(IdxT rs, int64_t nA, const int32_t* __restrict__ a_col,
                                                    const IdxT* __restrict__ b_rp, long long* s_red) {
    long long s = 0;
    for (int64_t e = threadIdx.x; e < nA; e += NT) {
        const int k = a_col[rs + e];
        s += (long long)b_rp[k + 1] - (long long)b_rp[k];
    }
    return block_sum_i64<NT>(s, s_red);
}

// ---------------------------------------------------------------------------
// Symbolic pass for the long-row list: nnz(C_i) and the column window of each
// long row.  The window is [0, n) when n fits one segment, else the row's
// [min column, max column] (one extra walk of the products).
template <typename IdxT>
__global__ void __launch_bounds__(kLongThreads) k_long_sym(SymArgs<IdxT> p0, const SymArgs<IdxT>* __restrict__ P,
                                                          BatchMap bm) {
    constexpr int NT = kLongThreads, NW = kLongWaves;
    __shared__ uint32_t s_bits[kLongSegWords];
    __shared__ FlatStage<NT, false> s_st;
    __shared__ long long s_red[NW];
    __shared__ int s_redi[NW];
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
        const int nblk = (int)((nA + NT - 1) / NT);
        const float* no_val = nullptr;
        // a row of one block is published once for all its walks
        int64_t tot1 = 0;
        long long prods;
        if (nblk == 1) {
            const LongEnt en = long_entry<NT, float, IdxT, false>(rs, nA, 0, p.a_col, no_val, p.b_rp);
            tot1 = flat_publish<NT, false>(s_st, en.b0, en.len, 0.0, s_red);
            prods = (long long)tot1;
        } else {
            prods = long_row_count<NT, IdxT>(rs, nA, p.a_col, p.b_rp, s_red);
        }
        auto walk_all = [&](auto&& fn, bool* unsorted) {
            if (nblk == 1) {
                flat_walk<NT, float, false, false, true>(s_st, tot1, p.b_col, no_val, w, NW, fn, unsorted);
                return;
            }
            for (int b = 0; b < nblk; ++b) {
                const LongEnt en = long_entry<NT, float, IdxT, false>(rs, nA, b, p.a_col, no_val, p.b_rp);
                const int64_t tot = flat_publish<NT, false>(s_st, en.b0, en.len, 0.0, s_red);
                flat_walk<NT, float, false, false, true>(s_st, tot, p.b_col, no_val, w, NW, fn, unsorted);
            }
        };

        int lo = 0;
        int64_t span = p.n;
        bool unsorted = false;
        if (p.n > seg_cols) {
            int cmin = INT32_MAX, cmax = -1;
            walk_all(
                [&](int col, double) {
                    cmin = min(cmin, col);
                    cmax = max(cmax, col);
                },
                &unsorted);
            cmin = block_min_i32<NT>(cmin, s_redi);
            cmax = block_max_i32<NT>(cmax, s_redi);
            lo = cmin;
            span = (cmax >= cmin) ? (int64_t)cmax - cmin + 1 : 0;
        }
        long long nnz = 0;
        for (int64_t s0 = 0; s0 < span; s0 += seg_cols) {
            const int seg_lo = lo + (int)s0;
            const int seg_w = (int)((min((int64_t)seg_cols, span - s0) + 31) >> 5);
            const int seg_hi = seg_lo + seg_w * 32;
            for (int x = threadIdx.x; x < seg_w; x += NT) s_bits[x] = 0u;
            __syncthreads();
            walk_all(
                [&](int col, double) {
                    if (col >= seg_lo && col < seg_hi) {
                        const int d = col - seg_lo;
                        atomicOr(&s_bits[d >> 5], 1u << (d & 31));
                    }
                },
                &unsorted);
            __syncthreads();
            long long pc = 0;
            for (int x = threadIdx.x; x < seg_w; x += NT) pc += __popc(s_bits[x]);
            nnz += block_sum_i64<NT>(pc, s_red);
        }
        if (p.n <= seg_cols && span > 0) {
            // one segment from column 0: narrow the window to the set bits
            // (the numeric pass then zeroes, scans and emits fewer words)
            const int seg_w = (int)((span + 31) >> 5);
            int cmin = INT32_MAX, cmax = -1;
            for (int x = threadIdx.x; x < seg_w; x += NT) {
                const uint32_t bw = s_bits[x];
                if (bw) {
                    cmin = min(cmin, x * 32 + __ffs(bw) - 1);
                    cmax = max(cmax, x * 32 + 31 - __clz(bw));
                }
            }
            cmin = block_min_i32<NT>(cmin, s_redi);
            cmax = block_max_i32<NT>(cmax, s_redi);
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
//    in LDS in one flattened walk of the products;
//  - a larger segment is cut into nch chunks of V consecutive ranks (a column
//    range each).  If the long B rows are in column order (checked by the
//    symbolic pass), each chunk is summed in LDS and written to C: the thread
//    holding an A entry binary-searches where the chunk's column range ends
//    in its B row (it starts where the previous chunk's ended), and the
//    ranges of all entries are walked flattened;
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
    __shared__ FlatStage<NT, true> s_st;
    __shared__ long long s_red[NW];
    __shared__ int s_bound[kLongMaxChunks + 1];
    __shared__ int s_next;

    const int w = threadIdx.x / kWave;
    const int nL = (int)*bm.n_long;
    for (;;) {
        if (threadIdx.x == 0) s_next = (int)atomicAdd(&bm.queue[1], 1u);
        __syncthreads();
        const int j = uniform_i32(s_next);
        if (j >= nL) break;
        const int2 ent = bm.long_list[j];
        const NumArgs<T, IdxT, IdxC> p = P ? P[uniform_i32(ent.x)] : p0;
        const int seg_cols = uniform_i32(p.th.group_lds_span);
        const int V = min(max(uniform_i32(p.th.group_lds_values), kLongMinVals), kLongVals);
        const bool sorted_b = (uniform_i32((int)p.ctr->bad_csr) & kUnsortedB) == 0u;
        const int64_t i = uniform_i32(ent.y);
        const IdxT rs = uniform(p.a_rp[i]);
        const int64_t nA = uniform((int64_t)p.a_rp[i + 1]) - (int64_t)rs;
        const int nblk = (int)((nA + NT - 1) / NT);
        const int2 wn = p.win[i];
        const int lo = uniform_i32(wn.x);
        const int64_t span = uniform_i32(wn.y);
        const int64_t cb = uniform((int64_t)p.c_rp[i]);
        const int64_t nc_row = uniform((int64_t)p.c_rp[i + 1]) - cb;

        // a row of one block keeps its entry in registers and its full
        // ranges published until a chunked accumulation replaces them
        LongEnt en1{0, 0, 0.0};
        int64_t tot1 = 0;
        bool full1 = false;
        if (nblk == 1) en1 = long_entry<NT, T, IdxT, true>(rs, nA, 0, p.a_col, p.a_val, p.b_rp);
        auto walk_all = [&](auto vals_tag, auto&& fn) {
            constexpr bool VL = decltype(vals_tag)::value;
            if (nblk == 1) {
                if (!full1) {
                    tot1 = flat_publish<NT, true>(s_st, en1.b0, en1.len, en1.a, s_red);
                    full1 = true;
                }
                flat_walk<NT, T, VL, true, false>(s_st, tot1, p.b_col, p.b_val, w, NW, fn);
                return;
            }
            for (int b = 0; b < nblk; ++b) {
                const LongEnt en = long_entry<NT, T, IdxT, true>(rs, nA, b, p.a_col, p.a_val, p.b_rp);
                const int64_t tot = flat_publish<NT, true>(s_st, en.b0, en.len, en.a, s_red);
                flat_walk<NT, T, VL, true, false>(s_st, tot, p.b_col, p.b_val, w, NW, fn);
            }
        };
        using NoVals = std::integral_constant<bool, false>;
        using Vals = std::integral_constant<bool, true>;

        int64_t off = 0;
        for (int64_t s0 = 0; s0 < span; s0 += seg_cols) {
            const int seg_lo = lo + (int)s0;
            const int seg_w = (int)((min((int64_t)seg_cols, span - s0) + 31) >> 5);
            const int seg_hi = seg_lo + seg_w * 32;
            for (int x = threadIdx.x; x < seg_w; x += NT) s_bits[x] = 0u;
            __syncthreads();
            walk_all(NoVals{}, [&](int col, double) {
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
                walk_all(Vals{}, [&](int col, double v) {
                    if (col >= seg_lo && col < seg_hi) atomicAdd(&s_vals[rank_of(col)], v);
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
                // with one block, each thread's position in its B row carries
                // from one chunk to the next (the chunk's range starts there)
                int64_t cur1 = 0;
                for (int c = 0; c < nch; ++c) {
                    const int clo = s_bound[c], chi = s_bound[c + 1];
                    const int r0 = c * V, rn = min(V, seg_nnz - r0);
                    for (int x = threadIdx.x; x < rn; x += NT) s_vals[x] = 0.0;
                    auto add = [&](int col, double v) { atomicAdd(&s_vals[rank_of(col) - r0], v); };
                    for (int b = 0; b < nblk; ++b) {
                        const LongEnt en = nblk == 1 ? en1 : long_entry<NT, T, IdxT, true>(rs, nA, b, p.a_col,
                                                                                           p.a_val, p.b_rp);
                        const int32_t* brow = p.b_col + en.b0;
                        const int64_t qlo = (nblk == 1 && c > 0) ? cur1 : lower_col(brow, 0, en.len, clo);
                        const int64_t qhi = lower_col(brow, qlo, en.len, chi);
                        cur1 = qhi;
                        // publishing (its barriers) also orders the zeroing above before the adds
                        const int64_t tot = flat_publish<NT, true>(s_st, en.b0 + qlo, qhi - qlo, en.a, s_red);
                        flat_walk<NT, T, true, true, false>(s_st, tot, p.b_col, p.b_val, w, NW, add);
                    }
                    full1 = false;
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
                walk_all(Vals{}, [&](int col, double v) {
                    if (col >= seg_lo && col < seg_hi)
                        __hip_atomic_fetch_add(&acc[rank_of(col)], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
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
