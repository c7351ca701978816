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
// the B rows the entries name.  Each wavefront takes steps of 64 * U
// consecutive products, lane l the products 64 u + l of the step (u < U), so
// that every load instruction reads 64 consecutive B entries; a lane finds
// the entry of a product by a binary search over pre in LDS when the product
// passes the end of its previous one.  Every wavefront
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

constexpr int kLongSegWords = 8192;     // 262144 columns per window segment (the wide shapes)
constexpr int kLongVals = 8192;         // numeric: FP64 accumulator slots in LDS (the large shape)
constexpr int kLongMinVals = 256;       // smallest rank chunk accepted

// Workgroup shapes.  Symbolic: threads and bitmap words per segment.  The
// narrow one serves batches whose products all have at most 65536 columns.
struct LongSymWide {
    static constexpr int NT = 512, SEGW = kLongSegWords;   // two workgroups per CU
};
struct LongSymNarrow {
    static constexpr int NT = 256, SEGW = 2048;            // four per CU
};
// Numeric: threads, bitmap words per segment, LDS accumulator slots, A
// entries staged per block, chunk-boundary positions kept in LDS, and which
// part of the split list it takes.  Large rows: one workgroup per CU (its
// LDS is ~159 KB).  Medium rows -- a window of at most 65536 columns and at
// most 2048 entries of C, the size of most rows of the uniform-random
// products -- take a quarter of the threads and ~43 KB of LDS, three
// workgroups per CU.
struct LongNumLarge {
    static constexpr int NT = 1024, SEGW = kLongSegWords, VMAX = kLongVals, NB = 512, POS = 3840;
    static constexpr bool MID = false;
};
struct LongNumMid {
    static constexpr int NT = 256, SEGW = 2048, VMAX = 2048, NB = 256, POS = 1024;
    static constexpr bool MID = true;
};
constexpr int kMidCols = LongNumMid::SEGW * 32;   // widest window of a medium row
constexpr int kMidPerCu = 3;                      // medium workgroups per CU
constexpr int kFlatU = 4;               // products per lane and step of a flattened walk that reads values
constexpr int kFlatUCols = 8;           // ... of one that reads columns only
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

// Thread t's entry of block `blk` (entries blk * NB + t of the A row at rs;
// threads from NB on hold none).
template <int NB, typename T, typename IdxT, bool VALS>
__device__ __forceinline__ LongEnt long_entry(IdxT rs, int64_t nA, int blk, const int32_t* __restrict__ a_col,
                                              const T* __restrict__ a_val, const IdxT* __restrict__ b_rp) {
    LongEnt en{0, 0, 0.0};
    const int64_t e = (int64_t)blk * NB + threadIdx.x;
    if ((int)threadIdx.x < NB && e < nA) {
        const int k = a_col[rs + e];
        const IdxT x0 = b_rp[k];
        const IdxT x1 = b_rp[k + 1];
        en.b0 = (int64_t)x0;
        en.len = (int64_t)x1 - (int64_t)x0;
        if (VALS) en.a = (double)a_val[rs + e];
    }
    return en;
}

// Publishes the range [q, q + len) (scaled by a) of each of the first NB
// threads (the others pass len = 0) for a flattened walk and returns the
// block's product count.  Collective: every thread of the workgroup (NT)
// calls it.  The scan's barrier also ends the walks of the previous
// publication before the stage is overwritten.  `buf` (NT / 64 partials)
// serves publications only: the barrier that ends each publication
// separates it from the next.
template <int NT, int NB, bool VALS>
__device__ __forceinline__ int64_t flat_publish(FlatStage<NB, VALS>& st, int64_t q, int64_t len, double a,
                                                long long* buf) {
    long long tot;
    const long long ex = block_excl_scan1_i64<NT>((long long)len, buf, &tot);
    if ((int)threadIdx.x < NB) {
        st.pre[threadIdx.x] = ex;
        st.qs[threadIdx.x] = q;
        if constexpr (VALS) st.a[threadIdx.x] = a;
    }
    if (threadIdx.x == 0) st.pre[NB] = tot;
    __syncthreads();
    return tot;
}

// Entry of product p among entries [lo, hi) of a published block: the e with
// pre[e] <= p < pre[e + 1], given pre[lo] <= p < pre[hi].
template <int NT, bool SVALS>
__device__ __forceinline__ int flat_find(const FlatStage<NT, SVALS>& st, int lo, int hi, int64_t p) {
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (st.pre[mid] <= p) lo = mid; else hi = mid;
    }
    return lo;
}

// Calls fn(col, v) for every product of a published block (ne entries,
// total products) that this wavefront owns; v = a_e * b_kj in FP64 when VALS
// (else 0).  The wavefront takes steps of 64 * U consecutive products; in
// step s, lane l takes products s + 64 u + l (u < U), so that each of the
// U loads of a step reads 64 consecutive B entries wherever the step lies
// inside one B row.  A lane's products only move forward: it keeps the
// bounds of its current entry and searches the later entries only when a
// product passes the end of it.  CHECK sets *unsorted when two consecutive
// entries of one B row are in descending column order.
template <int U, int NT, typename T, bool VALS, bool SVALS, bool CHECK, typename Fn>
__device__ __forceinline__ void flat_walk(const FlatStage<NT, SVALS>& st, int ne, int64_t total,
                                          const int32_t* __restrict__ b_col, const T* __restrict__ b_val,
                                          int wave, int nwaves, Fn&& fn, bool* unsorted = nullptr) {
    const int lane = lane_id();
    // this lane's current entry e: products [eb, nb), B entry of product p = base + p
    int e = 0;
    int64_t eb = 0, nb = st.pre[1], base = st.qs[0];
    double ea = 0.0;
    if constexpr (SVALS) ea = st.a[0];
    for (int64_t s = (int64_t)wave * (kWave * U); s < total; s += (int64_t)nwaves * (kWave * U)) {
        int64_t q[U];
        double a[U];
        bool on[U], first[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t p = s + u * kWave + lane;
            on[u] = p < total;
            q[u] = 0;
            a[u] = 0.0;
            first[u] = true;
            if (on[u]) {
                if (p >= nb) {
                    // pre[e + 1] = nb <= p < total = pre[ne]
                    e = flat_find(st, e + 1, ne, p);
                    eb = st.pre[e];
                    nb = st.pre[e + 1];
                    base = st.qs[e] - eb;
                    if constexpr (SVALS) ea = st.a[e];
                }
                q[u] = base + p;
                a[u] = ea;
                first[u] = p == eb;
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
            // the product before (u, l) is (u, l - 1); before (u, 0) it is
            // (u - 1, 63), and before (0, 0) it lies in an earlier step: read it
#pragma unroll
            for (int u = 0; u < U; ++u) {
                int prev = __shfl_up(c[u], 1, kWave);
                if (u > 0) {
                    const int last = __shfl(c[u - 1], kWave - 1, kWave);
                    if (lane == 0) prev = last;
                } else if (lane == 0 && on[0] && !first[0]) {
                    prev = b_col[q[0] - 1];
                }
                if (on[u] && !first[u] && prev > c[u]) *unsorted = true;
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
// [min column, max column] (one extra walk of the products).  The segment
// bitmap is all zero between segments: its words are cleared as they are
// counted.
template <typename IdxT, typename S>
__global__ void __launch_bounds__(S::NT) k_long_sym(SymArgs<IdxT> p0, const SymArgs<IdxT>* __restrict__ P,
                                                   BatchMap bm) {
    constexpr int NT = S::NT, NW = NT / kWave;
    __shared__ uint32_t s_bits[S::SEGW];
    __shared__ FlatStage<NT, false> s_st;
    __shared__ long long s_pub[NW];      // partials of the publications
    __shared__ long long s_red[NW];      // partials of the other reductions
    __shared__ int s_redi[NW];
    __shared__ long long s_cnt[NW];      // per-segment count, first and last set column
    __shared__ int s_cmin[NW], s_cmax[NW];
    __shared__ int s_next[2];

    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int nL = (int)*bm.n_long;
    if (nL == 0) return;   // the usual case on regular inputs: leave before touching the queue
    for (int x = threadIdx.x; x < S::SEGW; x += NT) s_bits[x] = 0u;
    if (threadIdx.x == 0) s_next[0] = (int)atomicAdd(&bm.queue[0], 1u);
    __syncthreads();
    for (int it = 0;; ++it) {
        const int j = uniform_i32(s_next[it & 1]);
        if (j >= nL) break;
        // take the next row now, so that its queue latency overlaps this one
        // (read after this row's barriers; the slot alternates because a
        // thread may still be reading this row's slot)
        if (threadIdx.x == 0) s_next[(it + 1) & 1] = (int)atomicAdd(&bm.queue[0], 1u);
        const int2 ent = bm.long_list[j];
        const SymArgs<IdxT> p = P ? P[uniform_i32(ent.x)] : p0;
        const int seg_cols = min(uniform_i32(p.th.group_lds_span), S::SEGW * 32);
        const int64_t i = uniform_i32(ent.y);
        const IdxT rs = uniform(p.a_rp[i]);
        const int64_t nA = uniform((int64_t)p.a_rp[i + 1]) - (int64_t)rs;
        const int nblk = (int)((nA + NT - 1) / NT);
        const float* no_val = nullptr;
        // a row of one block is published once for all its walks (the
        // publication's barriers also order the previous row's clearing of
        // the bitmap before this row's first walk)
        int64_t tot1 = 0;
        long long prods;
        if (nblk == 1) {
            const LongEnt en = long_entry<NT, float, IdxT, false>(rs, nA, 0, p.a_col, no_val, p.b_rp);
            tot1 = flat_publish<NT, NT, false>(s_st, en.b0, en.len, 0.0, s_pub);
            prods = (long long)tot1;
        } else {
            prods = long_row_count<NT, IdxT>(rs, nA, p.a_col, p.b_rp, s_red);
        }
        auto walk_all = [&](auto&& fn, bool* unsorted) {
            if (nblk == 1) {
                flat_walk<kFlatUCols, NT, float, false, false, true>(s_st, (int)nA, tot1, p.b_col, no_val, w, NW, fn,
                                                                     unsorted);
                return;
            }
            for (int b = 0; b < nblk; ++b) {
                const LongEnt en = long_entry<NT, float, IdxT, false>(rs, nA, b, p.a_col, no_val, p.b_rp);
                const int64_t tot = flat_publish<NT, NT, false>(s_st, en.b0, en.len, 0.0, s_pub);
                const int ne = (int)min((int64_t)NT, nA - (int64_t)b * NT);
                flat_walk<kFlatUCols, NT, float, false, false, true>(s_st, ne, tot, p.b_col, no_val, w, NW, fn,
                                                                     unsorted);
            }
        };

        int lo = 0;
        int64_t span = p.n;
        bool unsorted = false;
        const bool one_seg = p.n <= seg_cols;
        if (!one_seg) {
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
        int first = INT32_MAX, last = -1;
        for (int64_t s0 = 0; s0 < span; s0 += seg_cols) {
            if (s0 > 0) __syncthreads();   // the previous segment's words are clear
            const int seg_lo = lo + (int)s0;
            const int seg_w = (int)((min((int64_t)seg_cols, span - s0) + 31) >> 5);
            const int seg_hi = seg_lo + seg_w * 32;
            walk_all(
                [&](int col, double) {
                    if (col >= seg_lo && col < seg_hi) {
                        const int d = col - seg_lo;
                        atomicOr(&s_bits[d >> 5], 1u << (d & 31));
                    }
                },
                &unsorted);
            __syncthreads();
            // set bits, and the first and last set column (for a window of
            // one segment from column 0, narrowed below), clearing each word
            long long pc = 0;
            int cmin = INT32_MAX, cmax = -1;
            for (int x = threadIdx.x; x < seg_w; x += NT) {
                const uint32_t bw = s_bits[x];
                if (bw) {
                    pc += __popc(bw);
                    cmin = min(cmin, x * 32 + __ffs(bw) - 1);
                    cmax = max(cmax, x * 32 + 31 - __clz(bw));
                    s_bits[x] = 0u;
                }
            }
            pc = wave_sum_i64(pc);
            cmin = wave_min_i32(cmin);
            cmax = wave_max_i32(cmax);
            if (lane == 0) {
                s_cnt[w] = pc;
                s_cmin[w] = cmin;
                s_cmax[w] = cmax;
            }
            __syncthreads();
            long long sn = 0;
#pragma unroll
            for (int x = 0; x < NW; ++x) {
                sn += s_cnt[x];
                first = min(first, s_cmin[x]);
                last = max(last, s_cmax[x]);
            }
            nnz += sn;
        }
        if (one_seg && span > 0) {
            // one segment from column 0: narrow the window to the set bits
            // (the numeric pass then scans and emits fewer words)
            lo = last >= 0 ? first : 0;
            span = last >= 0 ? (int64_t)last - first + 1 : 0;
        }
        // the numeric pass walks the B rows of long rows in column order only
        // when they are stored that way
        if (ballot(unsorted) && lane == 0) atomicOr(&p.ctr->bad_csr, kUnsortedB);
        if (threadIdx.x == 0) {
            p.rnnz[i] = (int32_t)nnz;
            p.win[i] = make_int2(lo, (int)span);
            if (nnz) atomicAdd(&p.tiles[i / kScanTile], (unsigned long long)nnz);
            atomicAdd(&p.ctr->products, (unsigned long long)prods);
            atomicMax(&p.ctr->max_prod, (unsigned)min(prods, (long long)UINT32_MAX));
            atomicMax(&p.ctr->max_nnz, (unsigned)nnz);
            atomicMax(&p.ctr->max_group_nnz, (unsigned)nnz);
            // the numeric pass takes medium and large rows in workgroups of
            // their own shape; rows without an entry of C need no numeric work
            if (nnz > 0) {
                if (nnz <= p.th.mid_nnz && span <= kMidCols) {
                    const unsigned k = atomicAdd(&bm.n_split[0], 1u);
                    bm.split_list[k] = ent;
                } else {
                    const unsigned k = atomicAdd(&bm.n_split[1], 1u);
                    bm.split_list[bm.split_cap - 1u - k] = ent;
                }
            }
        }
        // s_cnt, s_cmin, s_cmax are read again only after the next row's
        // publication and walk (two barriers on)
    }
}

// ---------------------------------------------------------------------------
// Numeric pass for one part of the split list, one workgroup of shape S per
// row (1024 threads for large rows, 256 for medium ones).
// Per segment of the row's window (up to S::SEGW * 32 columns): (1) bitmap of the
// segment's columns, (2) prefix count of set bits per word (block scan), so
// the rank of a column -- its position in the sorted row -- is one LDS read
// and a popcount, (3) accumulation by rank, (4) columns written from the
// bitmap in ascending order.  Accumulation:
//  - a segment with at most V = group_lds_values (<= S::VMAX) entries is summed
//    in LDS in one flattened walk of the products;
//  - a larger segment is cut into nch chunks of V consecutive ranks (a column
//    range each).  If the long B rows are in column order (checked by the
//    symbolic pass), each chunk is summed in LDS and written to C; where
//    every chunk boundary falls in every B row of the row is found first
//    with all binary searches side by side (one per boundary and A entry,
//    positions kept in LDS), then the chunks' ranges are walked flattened;
//  - if a long B row is not in column order, every product of the segment is
//    added with FP64 atomics into device memory: C's own values for FP64, a
//    per-workgroup FP64 buffer for FP32 (rounded once on the copy out).  Only
//    this workgroup touches those slots, so the atomics are workgroup-scoped.
// Barriers are few (a row of one segment summed in one walk passes six): the
// bitmap and the LDS accumulator are all zero between uses, each thread
// clearing the words and slots it copies out, and the barriers of the next
// publication order that clearing before the next walk.
template <typename T, typename IdxT, typename IdxC, typename S>
__global__ void __launch_bounds__(S::NT) k_long_num(NumArgs<T, IdxT, IdxC> p0,
                                                   const NumArgs<T, IdxT, IdxC>* __restrict__ P, BatchMap bm) {
    constexpr int NT = S::NT, NW = NT / kWave, NB = S::NB;
    constexpr int kMaxChunks = S::SEGW * 32 / kLongMinVals;
    __shared__ uint32_t s_bits[S::SEGW];
    __shared__ uint32_t s_pfx[S::SEGW];              // set bits of the segment before each word
    __shared__ double s_vals[S::VMAX];
    __shared__ FlatStage<NB, true> s_st;
    __shared__ int32_t s_pos[S::POS];                // [chunk boundary][A entry]: position in the entry's B row
    __shared__ long long s_pub[NW];                  // partials of the publications
    __shared__ long long s_scan[NW];                 // partials of the prefix counts
    __shared__ int s_bound[kMaxChunks + 1];
    __shared__ int s_next[2];

    const int w = threadIdx.x / kWave;
    const int nL = (int)bm.n_split[S::MID ? 0 : 1];
    if (nL == 0) return;
    unsigned int* const queue = &bm.queue[S::MID ? 2 : 1];
    // medium rows from the start of the split list, large ones from its end
    auto entry = [&](int jj) { return bm.split_list[S::MID ? (unsigned)jj : bm.split_cap - 1u - (unsigned)jj]; };
    for (int x = threadIdx.x; x < S::SEGW; x += NT) s_bits[x] = 0u;
    for (int x = threadIdx.x; x < S::VMAX; x += NT) s_vals[x] = 0.0;
    if (threadIdx.x == 0) s_next[0] = (int)atomicAdd(queue, 1u);
    __syncthreads();
    for (int it = 0;; ++it) {
        const int j = uniform_i32(s_next[it & 1]);
        if (j >= nL) break;
        // the next row's queue entry, taken now (see k_long_sym)
        if (threadIdx.x == 0) s_next[(it + 1) & 1] = (int)atomicAdd(queue, 1u);
        const int2 ent = entry(j);
        const NumArgs<T, IdxT, IdxC> p = P ? P[uniform_i32(ent.x)] : p0;
        const int seg_cols = min(uniform_i32(p.th.group_lds_span), S::SEGW * 32);
        const int V = min(max(uniform_i32(p.th.group_lds_values), kLongMinVals), S::VMAX);
        const bool sorted_b = (uniform_i32((int)p.ctr->bad_csr) & kUnsortedB) == 0u;
        const int64_t i = uniform_i32(ent.y);
        const IdxT rs = uniform(p.a_rp[i]);
        const int64_t nA = uniform((int64_t)p.a_rp[i + 1]) - (int64_t)rs;
        const int nblk = (int)((nA + NB - 1) / NB);
        const int2 wn = p.win[i];
        const int lo = uniform_i32(wn.x);
        const int64_t span = uniform_i32(wn.y);
        const int64_t cb = uniform((int64_t)p.c_rp[i]);
        const int64_t nc_row = uniform((int64_t)p.c_rp[i + 1]) - cb;

        // a row of one block keeps its full ranges published until a chunked
        // accumulation replaces them (the entries are read again only then:
        // holding them in registers through the row would spill)
        int64_t tot1 = 0;
        bool full1 = false;
        auto walk_all = [&](auto vals_tag, auto&& fn) {
            constexpr bool VL = decltype(vals_tag)::value;
            if (nblk == 1) {
                if (!full1) {
                    const LongEnt en = long_entry<NB, T, IdxT, true>(rs, nA, 0, p.a_col, p.a_val, p.b_rp);
                    tot1 = flat_publish<NT, NB, true>(s_st, en.b0, en.len, en.a, s_pub);
                    full1 = true;
                }
                flat_walk<VL ? kFlatU : kFlatUCols, NB, T, VL, true, false>(s_st, (int)nA, tot1, p.b_col, p.b_val, w,
                                                                            NW, fn);
                return;
            }
            for (int b = 0; b < nblk; ++b) {
                const LongEnt en = long_entry<NB, T, IdxT, true>(rs, nA, b, p.a_col, p.a_val, p.b_rp);
                const int64_t tot = flat_publish<NT, NB, true>(s_st, en.b0, en.len, en.a, s_pub);
                const int ne = (int)min((int64_t)NB, nA - (int64_t)b * NB);
                flat_walk<VL ? kFlatU : kFlatUCols, NB, T, VL, true, false>(s_st, ne, tot, p.b_col, p.b_val, w, NW,
                                                                            fn);
            }
        };
        using NoVals = std::integral_constant<bool, false>;
        using Vals = std::integral_constant<bool, true>;

        int64_t off = 0;
        for (int64_t s0 = 0; s0 < span; s0 += seg_cols) {
            // a row's first walk follows a publication; a later segment's may not
            if (s0 > 0) __syncthreads();
            const int seg_lo = lo + (int)s0;
            const int seg_w = (int)((min((int64_t)seg_cols, span - s0) + 31) >> 5);
            const int seg_hi = seg_lo + seg_w * 32;
            walk_all(NoVals{}, [&](int col, double) {
                if (col >= seg_lo && col < seg_hi) {
                    const int d = col - seg_lo;
                    atomicOr(&s_bits[d >> 5], 1u << (d & 31));
                }
            });
            __syncthreads();
            // thread t owns words [w0, w1), w0 = t * per
            const int per = (seg_w + NT - 1) / NT;
            const int w0 = min((int)threadIdx.x * per, seg_w), w1 = min(w0 + per, seg_w);
            long long local = 0;
            for (int x = w0; x < w1; ++x) local += __popc(s_bits[x]);
            long long seg_nnz_ll;
            const int rank0 = (int)block_excl_scan1_i64<NT>(local, s_scan, &seg_nnz_ll);   // this thread's first rank
            {
                int run = rank0;
                for (int x = w0; x < w1; ++x) {
                    s_pfx[x] = (uint32_t)run;
                    run += __popc(s_bits[x]);
                }
            }
            if (off + seg_nnz_ll > nc_row) {  // pattern differs from the symbolic pass
                if (threadIdx.x == 0) atomicOr(&p.ctr->bad_csr, 4u);
                __syncthreads();
                for (int x = threadIdx.x; x < seg_w; x += NT) s_bits[x] = 0u;
                break;
            }
            const int seg_nnz = (int)seg_nnz_ll;
            __syncthreads();   // prefix counts complete
            auto rank_of = [&](int col) {
                const int d = col - seg_lo;
                const int x = d >> 5;
                return (int)s_pfx[x] + __popc(s_bits[x] & ((1u << (d & 31)) - 1u));
            };
            if (threadIdx.x == 0)
                atomicAdd(seg_nnz <= V ? &p.ctr->seg_lds : (sorted_b ? &p.ctr->seg_chunked : &p.ctr->seg_device), 1u);
            if (seg_nnz <= V) {
                // the whole segment in LDS (the accumulator is zero)
                walk_all(Vals{}, [&](int col, double v) {
                    if (col >= seg_lo && col < seg_hi) atomicAdd(&s_vals[rank_of(col)], v);
                });
                __syncthreads();
                for (int x = threadIdx.x; x < seg_nnz; x += NT) {
                    p.c_val[cb + off + x] = (T)s_vals[x];
                    s_vals[x] = 0.0;
                }
            } else if (sorted_b) {
                // rank chunks, each summed in LDS and written to C as it completes
                const int nch = (seg_nnz + V - 1) / V;
                // column boundaries of the chunks: chunk c holds ranks [cV, cV + V),
                // columns [s_bound[c], s_bound[c + 1])
                if (threadIdx.x == 0) {
                    s_bound[0] = seg_lo;
                    s_bound[nch] = seg_hi;
                }
                {
                    int r = w0 < w1 ? (int)s_pfx[w0] : 0;   // this thread's first rank
                    for (int x = w0; x < w1; ++x) {
                        const int r0 = r;
                        const uint32_t bw = s_bits[x];
                        const int c = __popc(bw);
                        // every multiple of V in [r0, r0 + c) but 0
                        for (int k = max(1, (r0 + V - 1) / V); k * V < r0 + c; ++k) {
                            uint32_t m = bw;
                            for (int t = k * V - r0; t > 0; --t) m &= m - 1;  // drop the lower set bits
                            s_bound[k] = seg_lo + x * 32 + (__ffs(m) - 1);
                        }
                        r += c;
                    }
                }
                __syncthreads();
                // positions of every boundary in every B row, all searches side
                // by side (one block of entries, and room for them in LDS)
                const int ne1 = (int)nA;
                const bool pos_lds = nblk == 1 && (int64_t)(nch + 1) * ne1 <= S::POS;
                if (pos_lds) {
                    for (int x = threadIdx.x; x < (nch + 1) * ne1; x += NT) {
                        const int c = x / ne1, e = x - c * ne1;
                        const int64_t eb0 = s_st.qs[e];   // the full publication (the bitmap walk's)
                        const int64_t elen = s_st.pre[e + 1] - s_st.pre[e];
                        s_pos[x] = (int32_t)lower_col(p.b_col + eb0, 0, elen, s_bound[c]);
                    }
                    __syncthreads();
                }
                for (int c = 0; c < nch; ++c) {
                    const int r0 = c * V, rn = min(V, seg_nnz - r0);
                    auto add = [&](int col, double v) { atomicAdd(&s_vals[rank_of(col) - r0], v); };
                    for (int b = 0; b < nblk; ++b) {
                        int64_t q = 0, len = 0;
                        double a = 0.0;
                        if (pos_lds) {
                            // from the stage this thread published for the previous
                            // chunk (B entry b0 + its first position; the full
                            // ranges, b0 itself, before the first chunk)
                            if ((int)threadIdx.x < ne1) {
                                const int x = threadIdx.x;
                                const int32_t plo = s_pos[c * ne1 + x], phi = s_pos[(c + 1) * ne1 + x];
                                const int32_t prev = c == 0 ? 0 : s_pos[(c - 1) * ne1 + x];
                                q = s_st.qs[x] - prev + plo;
                                len = phi - plo;
                                a = s_st.a[x];
                            }
                        } else {
                            const LongEnt en = long_entry<NB, T, IdxT, true>(rs, nA, b, p.a_col, p.a_val, p.b_rp);
                            const int32_t* brow = p.b_col + en.b0;
                            const int64_t qlo = lower_col(brow, 0, en.len, s_bound[c]);
                            const int64_t qhi = lower_col(brow, qlo, en.len, s_bound[c + 1]);
                            q = en.b0 + qlo;
                            len = qhi - qlo;
                            a = en.a;
                        }
                        // the publication's barriers also order the previous chunk's
                        // copy-out (and clearing) before this chunk's adds; each
                        // thread reads only its own stage slot above, before it
                        // rewrites that slot here
                        const int64_t tot = flat_publish<NT, NB, true>(s_st, q, len, a, s_pub);
                        const int ne = (int)min((int64_t)NB, nA - (int64_t)b * NB);
                        flat_walk<kFlatU, NB, T, true, true, false>(s_st, ne, tot, p.b_col, p.b_val, w, NW, add);
                    }
                    full1 = false;
                    __syncthreads();
                    for (int x = threadIdx.x; x < rn; x += NT) {
                        p.c_val[cb + off + r0 + x] = (T)s_vals[x];
                        s_vals[x] = 0.0;
                    }
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
                // the adds of every wavefront are complete (and their rank reads
                // done) before the buffer is read back and the bitmap cleared
                // (all of the workgroup's accesses go through one CU, so a
                // workgroup-scope fence is enough: an agent-scope one would write
                // back and invalidate the whole L2 of the XCD, per row)
                __threadfence_block();
                __syncthreads();
                if constexpr (sizeof(T) != sizeof(double))
                    for (int x = threadIdx.x; x < seg_nnz; x += NT) p.c_val[cb + off + x] = (T)acc[x];
            }
            // columns in ascending order: wavefront w takes a contiguous block of
            // words, its lanes words 64 apart inside it, so that a store
            // instruction writes neighbouring entries and each stretch of C is
            // written by one wavefront (no line is left half-written by
            // several); the words are cleared for the next segment or row
            const int wper = (seg_w + NW - 1) / NW;
            const int wx1 = min(seg_w, (w + 1) * wper);
            for (int x = w * wper + lane_id(); x < wx1; x += kWave) {
                uint32_t bw = s_bits[x];
                int64_t o = cb + off + s_pfx[x];
                s_bits[x] = 0u;
                while (bw) {
                    const int b = __ffs(bw) - 1;
                    bw &= bw - 1;
                    p.c_col[o++] = seg_lo + x * 32 + b;
                }
            }
            off += seg_nnz;
        }
        // a row without segments (no partial product) passed no barrier since
        // the next row's queue slot was written
        if (span <= 0) __syncthreads();
    }
}

// Rewinds the numeric pass's queue counters (a kernel, so that the sequence
// can be captured in a graph).
__global__ void k_long_rewind(unsigned int* queue) {
    if (threadIdx.x < 2) queue[1 + threadIdx.x] = 0u;
}

}  // namespace reap
