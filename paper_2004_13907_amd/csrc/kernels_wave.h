// Wavefront-per-row kernels: symbolic (row product count, binning, per-row
// column count) and numeric (products, accumulation, ascending-column write)
// for rows with at most 64 entries in A whose products fit the grouped lane
// mapping below in a bounded number of 64-lane steps.
//
// Latency structure.  A wavefront owns a chunk of kRowsPerWave consecutive
// rows.  The A entries of the whole chunk and the extents of the B rows they
// name are first staged in LDS (two dependent rounds of loads per chunk, not
// per row).  For each row every product's B index is then computed from LDS,
// and all of the row's B gathers are issued back to back before any of them
// is consumed.
//
// Lane mapping of a row's products: G lanes (a power of two no smaller than
// the row's longest B row) per A entry, 64/G entries per step; the owner of a
// lane is a shift away.  Rows whose B rows are longer than 64 entries, or that
// would need more steps than the kernels hold, are long rows (kernels_long.h).
#pragma once
#include "device_utils.h"
#include "kernels_numeric.h"
#include "kernels_symbolic.h"
#include "spgemm_common.h"

namespace reap {

// A entries of one chunk of rows, with the extent of the B row each names.
template <typename IdxT>
struct WaveStage {
    int64_t rs0;                       // A.row_ptr of the chunk's first row
    int32_t rowoff[kRowsPerWave + 1];  // entries of row r: [rowoff[r], rowoff[r+1]) after rs0
    IdxT b0[kStageCap];                // first B entry of the named row
    int32_t len[kStageCap];            // its length (clamped to 2^24)
};

// Stages rows [row0, row0 + nrows).  Returns false (nothing staged) when the
// chunk has more than kStageCap entries; the caller then loads rows directly.
template <typename IdxT>
__device__ __forceinline__ bool stage_chunk(WaveStage<IdxT>& st, int64_t row0, int nrows,
                                            const IdxT* __restrict__ a_rp, const int32_t* __restrict__ a_col,
                                            const IdxT* __restrict__ b_rp) {
    const int lane = lane_id();
    int64_t rpv = 0;
    if (lane <= nrows) rpv = (int64_t)a_rp[row0 + lane];
    const int64_t rs0 = uniform_i64(shfl(rpv, 0));
    const int64_t E = uniform_i64(shfl(rpv, nrows)) - rs0;
    if (E > kStageCap) return false;
    if (lane <= nrows) st.rowoff[lane] = (int32_t)(rpv - rs0);
    if (lane == 0) st.rs0 = rs0;
    constexpr int U = kStageCap / kWave;
    int k[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int x = u * kWave + lane;
        k[u] = 0;
        if (x < E) k[u] = a_col[rs0 + x];
    }
    IdxT x0[U], x1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int x = u * kWave + lane;
        x0[u] = 0;
        x1[u] = 0;
        if (x < E) {
            x0[u] = b_rp[k[u]];
            x1[u] = b_rp[k[u] + 1];
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int x = u * kWave + lane;
        if (x < E) {
            st.b0[x] = x0[u];
            st.len[x] = (int32_t)min((int64_t)x1[u] - (int64_t)x0[u], (int64_t)(1 << 24));
        }
    }
    wave_sync();
    return true;
}

// Per-row entry view: lane j < nA gets the j-th entry's B extent, from the
// stage when staged, else straight from memory.  With VALS the A value is
// loaded too (issued here, first consumed after the row's gathers).
template <typename T, typename IdxT, bool VALS>
__device__ __forceinline__ void row_entries(const WaveStage<IdxT>& st, bool staged, int r, int64_t i,
                                            const IdxT* __restrict__ a_rp, const int32_t* __restrict__ a_col,
                                            const T* __restrict__ a_val, const IdxT* __restrict__ b_rp,
                                            int& nA, IdxT& b0, int& len, T& a) {
    const int lane = lane_id();
    b0 = 0;
    len = 0;
    a = (T)0;
    if (staged) {
        const int off = uniform_i32(st.rowoff[r]);
        nA = uniform_i32(st.rowoff[r + 1]) - off;
        const int64_t abase = VALS ? uniform_i64(st.rs0) + off : 0;
        if (lane < nA && nA <= kWave) {
            b0 = st.b0[off + lane];
            len = st.len[off + lane];
            if (VALS) a = a_val[abase + lane];
        }
    } else {
        const IdxT rs = uniform(a_rp[i]);
        const int64_t n64 = (int64_t)uniform(a_rp[i + 1]) - (int64_t)rs;
        nA = (int)min(n64, (int64_t)(kWave + 1));
        if (lane < nA && nA <= kWave) {
            const int k = a_col[rs + lane];
            const IdxT x0 = b_rp[k];
            const IdxT x1 = b_rp[k + 1];
            b0 = x0;
            len = (int)min((int64_t)x1 - (int64_t)x0, (int64_t)(1 << 24));
            if (VALS) a = a_val[rs + lane];
        }
    }
}

// One A entry as the product loops see it.
template <typename IdxT>
struct Ent {
    IdxT b0;      // first B index of the entry
    int32_t len;  // B row length
};

// Per-wavefront LDS for one row's product mapping.
template <typename IdxT>
struct RowTable {
    Ent<IdxT> ent[kWave];
    double a[kWave];
};

struct RowPlan {
    int P;       // partial products of the row
    int nIt;     // 64-lane steps
    int logG;    // log2 of lanes per entry
    int nA;
};

// 64-lane steps of a row under the grouped mapping, or a number above every
// step limit when a B row has more than 64 entries.  Lanes >= nA must carry
// len = 0.
__device__ __forceinline__ int grouped_steps(int nA, int len) {
    const int maxlen = dpp_reduce_max(len);
    const int logG = maxlen <= 1 ? 0 : 32 - __clz(maxlen - 1);
    if (logG > 6) return kWaveMaxIt + 1;
    const int shiftE = 6 - logG;
    return (nA + (1 << shiftE) - 1) >> shiftE;
}

// Plans the grouped mapping and writes the row's entry table.  Lanes >= nA
// must carry len = 0, and the classification guarantees at most MAXIT steps
// (a longer plan is cut to MAXIT steps; the numeric pass then finds fewer
// columns than the symbolic pass did and leaves the extra slots zero).
// `slot` receives this lane's index into tb.a, to be written once the A value
// has arrived.
template <typename IdxT, int MAXIT>
__device__ __forceinline__ RowPlan plan_row(int nA, IdxT b0, int len, RowTable<IdxT>& tb, int& slot) {
    const int lane = lane_id();
    RowPlan pl;
    pl.nA = nA;
    pl.P = dpp_reduce_sum(len);
    const int maxlen = dpp_reduce_max(len);
    pl.logG = min(maxlen <= 1 ? 0 : 32 - __clz(maxlen - 1), 6);  // lanes per entry = 2^logG
    const int shiftE = 6 - pl.logG;                               // entries per step = 2^shiftE
    pl.nIt = min((nA + (1 << shiftE) - 1) >> shiftE, MAXIT);
    slot = lane;
    if (lane < nA) tb.ent[lane] = Ent<IdxT>{b0, len};
    wave_sync();
    return pl;
}

// Gathers a row's products for every step t < pl.nIt: ok[t] says whether this
// lane holds a product, own[t] is its entry slot in tb, col[t] / bv[t] its B
// column and value (VALS).  Lanes without a product load the row's first
// product (`safe`, a valid index) so the loads need no branches; all loads are
// issued before any is used.
template <bool VALS, typename T, typename IdxT, int MAXIT>
__device__ __forceinline__ void row_gather(const RowTable<IdxT>& tb, const RowPlan& pl, IdxT safe,
                                           const int32_t* __restrict__ b_col, const T* __restrict__ b_val,
                                           bool (&ok)[MAXIT], int (&own)[MAXIT], int (&col)[MAXIT],
                                           T (&bv)[MAXIT]) {
    const int lane = lane_id();
    const int nIt = uniform_i32(pl.nIt);
    const int nA = uniform_i32(pl.nA);
    const int logG = uniform_i32(pl.logG);
    IdxT bidx[MAXIT];
    // group g of lanes takes entries g*nIt .. g*nIt + nIt - 1, so the entries
    // side by side in one step are far apart in the row (their B rows share
    // fewer columns, which keeps LDS atomics from colliding)
    const int e0 = (lane >> logG) * nIt;
    const int off = lane & ((1 << logG) - 1);
#pragma unroll
    for (int t = 0; t < MAXIT; ++t) {
        ok[t] = false;
        own[t] = 0;
        bidx[t] = safe;
        if (t < nIt) {
            const int e = e0 + t;
            const int ec = min(e, kWave - 1);
            const Ent<IdxT> en = tb.ent[ec];
            ok[t] = (e < nA) && (off < en.len);
            own[t] = ec;
            bidx[t] = ok[t] ? en.b0 + (IdxT)off : safe;
        }
    }
#pragma unroll
    for (int t = 0; t < MAXIT; ++t) {
        if (t < nIt) {
            col[t] = b_col[bidx[t]];
            if (VALS) bv[t] = b_val[bidx[t]];
        }
    }
}

// LDS position of bitmap word w: one spare word after every 32, so words a
// multiple of 32 apart (columns a multiple of 1024 apart, common in banded
// matrices) fall in different LDS banks.
__device__ __forceinline__ int pad_word(int w) { return w + (w >> 5); }
constexpr int padded_words(int n) { return n + n / 32 + 1; }
// Row stride of a per-wavefront bitmap: padded_words rounded up to 4 words,
// so it can be cleared with 16-byte stores.
constexpr int bitmap_stride(int n) { return (padded_words(n) + 3) & ~3; }

// Clears words [0, padded_words(nw)) of a 16-byte aligned bitmap row (and up
// to 3 words after them, inside the row stride), four words per lane.
__device__ __forceinline__ void clear_bitmap(uint32_t* bits, int nw) {
    for (int x = 4 * lane_id(); x < padded_words(nw); x += 4 * kWave)
        *reinterpret_cast<uint4*>(bits + x) = make_uint4(0u, 0u, 0u, 0u);
}

// First B index of the row (the first entry with a non-empty B row).
template <typename IdxT>
__device__ __forceinline__ IdxT row_safe_index(IdxT b0, int len) {
    const uint64_t ne = ballot(len > 0);
    const int fl = ne ? __ffsll((unsigned long long)ne) - 1 : 0;
    return shfl(b0, fl);
}

// Distinct columns of one row (the symbolic pass proper): the row's products
// are gathered, the column window [min, max] is found, and the columns are
// set in an LDS bitmap over the window (or, when the window is wider than
// th.wave_max_span, inserted in an LDS hash set).  Lanes without a product set
// a bit in the dummy word bits[kWaveBitsWords], so no lane needs a branch.
template <typename IdxT, int MAXIT>
__device__ __forceinline__ void sym_row(const RowTable<IdxT>& tb, const RowPlan& pl, IdxT safe,
                                        const int32_t* __restrict__ b_col, uint32_t* bits, const Thresholds& th,
                                        uint8_t& cls, int& nnz, int2& win) {
    const int lane = lane_id();
    const int nIt = uniform_i32(pl.nIt);
    bool ok[MAXIT];
    int own[MAXIT];
    int col[MAXIT];
    float bv_unused[MAXIT];
    row_gather<false, float, IdxT, MAXIT>(tb, pl, safe, b_col, nullptr, ok, own, col, bv_unused);
    int cmin = INT32_MAX, cmax = -1;
#pragma unroll
    for (int t = 0; t < MAXIT; ++t) {
        if (t < nIt) {
            cmin = ok[t] ? min(cmin, col[t]) : cmin;
            cmax = ok[t] ? max(cmax, col[t]) : cmax;
        }
    }
    cmin = dpp_reduce_min(cmin);
    cmax = dpp_reduce_max(cmax);
    const int64_t span = (int64_t)cmax - cmin + 1;
    if (span <= th.wave_max_span) {
        const int nw = (int)((span + 31) >> 5);
        clear_bitmap(bits, nw);
        wave_sync();
#pragma unroll
        for (int t = 0; t < MAXIT; ++t) {
            if (t < nIt) {
                const int d = ok[t] ? col[t] - cmin : kWaveBitsWords * 32;
                atomicOr(&bits[pad_word(d >> 5)], 1u << (d & 31));
            }
        }
        wave_sync();
        int pc = 0;
        for (int x = lane; x < nw; x += kWave) pc += __popc(bits[pad_word(x)]);
        nnz = dpp_reduce_sum(pc);
        win = make_int2(cmin, nw);
        // the compact bitmap class, or the long-row kernels
        cls = (nnz <= th.wave_small_nnz && nw <= kWaveSmallWords && uniform_i32(pl.P) <= kWaveSmallProducts)
                  ? kClsWaveBmpS
                  : kClsGroup;
    } else if (uniform_i32(pl.P) <= th.wave_hash_products && nIt <= kWaveHashIt) {
        for (int x = lane; x < kWaveHashSlots; x += kWave) bits[x] = 0xFFFFFFFFu;
        wave_sync();
        int mine = 0;
#pragma unroll
        for (int t = 0; t < MAXIT; ++t) {
            if (t < nIt && ok[t]) {
                const uint32_t key = (uint32_t)col[t];
                uint32_t h = hash_col(col[t]) >> (32 - 9);
                while (true) {
                    const uint32_t old = atomicCAS(&bits[h], 0xFFFFFFFFu, key);
                    if (old == 0xFFFFFFFFu) {
                        ++mine;
                        break;
                    }
                    if (old == key) break;
                    h = (h + 1) & (kWaveHashSlots - 1);
                }
            }
        }
        nnz = dpp_reduce_sum(mine);
        cls = kClsWaveHash;
    }
    wave_sync();
}

// ---------------------------------------------------------------------------
// Symbolic, one wavefront per row.  Classifies every row and counts the
// distinct columns of rows that stay here: an LDS bitmap over the row's column
// window [min, max] when it spans at most th.wave_max_span columns, else an
// LDS hash set when the row has at most th.wave_hash_products products.  Rows
// with more than 64 entries or th.wave_max_products products go to the
// long-row list.
// TAB: arguments from the batch table (else the by-value argument of a single product).
template <typename IdxT, bool TAB>
__global__ void __launch_bounds__(kWaveKernelWaves * 64) __attribute__((amdgpu_waves_per_eu(5)))
k_sym_wave(SymArgs<IdxT> p0, const SymArgs<IdxT>* __restrict__ P, BatchMap bm) {
    constexpr int W = kWaveKernelWaves;
    constexpr int MAXIT = kWaveMaxIt;
    __shared__ __align__(16) uint32_t s_bits[W][bitmap_stride(kWaveBitsWords)];  // padded, + a dummy word
    __shared__ RowTable<IdxT> s_tb[W];
    __shared__ WaveStage<IdxT> s_stage[W];
    __shared__ WGPart s_part[W];

    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int gb = xcd_contiguous_block(blockIdx.x, gridDim.x);
    const int q = TAB && bm.nprod > 1 ? find_product(bm.blk_start, bm.nprod, gb) : 0;
    const int blk = gb - (TAB && bm.nprod > 1 ? bm.blk_start[q] : 0);
    const SymArgs<IdxT> p = TAB ? P[q] : p0;
    const int64_t row0 = ((int64_t)blk * W + w) * kRowsPerWave;
    uint32_t* bits = s_bits[w];
    RowTable<IdxT>& tb = s_tb[w];
    WaveStage<IdxT>& st = s_stage[w];

    unsigned long long prod_acc = 0;
    unsigned int cnt[kNumClasses] = {0, 0, 0, 0, 0};
    unsigned int maxp = 0, maxn = 0;
    uint32_t group_flags = 0;

    const int nrows = (int)max((int64_t)0, min((int64_t)kRowsPerWave, p.m - row0));
    const bool staged = nrows > 0 && stage_chunk<IdxT>(st, row0, nrows, p.a_rp, p.a_col, p.b_rp);

    for (int r = 0; r < nrows; ++r) {
        const int64_t i = row0 + r;
        int nA;
        IdxT b0;
        int len;
        float a_unused;
        row_entries<float, IdxT, false>(st, staged, r, i, p.a_rp, p.a_col, nullptr, p.b_rp, nA, b0, len, a_unused);
        uint8_t cls = kClsGroup;
        int nnz = 0;
        int2 win = make_int2(0, 0);
        if (nA == 0) {
            cls = kClsEmpty;
        } else if (nA <= kWave) {
            const int P = dpp_reduce_sum(len);
            if (P == 0) {
                cls = kClsEmpty;
            } else if (P <= p.th.wave_max_products && grouped_steps(nA, len) <= kWaveSmallIt) {
                // the grouped lane mapping fits: the row stays with one wavefront
                // (bitmap or hash); rows that would need the flattened mapping or
                // the large bitmap class go to the long-row kernels
                int slot_unused;
                const RowPlan pl = plan_row<IdxT, MAXIT>(nA, b0, len, tb, slot_unused);
                const IdxT safe = row_safe_index(b0, len);
                sym_row<IdxT, MAXIT>(tb, pl, safe, p.b_col, bits, p.th, cls, nnz, win);
                if (cls != kClsGroup) {
                    prod_acc += (unsigned long long)P;
                    maxp = max(maxp, (unsigned)P);
                    maxn = max(maxn, (unsigned)nnz);
                }
            }
        }
        if (lane == 0) {
            p.cls[i] = cls;
            if (cls != kClsGroup) {
                p.rnnz[i] = nnz;
                p.win[i] = win;
            }
        }
#pragma unroll
        for (int c = 0; c < kNumClasses; ++c) cnt[c] += (cls == c) ? 1u : 0u;
        if (cls == kClsGroup) group_flags |= 1u << r;
    }

    // append this wavefront's long rows to the batch's list with one atomic
    if (group_flags) {
        const bool mine = lane < kRowsPerWave && ((group_flags >> (lane & 31)) & 1u);
        const uint64_t lm = ballot(mine);
        int base = 0;
        if (lane == 0) base = (int)atomicAdd(bm.n_long, (unsigned)__popcll(lm));
        base = shfl(base, 0);
        if (mine) bm.long_list[base + mbcnt(lm)] = make_int2(q, (int)(row0 + lane));
    }

    if (lane == 0) {
        WGPart& s = s_part[w];
        s.products = prod_acc;
        for (int c = 0; c < kNumClasses; ++c) s.cls[c] = cnt[c];
        s.max_prod = maxp;
        s.max_nnz = maxn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        WGPart t = s_part[0];
        for (int v = 1; v < W; ++v) {
            t.products += s_part[v].products;
            for (int c = 0; c < kNumClasses; ++c) t.cls[c] += s_part[v].cls[c];
            t.max_prod = max(t.max_prod, s_part[v].max_prod);
            t.max_nnz = max(t.max_nnz, s_part[v].max_nnz);
        }
        p.parts[blk] = t;
    }
}

// Numeric work of one row: gather, bitmap over the window, per-word prefix
// counts, rank each product's column, accumulate, write the sorted row.
// Lanes without a product aim at the dummy word bits[pad_word(WMAX)] and the dummy slot
// vals[NCMAX], so no lane needs a branch.
template <typename T, typename IdxT, typename IdxC, int NCMAX, int WMAX, int MAXIT>
__device__ __forceinline__ void num_row_bmp(const NumArgs<T, IdxT, IdxC>& p, int64_t i, RowTable<IdxT>& tb,
                                            const RowPlan& pl, IdxT safe, int slot, bool has_entry, T a,
                                            uint32_t* bits, uint32_t* pfx, double* vals, int32_t* cols_l) {
    const int lane = lane_id();
    const int nIt = uniform_i32(pl.nIt);
    bool ok[MAXIT];
    int own[MAXIT];
    int col[MAXIT];
    T bv[MAXIT];
    row_gather<true, T, IdxT, MAXIT>(tb, pl, safe, p.b_col, p.b_val, ok, own, col, bv);
    const int2 wn = p.win[i];
    const int lo = uniform_i32(wn.x), nw = uniform_i32(wn.y);
    const int64_t cb = uniform((int64_t)p.c_rp[i]);
    const int nc = (int)(uniform((int64_t)p.c_rp[i + 1]) - cb);
    if (has_entry) tb.a[slot] = (double)a;
    clear_bitmap(bits, nw);
    for (int x = lane; x < nc; x += kWave) vals[x] = 0.0;
    wave_sync();
    int dd[MAXIT];
    double prod[MAXIT];
    const int ge0 = (lane >> uniform_i32(pl.logG)) * nIt;
#pragma unroll
    for (int t = 0; t < MAXIT; ++t) {
        if (t < nIt) {
            const int d = ok[t] ? col[t] - lo : WMAX * 32;
            dd[t] = d;
            atomicOr(&bits[pad_word(d >> 5)], 1u << (d & 31));
            const int ow = min(ge0 + t, kWave - 1);
            prod[t] = tb.a[ow] * (double)bv[t];
        }
    }
    wave_sync();
    // prefix count of set bits per word: lane l owns words [l*per, l*per + per)
    const int per = (nw + kWave - 1) / kWave;
    const int w0 = min(lane * per, nw), w1 = min(w0 + per, nw);
    int local = 0;
    for (int x = w0; x < w1; ++x) local += __popc(bits[pad_word(x)]);
    int run = dpp_incl_scan(local) - local;
    for (int x = w0; x < w1; ++x) {
        const uint32_t word = bits[pad_word(x)];
        pfx[pad_word(x)] = (uint32_t)run;
        run += __popc(word);
    }
    wave_sync();
#pragma unroll
    for (int t = 0; t < MAXIT; ++t) {
        if (t < nIt) {
            const int d = dd[t];
            const int pw = pad_word(d >> 5);
            int rk = (int)pfx[pw] + __popc(bits[pw] & ((1u << (d & 31)) - 1u));
            rk = (ok[t] && rk < nc) ? rk : NCMAX;  // rk < nc whenever the pattern matches the symbolic pass
            atomicAdd(&vals[rk], prod[t]);
            cols_l[rk] = d + lo;
        }
    }
    wave_sync();
    for (int x = lane; x < nc; x += kWave) {
        p.c_col[cb + x] = cols_l[x];
        p.c_val[cb + x] = (T)vals[x];
    }
    wave_sync();
}

// ---------------------------------------------------------------------------
// Numeric, one wavefront per row of class `want` (bitmap window of at most WMAX
// words, at most NCMAX entries).  The bitmap words and their prefix counts are
// two 32-bit LDS arrays (dense words, so the bitmap ORs of a step spread over
// the banks), and a column's rank (its position in the sorted row) is two LDS
// reads plus a popcount.
template <typename T, typename IdxT, typename IdxC, int NCMAX, int WMAX, int MAXIT, int W, bool TAB>
__global__ void __launch_bounds__(W * 64) __attribute__((amdgpu_waves_per_eu(4)))
k_num_wave_bmp(NumArgs<T, IdxT, IdxC> p0, const NumArgs<T, IdxT, IdxC>* __restrict__ P, BatchMap bm, uint8_t want) {
    __shared__ __align__(16) uint32_t s_bits[W][bitmap_stride(WMAX)];  // bitmap words (padded, + dummy)
    __shared__ uint32_t s_pfx[W][padded_words(WMAX)];                  // set bits before each word
    __shared__ double s_vals[W][NCMAX + 1];
    __shared__ int32_t s_cols[W][NCMAX + 1];
    __shared__ RowTable<IdxT> s_tb[W];
    __shared__ WaveStage<IdxT> s_stage[W];

    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    uint32_t* bits = s_bits[w];
    uint32_t* pfx = s_pfx[w];
    double* vals = s_vals[w];
    int32_t* cols_l = s_cols[w];
    RowTable<IdxT>& tb = s_tb[w];
    WaveStage<IdxT>& st = s_stage[w];

    const int gb = xcd_contiguous_block(blockIdx.x, gridDim.x);
    const int q = TAB && bm.nprod > 1 ? find_product(bm.blk_start, bm.nprod, gb) : 0;
    const int blk = gb - (TAB && bm.nprod > 1 ? bm.blk_start[q] : 0);
    const NumArgs<T, IdxT, IdxC> p = TAB ? P[q] : p0;
    const int64_t row0 = ((int64_t)blk * W + w) * kRowsPerWave;
    const int nrows = (int)max((int64_t)0, min((int64_t)kRowsPerWave, p.m - row0));
    const bool mine = lane < nrows && p.cls[row0 + lane] == want;
    uint64_t todo = ballot(mine);
    if (!todo) return;
    const bool staged = stage_chunk<IdxT>(st, row0, nrows, p.a_rp, p.a_col, p.b_rp);

    while (todo) {
        const int r = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        const int64_t i = row0 + r;
        int nA;
        IdxT b0;
        int len;
        T a;
        row_entries<T, IdxT, true>(st, staged, r, i, p.a_rp, p.a_col, p.a_val, p.b_rp, nA, b0, len, a);
        int slot;
        const RowPlan pl = plan_row<IdxT, MAXIT>(nA, b0, len, tb, slot);
        const IdxT safe = row_safe_index(b0, len);
        num_row_bmp<T, IdxT, IdxC, NCMAX, WMAX, MAXIT>(p, i, tb, pl, safe, slot, len > 0, a, bits, pfx, vals,
                                                       cols_l);
    }
}

// ---------------------------------------------------------------------------
// Numeric, one wavefront per row whose column window is too wide for a bitmap
// (at most kWaveHashProducts products): LDS hash table keyed by column, then
// the occupied slots are compacted and each entry is placed by counting the
// smaller columns.
template <typename T, typename IdxT, typename IdxC, int W, bool TAB>
__global__ void __launch_bounds__(W * 64) k_num_wave_hash(NumArgs<T, IdxT, IdxC> p0, const NumArgs<T, IdxT, IdxC>* __restrict__ P,
                                                          BatchMap bm, uint8_t want) {
    constexpr int MAXIT = kWaveHashIt;
    __shared__ uint32_t s_keys[W][kWaveHashSlots];
    __shared__ double s_hv[W][kWaveHashSlots];
    __shared__ int32_t s_ck[W][kWaveHashProducts];
    __shared__ double s_cv[W][kWaveHashProducts];
    __shared__ RowTable<IdxT> s_tb[W];
    __shared__ WaveStage<IdxT> s_stage[W];

    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    uint32_t* keys = s_keys[w];
    double* hv = s_hv[w];
    int32_t* ck = s_ck[w];
    double* cv = s_cv[w];
    RowTable<IdxT>& tb = s_tb[w];
    WaveStage<IdxT>& st = s_stage[w];
    constexpr uint32_t kEmpty = 0xFFFFFFFFu;

    const int gb = xcd_contiguous_block(blockIdx.x, gridDim.x);
    const int q = TAB && bm.nprod > 1 ? find_product(bm.blk_start, bm.nprod, gb) : 0;
    const int blk = gb - (TAB && bm.nprod > 1 ? bm.blk_start[q] : 0);
    const NumArgs<T, IdxT, IdxC> p = TAB ? P[q] : p0;
    const int64_t row0 = ((int64_t)blk * W + w) * kRowsPerWave;
    const int nrows = (int)max((int64_t)0, min((int64_t)kRowsPerWave, p.m - row0));
    const bool mine = lane < nrows && p.cls[row0 + lane] == want;
    uint64_t todo = ballot(mine);
    if (!todo) return;
    const bool staged = stage_chunk<IdxT>(st, row0, nrows, p.a_rp, p.a_col, p.b_rp);

    while (todo) {
        const int r = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        const int64_t i = row0 + r;
        int nA;
        IdxT b0;
        int len;
        T a;
        row_entries<T, IdxT, true>(st, staged, r, i, p.a_rp, p.a_col, p.a_val, p.b_rp, nA, b0, len, a);
        int slot;
        const RowPlan pl = plan_row<IdxT, MAXIT>(nA, b0, len, tb, slot);
        const IdxT safe = row_safe_index(b0, len);
        bool ok[MAXIT];
        int own[MAXIT];
        int col[MAXIT];
        T bv[MAXIT];
        row_gather<true, T, IdxT, MAXIT>(tb, pl, safe, p.b_col, p.b_val, ok, own, col, bv);
        const int64_t cb = uniform((int64_t)p.c_rp[i]);
        if (len > 0) tb.a[slot] = (double)a;
        for (int x = lane; x < kWaveHashSlots; x += kWave) {
            keys[x] = kEmpty;
            hv[x] = 0.0;
        }
        wave_sync();
#pragma unroll
        for (int t = 0; t < MAXIT; ++t) {
            if (t < uniform_i32(pl.nIt) && ok[t]) {
                const double v = tb.a[own[t]] * (double)bv[t];
                const uint32_t key = (uint32_t)col[t];
                uint32_t h = hash_col(col[t]) >> (32 - 9);
                while (true) {
                    const uint32_t old = atomicCAS(&keys[h], kEmpty, key);
                    if (old == kEmpty || old == key) break;
                    h = (h + 1) & (kWaveHashSlots - 1);
                }
                atomicAdd(&hv[h], v);
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
    }
}

}  // namespace reap
