// Wavefront-per-row kernels: symbolic (row product count, binning, per-row
// column count) and numeric (products, accumulation, ascending-column write)
// for rows whose products fit one wavefront in at most kRowSteps steps.
//
// Lane mapping of a row's products.  A lane takes kLaneEntries consecutive
// entries of one B row per step: G = ceil(L / kLaneEntries) lanes cover an A
// entry whose B row has at most L entries (L = the row's longest B row, G not
// restricted to powers of two), E = floor(64 / G) A entries share a step, and
// the row takes S = ceil(nA / E) steps.  Group g of lanes takes the entries
// g*S .. g*S + S - 1, so the entries side by side in one step are far apart in
// the row (their B rows share fewer columns).  Every load of the row is issued
// before any is used.
//
// The A entries of kRowsPerWave consecutive rows, with the extent of the B row
// each names (and, for the numeric pass, the A value), are staged in LDS once
// per chunk of rows: one 8- or 16-byte LDS read per step gives a lane its
// entry.
//
// Column sets live in a circular LDS bitmap of kWaveBitsWords 32-bit words
// indexed by the absolute column (word (col >> 5) mod kWaveBitsWords), which
// holds any row whose columns span fewer than kBmpMaxWords words: no window
// offset is subtracted per product.  In the numeric kernels word w is stored
// at position w ^ (((w >> 7) & 3) << 2): the 4-word quads inside each 16-word
// block are permuted by bits 7-8 of the word, so that words 128 apart
// (columns 4096 apart, the plane stride of a 64^3 stencil) fall in different
// LDS banks.  The symbolic kernel, whose time is its vector instructions,
// stores word w at position w and keeps its bitmap zero between rows.
// The numeric pass ranks each column by a prefix count per word taken in
// window order from the row's first word, so the rank of a column is its
// position in the sorted row (no sort).  Slots without a product aim at a
// dummy word (and a dummy accumulator) of their own lane, so the slot loops
// need no branches and all their LDS reads are issued before any is used.
#pragma once
#include "device_utils.h"
#include "kernels_numeric.h"
#include "kernels_symbolic.h"
#include "spgemm_common.h"

namespace reap {

constexpr int kLaneEntries = 4;                     // consecutive B entries per lane and step
constexpr int kRowSteps = kWaveMaxProducts / (kWave * kLaneEntries);  // steps of a wavefront row
constexpr int kBmpMask = kWaveBitsWords - 1;
constexpr int kBmpMaxWords = kWaveBitsWords - 16;   // the scan starts at a 16-aligned word
constexpr int kBmpAlloc = kWaveBitsWords + kWave;   // plus one dummy word per lane
constexpr int kNumStageRows = kRowsPerWave / 2;     // rows per staged chunk in the numeric kernels
constexpr int kNumStageCap = kStageCap / 2;

// An A entry as staged: the B row it names and, with VALS, its value.
template <typename IdxT, bool VALS>
struct StEnt {
    IdxT b0;       // first B entry of the named row
    int32_t len;   // its length (clamped to 2^24)
};
template <typename IdxT>
struct StEnt<IdxT, true> {
    IdxT b0;
    int32_t len;
    double a;
};

template <typename IdxT, bool VALS, int ROWS, int CAP>
struct alignas(16) ChunkStage {
    StEnt<IdxT, VALS> ent[CAP];    // first, so that 16-byte entries stay 16-byte aligned
    int32_t rowoff[ROWS + 1];      // entries of row r: [rowoff[r], rowoff[r + 1])
};

// Stages rows [row0, row0 + nrows) (nrows <= ROWS).  Returns false (nothing
// staged) when the chunk has more than CAP entries; rows are then staged one
// at a time by stage_row.
template <typename T, typename IdxT, bool VALS, int ROWS, int CAP>
__device__ __forceinline__ bool stage_chunk(ChunkStage<IdxT, VALS, ROWS, CAP>& st, int64_t row0, int nrows,
                                            const IdxT* __restrict__ a_rp, const int32_t* __restrict__ a_col,
                                            const T* __restrict__ a_val, const IdxT* __restrict__ b_rp) {
    const int lane = lane_id();
    int64_t rpv = 0;
    if (lane <= nrows) rpv = (int64_t)a_rp[row0 + lane];
    const int64_t rs0 = uniform_i64(shfl(rpv, 0));
    const int64_t E = uniform_i64(shfl(rpv, nrows)) - rs0;
    if (E > CAP) return false;
    if (lane <= nrows) st.rowoff[lane] = (int32_t)(rpv - rs0);
    constexpr int U = (CAP + kWave - 1) / kWave;
    int k[U];
    double a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int x = u * kWave + lane;
        k[u] = 0;
        a[u] = 0.0;
        if (x < E) {
            k[u] = a_col[rs0 + x];
            if (VALS) a[u] = (double)a_val[rs0 + x];
        }
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
            StEnt<IdxT, VALS> en;
            en.b0 = x0[u];
            en.len = (int32_t)min((int64_t)x1[u] - (int64_t)x0[u], (int64_t)(1 << 24));
            if constexpr (VALS) en.a = a[u];
            st.ent[x] = en;
        }
    }
    wave_sync();
    return true;
}

// Stages the rows row0 + r * stride (r < nrows <= ROWS) as stage_chunk stages
// consecutive rows (entry offsets per row in rowoff).  Returns false (nothing
// staged) when they have more than CAP entries.
template <typename T, typename IdxT, bool VALS, int ROWS, int CAP>
__device__ __forceinline__ bool stage_rows_strided(ChunkStage<IdxT, VALS, ROWS, CAP>& st, int64_t row0, int stride,
                                                   int nrows, const IdxT* __restrict__ a_rp,
                                                   const int32_t* __restrict__ a_col, const T* __restrict__ a_val,
                                                   const IdxT* __restrict__ b_rp) {
    const int lane = lane_id();
    int64_t beg = 0, len = 0;
    if (lane < nrows) {
        const int64_t i = row0 + (int64_t)lane * stride;
        beg = (int64_t)a_rp[i];
        len = (int64_t)a_rp[i + 1] - beg;
    }
    // each row's first A entry and its offset in the stage (wavefront-uniform)
    int64_t begs[ROWS];
    int64_t offs[ROWS + 1];
    offs[0] = 0;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        begs[r] = uniform_i64(shfl(beg, r));
        offs[r + 1] = offs[r] + (r < nrows ? uniform_i64(shfl(len, r)) : (int64_t)0);
    }
    const int64_t E = offs[ROWS];
    if (E > CAP) return false;
    if (lane <= ROWS) {
        int64_t o = offs[0];
#pragma unroll
        for (int r = 1; r <= ROWS; ++r) o = lane == r ? offs[r] : o;
        st.rowoff[lane] = (int32_t)o;
    }
    constexpr int U = (CAP + kWave - 1) / kWave;
    int k[U];
    double a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int x = u * kWave + lane;
        k[u] = 0;
        a[u] = 0.0;
        if (x < E) {
            // the row of stage entry x and its place in A
            int64_t src = begs[0] + x;
#pragma unroll
            for (int r = 1; r < ROWS; ++r)
                if (x >= offs[r]) src = begs[r] + (x - offs[r]);
            k[u] = a_col[src];
            if (VALS) a[u] = (double)a_val[src];
        }
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
            StEnt<IdxT, VALS> en;
            en.b0 = x0[u];
            en.len = (int32_t)min((int64_t)x1[u] - (int64_t)x0[u], (int64_t)(1 << 24));
            if constexpr (VALS) en.a = a[u];
            st.ent[x] = en;
        }
    }
    wave_sync();
    return true;
}

// Stages the entries of one row (at most 64) at the start of the stage.
template <typename T, typename IdxT, bool VALS, int ROWS, int CAP>
__device__ __forceinline__ void stage_row(ChunkStage<IdxT, VALS, ROWS, CAP>& st, IdxT rs, int nA,
                                          const int32_t* __restrict__ a_col, const T* __restrict__ a_val,
                                          const IdxT* __restrict__ b_rp) {
    const int lane = lane_id();
    if (lane < nA) {
        const int k = a_col[rs + lane];
        StEnt<IdxT, VALS> en;
        const IdxT x0 = b_rp[k];
        const IdxT x1 = b_rp[k + 1];
        en.b0 = x0;
        en.len = (int32_t)min((int64_t)x1 - (int64_t)x0, (int64_t)(1 << 24));
        if constexpr (VALS) en.a = (double)a_val[rs + lane];
        st.ent[lane] = en;
    }
    wave_sync();
}

// Reductions over the wavefront for any associative op (result on every lane).
template <typename V, typename Op>
__device__ __forceinline__ V wave_reduce(V v, Op op) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, kWave));
    return v;
}

// Geometry of one row's lane mapping (see the file comment).
struct RowGeo {
    int S;    // steps (uniform)
    int E;    // A entries per step (uniform)
    int g;    // this lane's group: its entry slot within a step
    int q0;   // this lane's first offset inside its entry's B row
};

// kWave / G for G = g0 .. g0 + 7, one byte each (no division in the row setup).
constexpr uint64_t pack_entries_per_step(int g0) {
    uint64_t v = 0;
    for (int x = 0; x < 8; ++x) v |= (uint64_t)(kWave / (g0 + x)) << (8 * x);
    return v;
}

// L: the row's longest B row (at most kLaneEntries * 16 for the rows that
// take this mapping); nA: its A entries (at most 64).  S is ceil(nA / E), or
// kRowSteps + 1 for a row of more steps than a wavefront row takes.
__device__ __forceinline__ RowGeo row_geo(int L, int nA) {
    RowGeo r;
    const int G = min(max(1, (L + kLaneEntries - 1) / kLaneEntries), 16);   // lanes per A entry
    const int gi = G - 1;
    r.E = (int)(((gi < 8 ? pack_entries_per_step(1) : pack_entries_per_step(9)) >> (8 * (gi & 7))) & 0xFFu);
    r.S = 1;
#pragma unroll
    for (int k = 1; k <= kRowSteps; ++k) r.S += nA > k * r.E ? 1 : 0;
    const int lane = lane_id();
    // lane / G exactly: (lane + 1/2) / G is at least 1/(2G) away from an integer
    r.g = (int)(((float)lane + 0.5f) * __builtin_amdgcn_rcpf((float)G));
    r.q0 = (lane - r.g * G) * kLaneEntries;
    return r;
}

// Reads of B's entries, kLaneEntries consecutive ones per call.  With BUF the
// reads are raw buffer loads through descriptors whose range is B's arrays:
// 32-bit byte offsets, and the hardware returns 0 for entries past the end
// of B instead of faulting, so a lane's four reads need no clamp (the host
// selects BUF when B's values take fewer than 2^31 bytes).  Without BUF the
// reads are global loads, and a lane whose four entries would pass B's last
// entry clamps them.
template <typename T, bool BUF>
struct BReader;

template <typename T>
struct BReader<T, true> {
    static_assert(kLaneEntries == 4, "a lane's entries are one 16-byte load per array");
    __amdgpu_buffer_rsrc_t col, val;
    int64_t n;   // entries of B
    __device__ __forceinline__ BReader(const int32_t* c, const T* v, int64_t nnz) : n(nnz) {
        col = __builtin_amdgcn_make_buffer_rsrc((void*)c, (short)0, (int)(nnz * 4), kBufferWord3);
        val = __builtin_amdgcn_make_buffer_rsrc((void*)v, (short)0, (int)(nnz * (int64_t)sizeof(T)), kBufferWord3);
    }
    // With values, a lane's four entries are one 16-byte load of columns and
    // one (FP32) or two (FP64) of values, written out: the vector memory unit's
    // work goes by instructions, and the compiler does not merge the
    // per-entry loads there by itself.  A lane whose four entries would pass
    // B's last one reads them one by one (each read past the range returns 0).
    // Columns alone are read entry by entry (merged by the compiler; the
    // symbolic kernel, bound by its vector instructions, keeps no range test).
    template <bool VALS>
    __device__ __forceinline__ void load(int64_t base, int32_t (&c)[kLaneEntries], T (&v)[kLaneEntries]) const {
        const int oc = (int)base * 4;
        const int ov = (int)base * (int)sizeof(T);
        if (VALS && base + kLaneEntries <= n) {
            const auto qc = __builtin_amdgcn_raw_buffer_load_b128(col, oc, 0, 0);
#pragma unroll
            for (int u = 0; u < kLaneEntries; ++u) c[u] = (int32_t)qc[u];
            if constexpr (VALS) {
                if constexpr (sizeof(T) == 8) {
                    const auto q0 = __builtin_amdgcn_raw_buffer_load_b128(val, ov, 0, 0);
                    const auto q1 = __builtin_amdgcn_raw_buffer_load_b128(val, ov + 16, 0, 0);
                    v[0] = __builtin_bit_cast(T, ((uint64_t)(uint32_t)q0[1] << 32) | (uint32_t)q0[0]);
                    v[1] = __builtin_bit_cast(T, ((uint64_t)(uint32_t)q0[3] << 32) | (uint32_t)q0[2]);
                    v[2] = __builtin_bit_cast(T, ((uint64_t)(uint32_t)q1[1] << 32) | (uint32_t)q1[0]);
                    v[3] = __builtin_bit_cast(T, ((uint64_t)(uint32_t)q1[3] << 32) | (uint32_t)q1[2]);
                } else {
                    const auto q = __builtin_amdgcn_raw_buffer_load_b128(val, ov, 0, 0);
#pragma unroll
                    for (int u = 0; u < kLaneEntries; ++u) v[u] = __builtin_bit_cast(T, (uint32_t)q[u]);
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < kLaneEntries; ++u) c[u] = __builtin_amdgcn_raw_buffer_load_b32(col, oc + 4 * u, 0, 0);
            if constexpr (VALS) {
#pragma unroll
                for (int u = 0; u < kLaneEntries; ++u) {
                    if constexpr (sizeof(T) == 8)
                        v[u] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(val, ov + 8 * u, 0, 0));
                    else
                        v[u] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(val, ov + 4 * u, 0, 0));
                }
            }
        }
    }
};

template <typename T>
struct BReader<T, false> {
    const int32_t* col;
    const T* val;
    int64_t last;
    __device__ __forceinline__ BReader(const int32_t* c, const T* v, int64_t nnz) : col(c), val(v), last(nnz - 1) {}
    template <bool VALS>
    __device__ __forceinline__ void load(int64_t base, int32_t (&c)[kLaneEntries], T (&v)[kLaneEntries]) const {
#pragma unroll
        for (int u = 0; u < kLaneEntries; ++u) {
            const int64_t idx = min(base + u, last);
            c[u] = col[idx];
            if (VALS) v[u] = val[idx];
        }
    }
};

// Issues every load of this lane's products of a row of S steps: for step t
// the lane's B entries b0 + q0 + u (u < kLaneEntries) of its A entry, rem[t]
// of which belong to the row (the rest are read but never used; lanes
// without an entry read entries 0..3).
template <int S, typename T, typename IdxT, bool VALS, bool BUF>
__device__ __forceinline__ void row_loads(const StEnt<IdxT, VALS>* ent, int nA, const RowGeo& rg,
                                          const BReader<T, BUF>& br, int32_t (&c)[S][kLaneEntries],
                                          T (&v)[S][kLaneEntries], int (&rem)[S], double (&a)[S]) {
    StEnt<IdxT, VALS> en[S];
#pragma unroll
    for (int t = 0; t < S; ++t) en[t] = ent[min(rg.g * S + t, nA - 1)];
#pragma unroll
    for (int t = 0; t < S; ++t) {
        const bool act = rg.g < rg.E && rg.g * S + t < nA;
        rem[t] = act ? en[t].len - rg.q0 : 0;
        a[t] = 0.0;
        if constexpr (VALS) a[t] = en[t].a;
        br.template load<VALS>(act ? (int64_t)en[t].b0 + rg.q0 : (int64_t)0, c[t], v[t]);
    }
}

// Circular-bitmap position of slot (t, u): the word of its column (see the
// file comment; SWZ: the numeric kernels' quad permutation), or this lane's
// dummy word when the slot holds no product.
template <int S, bool SWZ>
__device__ __forceinline__ void slot_positions(const int32_t (&c)[S][kLaneEntries], const int (&rem)[S],
                                               int (&pos)[S][kLaneEntries]) {
    const int dummy = kWaveBitsWords + lane_id();
#pragma unroll
    for (int t = 0; t < S; ++t) {
#pragma unroll
        for (int u = 0; u < kLaneEntries; ++u) {
            const uint32_t cc = (uint32_t)c[t][u];
            const int ps = SWZ ? (int)(((cc >> 5) & kBmpMask) ^ ((cc >> 10) & 12u)) : (int)((cc >> 5) & kBmpMask);
            pos[t][u] = u < rem[t] ? ps : dummy;
        }
    }
}

// Position of quad qd (words 4qd .. 4qd+3 of the circular order) in LDS: the
// word swizzle moves whole quads (it flips word bits 2-3, i.e. quad bits 0-1).
template <bool SWZ>
__device__ __forceinline__ int bmp_quad_pos(int qd) {
    qd &= kBmpMask >> 2;
    return SWZ ? qd ^ ((qd >> 5) & 3) : qd;
}

// Clears the quads holding window words [w0, w0 + nw) (nw <= kBmpMaxWords):
// one 16-byte store per quad, consecutive quads on consecutive lanes.
template <bool SWZ>
__device__ __forceinline__ void bmp_clear(uint32_t* bits, int w0, int nw) {
    const int qa = w0 >> 2, nq = ((w0 + nw - 1) >> 2) - qa + 1;
    for (int x = lane_id(); x < nq; x += kWave)
        *reinterpret_cast<uint4*>(bits + 4 * bmp_quad_pos<SWZ>(qa + x)) = make_uint4(0u, 0u, 0u, 0u);
}


// Sets the bit of every slot's column.  A lane's entries of one step are
// consecutive entries of one B row, so neighbouring ones often share a word:
// their bits are merged in registers and the word is updated once.  With
// UNCOND every slot still issues its OR, the merged ones into this lane's
// dummy word (fewer vector instructions: the symbolic kernel); without, a
// merged slot's lane sits out (fewer LDS accesses: the numeric kernels).
template <int S, bool UNCOND>
__device__ __forceinline__ void bmp_or(uint32_t* bits, const int32_t (&c)[S][kLaneEntries],
                                       const int (&pos)[S][kLaneEntries]) {
    const int dummy = kWaveBitsWords + lane_id();
#pragma unroll
    for (int t = 0; t < S; ++t) {
        uint32_t m[kLaneEntries];
        int at[kLaneEntries];
#pragma unroll
        for (int u = 0; u < kLaneEntries; ++u) {
            m[u] = 1u << (c[t][u] & 31);
            at[u] = pos[t][u];
        }
#pragma unroll
        for (int u = kLaneEntries - 1; u > 0; --u)
            if (pos[t][u] == pos[t][u - 1]) {
                m[u - 1] |= m[u];
                if (UNCOND)
                    at[u] = dummy;
                else
                    m[u] = 0u;
            }
#pragma unroll
        for (int u = 0; u < kLaneEntries; ++u)
            if (UNCOND || m[u]) atomicOr(&bits[at[u]], m[u]);
    }
}

// Set bits of the window's quads (unswizzled layout), summed over the
// wavefront; each quad is cleared once read, so the bitmap is zero again for
// the next row.
__device__ __forceinline__ int bmp_count_clear(uint32_t* bits, int w0, int nw) {
    const int qa = w0 >> 2, nq = ((w0 + nw - 1) >> 2) - qa + 1;
    int pc = 0;
    for (int x = lane_id(); x < nq; x += kWave) {
        uint4* qp = reinterpret_cast<uint4*>(bits + 4 * bmp_quad_pos<false>(qa + x));
        const uint4 q = *qp;
        *qp = make_uint4(0u, 0u, 0u, 0u);
        pc += __popc(q.x) + __popc(q.y) + __popc(q.z) + __popc(q.w);
    }
    return dpp_reduce_sum(pc);
}

// Symbolic work of one row of S steps: column window, then the distinct
// columns counted with the bitmap (or a hash set when the window is too wide).
template <int S, typename IdxT, bool BUF>
__device__ __forceinline__ void sym_row(const StEnt<IdxT, false>* ent, int nA, int P, const RowGeo& rg,
                                        const BReader<float, BUF>& br, uint32_t* bits, const Thresholds& th,
                                        uint8_t& cls, int& nnz, int2& win) {
    const int lane = lane_id();
    int32_t c[S][kLaneEntries];
    float v_unused[S][kLaneEntries];
    int rem[S];
    double a_unused[S];
    row_loads<S, float, IdxT, false, BUF>(ent, nA, rg, br, c, v_unused, rem, a_unused);
    uint32_t cmin = 0xFFFFFFFFu;
    int cmax = -1;
#pragma unroll
    for (int t = 0; t < S; ++t) {
#pragma unroll
        for (int u = 0; u < kLaneEntries; ++u) {
            const uint32_t cc = u < rem[t] ? (uint32_t)c[t][u] : 0xFFFFFFFFu;
            cmin = min(cmin, cc);
            cmax = max(cmax, (int)cc);
        }
    }
    cmin = wave_reduce(cmin, [](uint32_t x, uint32_t y) { return min(x, y); });
    cmax = dpp_reduce_max(cmax);
    const int nw = (cmax >> 5) - (int)(cmin >> 5) + 1;
    if (nw <= kBmpMaxWords && (int64_t)cmax - (int64_t)cmin + 1 <= (int64_t)th.wave_max_span) {
        int pos[S][kLaneEntries];
        slot_positions<S, false>(c, rem, pos);
        bmp_or<S, true>(bits, c, pos);
        wave_sync();
        nnz = bmp_count_clear(bits, (int)(cmin >> 5), nw);
        win = make_int2((int)cmin, nw);
        cls = nnz <= th.wave_small_nnz ? kClsWaveBmpS : kClsGroup;
    } else if (P <= th.wave_hash_products) {
        // an LDS hash set of the row's columns in the bitmap area (1 << th.wave_hash_log2
        // keys, the numeric kernel's table size; at most twice the row's products)
        const int hlog = th.wave_hash_log2, hslots = 1 << hlog;
        for (int j = 0; j < hslots / (4 * kWave); ++j)
            *reinterpret_cast<uint4*>(bits + 4 * (j * kWave + lane)) =
                make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
        wave_sync();
        int mine = 0;
#pragma unroll
        for (int t = 0; t < S; ++t) {
#pragma unroll
            for (int u = 0; u < kLaneEntries; ++u) {
                const uint32_t key = (uint32_t)c[t][u];
                if (u < rem[t]) {
                    uint32_t h = hash_col((int)key) >> (32 - hlog);
                    while (true) {
                        const uint32_t old = atomicCAS(&bits[h], 0xFFFFFFFFu, key);
                        if (old == 0xFFFFFFFFu) {
                            ++mine;
                            break;
                        }
                        if (old == key) break;
                        h = (h + 1) & (hslots - 1);
                    }
                }
            }
        }
        nnz = dpp_reduce_sum(mine);
        cls = kClsWaveHash;
        wave_sync();
#pragma unroll
        for (int j = 0; j < hslots / (4 * kWave); ++j)   // the bitmap is zero between rows
            *reinterpret_cast<uint4*>(bits + 4 * (j * kWave + lane)) = make_uint4(0u, 0u, 0u, 0u);
    }
    wave_sync();
}

// ---------------------------------------------------------------------------
// Symbolic, one wavefront per row.  Classifies every row and counts the
// distinct columns of rows that stay here: the circular LDS bitmap when the
// row's columns span at most th.wave_max_span columns (and kBmpMaxWords
// words), else an LDS hash set when the row has at most th.wave_hash_products
// products.  Rows with more than 64 entries in A, a B row longer than
// kLaneEntries * 16, more than kRowSteps steps, more than
// th.wave_max_products products, or more entries of C than the wavefront
// numeric kernels hold go to the long-row list.
// TAB: arguments from the batch table (else the by-value argument of a single product).
template <typename IdxT, bool TAB, bool BUF>
__global__ void __launch_bounds__(kWaveKernelWaves * 64) __attribute__((amdgpu_waves_per_eu(6)))
k_sym_wave(SymArgs<IdxT> p0, const SymArgs<IdxT>* __restrict__ P, BatchMap bm) {
    constexpr int W = kWaveKernelWaves;
    __shared__ __align__(16) uint32_t s_bits[W][kBmpAlloc];
    __shared__ __align__(16) ChunkStage<IdxT, false, kRowsPerWave, kStageCap> s_stage[W];
    __shared__ WGPart s_part[W];
    __shared__ int s_nnz[W];
    static_assert(W == 4, "tile sum adds four wavefronts");

    const int w = uniform_i32(threadIdx.x / kWave);
    const int lane = lane_id();
    const int gb = xcd_contiguous_block(blockIdx.x, gridDim.x);
    const int q = TAB && bm.nprod > 1 ? find_product(bm.blk_start, bm.nprod, gb) : 0;
    const int blk = gb - (TAB && bm.nprod > 1 ? bm.blk_start[q] : 0);
    const SymArgs<IdxT> p = TAB ? P[q] : p0;
    const int64_t row0 = ((int64_t)blk * W + w) * kRowsPerWave;
    uint32_t* bits = s_bits[w];
    auto& st = s_stage[w];
    // the bitmap starts zero and every row leaves it zero (its count clears
    // the window; the hash set clears its slots)
    for (int x = lane; x < kBmpAlloc / 4; x += kWave)
        *reinterpret_cast<uint4*>(bits + 4 * x) = make_uint4(0u, 0u, 0u, 0u);

    unsigned long long prod_acc = 0;
    unsigned int cnt[kNumClasses] = {0, 0, 0, 0, 0};
    unsigned int maxp = 0, maxn = 0;
    uint32_t group_flags = 0;
    // row r's results are kept by lane r and stored together at the end
    uint8_t my_cls = 0;
    int my_nnz = 0;
    int2 my_win = make_int2(0, 0);
    int wave_nnz = 0;   // a wavefront row has at most 1024 entries: no overflow

    const int nrows = (int)max((int64_t)0, min((int64_t)kRowsPerWave, p.m - row0));
    const bool staged = nrows > 0 && stage_chunk<float, IdxT, false>(st, row0, nrows, p.a_rp, p.a_col,
                                                                        (const float*)nullptr, p.b_rp);
    const BReader<float, BUF> br(p.b_col, nullptr, (int64_t)uniform(p.b_rp[p.k]));

    for (int r = 0; r < nrows; ++r) {
        const int64_t i = row0 + r;
        int nA, off;
        if (staged) {
            off = uniform_i32(st.rowoff[r]);
            nA = uniform_i32(st.rowoff[r + 1]) - off;
        } else {
            const IdxT rs = uniform(p.a_rp[i]);
            nA = (int)min((int64_t)uniform(p.a_rp[i + 1]) - (int64_t)rs, (int64_t)kWave + 1);
            off = 0;
            if (nA <= kWave) stage_row<float, IdxT, false>(st, rs, nA, p.a_col, (const float*)nullptr, p.b_rp);
        }
        uint8_t cls = kClsGroup;
        int nnz = 0;
        int rowP = 0;   // the row's products, for the statistics of wavefront rows
        int2 win = make_int2(0, 0);
        if (nA == 0) {
            cls = kClsEmpty;
        } else if (nA <= kWave) {
            const StEnt<IdxT, false>* ent = st.ent + off;
            const int len = lane < nA ? ent[lane].len : 0;
            const int P = dpp_reduce_sum(len);
            const int L = dpp_reduce_max(len);
            const bool fits = P <= p.th.wave_max_products && L <= kLaneEntries * 16;
            const RowGeo rg = row_geo(fits ? L : 1, nA);
            if (P == 0) {
                cls = kClsEmpty;
            } else if (fits && rg.S <= kRowSteps) {
                switch (rg.S) {
                    case 1: sym_row<1, IdxT, BUF>(ent, nA, P, rg, br, bits, p.th, cls, nnz, win); break;
                    case 2: sym_row<2, IdxT, BUF>(ent, nA, P, rg, br, bits, p.th, cls, nnz, win); break;
                    case 3: sym_row<3, IdxT, BUF>(ent, nA, P, rg, br, bits, p.th, cls, nnz, win); break;
                    default: sym_row<4, IdxT, BUF>(ent, nA, P, rg, br, bits, p.th, cls, nnz, win); break;
                }
                rowP = P;
            }
        }
        if (lane == r) {
            my_cls = cls;
            my_nnz = nnz;
            my_win = win;
        }
        // the statistics in scalar registers (the class, count and products are wavefront-uniform)
        const int ucls = uniform_i32(cls), unnz = uniform_i32(nnz), uP = uniform_i32(rowP);
        if (ucls != kClsGroup) {
            wave_nnz += unnz;   // the wavefront's share of its scan tile's sum
            if (ucls != kClsEmpty) {
                prod_acc += (unsigned long long)uP;
                maxp = max(maxp, (unsigned)uP);
                maxn = max(maxn, (unsigned)unnz);
            }
        }
#pragma unroll
        for (int cl = 0; cl < kNumClasses; ++cl) cnt[cl] += (ucls == cl) ? 1u : 0u;
        if (ucls == kClsGroup) group_flags |= 1u << r;
    }
    if (lane < nrows) {
        p.cls[row0 + lane] = my_cls;
        if (my_cls != kClsGroup) {
            p.rnnz[row0 + lane] = my_nnz;
            p.win[row0 + lane] = my_win;
        }
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
        s_nnz[w] = wave_nnz;
        WGPart& s = s_part[w];
        s.products = prod_acc;
        for (int cl = 0; cl < kNumClasses; ++cl) s.cls[cl] = cnt[cl];
        s.max_prod = maxp;
        s.max_nnz = maxn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        WGPart t = s_part[0];
        for (int x = 1; x < W; ++x) {
            t.products += s_part[x].products;
            for (int cl = 0; cl < kNumClasses; ++cl) t.cls[cl] += s_part[x].cls[cl];
            t.max_prod = max(t.max_prod, s_part[x].max_prod);
            t.max_nnz = max(t.max_nnz, s_part[x].max_nnz);
        }
        p.parts[blk] = t;
        const int tn = s_nnz[0] + s_nnz[1] + s_nnz[2] + s_nnz[3];
        if (tn) atomicAdd(&p.tiles[(int64_t)blk * kRowsPerBlock / kScanTile], (unsigned long long)tn);
    }
}

// The four 8-bit prefix counts of a word quad: r, r + s1, r + s2, r + s3
// (s_k the set bits of the quad's first k words).
__device__ __forceinline__ uint32_t pack_prefix4(int r, int s1, int s2, int s3) {
    return (uint32_t)(r & 0xFF) | ((uint32_t)((r + s1) & 0xFF) << 8) | ((uint32_t)((r + s2) & 0xFF) << 16) |
           ((uint32_t)((r + s3) & 0xFF) << 24);
}

// LDS of one wavefront of the compact bitmap numeric kernel.
template <typename IdxT, int NCMAX>
struct alignas(16) NumBmpLds {
    uint32_t bits[kBmpAlloc];     // circular bitmap (+ a dummy word per lane)
    uint8_t pfx[kBmpAlloc];       // entries of the row before each word (8 bits: rows hold < 256)
    double vals[NCMAX + kWave];   // accumulators by rank (+ a dummy per lane)
    int32_t cols[NCMAX + kWave];  // columns by rank
    ChunkStage<IdxT, true, kNumStageRows, kNumStageCap> st;
};

// Numeric work of one compact-class row of S steps.
template <int S, typename T, typename IdxT, typename IdxC, int NCMAX, bool BUF>
__device__ __forceinline__ void num_row_bmp(const NumArgs<T, IdxT, IdxC>& p, int64_t i,
                                            const StEnt<IdxT, true>* ent, int nA, const RowGeo& rg,
                                            const BReader<T, BUF>& br, NumBmpLds<IdxT, NCMAX>& sh) {
    const int lane = lane_id();
    int32_t c[S][kLaneEntries];
    T v[S][kLaneEntries];
    int rem[S];
    double a[S];
    row_loads<S, T, IdxT, true, BUF>(ent, nA, rg, br, c, v, rem, a);
    const int2 wn = p.win[i];
    const int lo_w = uniform_i32(wn.x) >> 5;
    const int nw = uniform_i32(wn.y);
    const int64_t cb = uniform((int64_t)p.c_rp[i]);
    const int nc = (int)(uniform((int64_t)p.c_rp[i + 1]) - cb);
    // from the 16-aligned word where the prefix scan below starts
    bmp_clear<true>(sh.bits, lo_w & ~15, nw + (lo_w & 15));
    for (int x = lane; x < nc; x += kWave) sh.vals[x] = 0.0;
    int pos[S][kLaneEntries];
    slot_positions<S, true>(c, rem, pos);
    wave_sync();
    bmp_or<S, false>(sh.bits, c, pos);
    wave_sync();
    // prefix counts in window order, in rounds of 512 words over the window:
    // in round j lane l takes the word quads s0/4 + 128 j + l and
    // s0/4 + 128 j + 64 + l (s0 the row's first word rounded down to 16), so
    // that the lanes' 16-byte reads and 4-byte writes are side by side in LDS;
    // one wavefront scan of both quads' counts, packed as two 16-bit halves
    // (a round holds at most 16384 bits), gives each quad its prefix.  Words
    // past the window get prefixes too; no rank reads them.
    {
        const int q0 = ((lo_w & kBmpMask) & ~15) >> 2;   // first quad of the window
        const int rounds = ((lo_w & 15) + nw + 8 * kWave - 1) / (8 * kWave);
        int carry = 0;
        for (int j = 0; j < rounds; ++j) {
            const int qa = bmp_quad_pos<true>(q0 + j * 2 * kWave + lane);
            const int qb = bmp_quad_pos<true>(q0 + j * 2 * kWave + kWave + lane);
            const uint4 va = *reinterpret_cast<const uint4*>(sh.bits + 4 * qa);
            const uint4 vb = *reinterpret_cast<const uint4*>(sh.bits + 4 * qb);
            // running bit counts over each quad's words
            const int a1 = __popc(va.x), a2 = a1 + __popc(va.y), a3 = a2 + __popc(va.z), ta = a3 + __popc(va.w);
            const int b1 = __popc(vb.x), b2 = b1 + __popc(vb.y), b3 = b2 + __popc(vb.z), tb = b3 + __popc(vb.w);
            const int incl = dpp_incl_scan(ta | (tb << 16));
            const int all = __builtin_amdgcn_readlane(incl, kWave - 1);
            const int ra = carry + (incl & 0xFFFF) - ta;
            const int rb = carry + (all & 0xFFFF) + (incl >> 16) - tb;
            carry += (all & 0xFFFF) + (all >> 16);
            *reinterpret_cast<uint32_t*>(sh.pfx + 4 * qa) = pack_prefix4(ra, a1, a2, a3);
            *reinterpret_cast<uint32_t*>(sh.pfx + 4 * qb) = pack_prefix4(rb, b1, b2, b3);
        }
    }
    wave_sync();
    // ranks, two steps at a time, the reads of both issued before any is
    // used; a slot without a product reads its lane's dummy word, whose
    // prefix byte (255) puts its rank out of range
#pragma unroll
    for (int t0 = 0; t0 < S; t0 += 2) {
        constexpr int H = 2;
        uint32_t rword[H][kLaneEntries];
        uint32_t rpfx[H][kLaneEntries];
#pragma unroll
        for (int dt = 0; dt < H; ++dt)
            if (t0 + dt < S)
#pragma unroll
                for (int u = 0; u < kLaneEntries; ++u) {
                    rword[dt][u] = sh.bits[pos[t0 + dt][u]];
                    rpfx[dt][u] = sh.pfx[pos[t0 + dt][u]];
                }
#pragma unroll
        for (int dt = 0; dt < H; ++dt) {
            const int t = t0 + dt;
            if (t < S) {
#pragma unroll
                for (int u = 0; u < kLaneEntries; ++u) {
                    // bits of the word below the column (width taken mod 32 by the instruction)
                    const uint32_t below = __builtin_amdgcn_ubfe(rword[dt][u], 0u, (uint32_t)c[t][u]);
                    const int rk0 = (int)(rpfx[dt][u] & 0xFFu) + __popc(below);
                    // rk0 < nc for every product whenever the pattern matches the symbolic
                    // pass; a larger rank lands in a slot that is never copied out (ranks
                    // nc .. NCMAX - 1, or this lane's dummy)
                    const int rk = min(rk0, NCMAX + lane);
                    atomicAdd(&sh.vals[rk], a[t] * (double)v[t][u]);
                    sh.cols[rk] = c[t][u];
                }
            }
        }
    }
    wave_sync();
    for (int x = lane; x < nc; x += kWave) {
        p.c_col[cb + x] = sh.cols[x];
        p.c_val[cb + x] = (T)sh.vals[x];
    }
    wave_sync();
}

// ---------------------------------------------------------------------------
// Numeric, one wavefront per row of the compact bitmap class (at most NCMAX
// entries of C, columns spanning fewer than kBmpMaxWords words): products
// held in registers, circular bitmap of the row's columns, per-word prefix
// counts in window order, each product added into the LDS slot of its
// column's rank, the row written in ascending column order.  Each wavefront
// walks the kRowsPerWave rows of its symbolic chunk, staged in halves.
template <typename T, typename IdxT, typename IdxC, int NCMAX, int W, bool TAB, bool BUF>
__global__ void __launch_bounds__(W * 64) __attribute__((amdgpu_waves_per_eu(4)))
k_num_wave_bmp(NumArgs<T, IdxT, IdxC> p0, const NumArgs<T, IdxT, IdxC>* __restrict__ P, BatchMap bm, uint8_t want) {
    static_assert(NCMAX < 255, "prefix counts are stored in 8 bits, 255 marks a dummy word");
    __shared__ __align__(16) NumBmpLds<IdxT, NCMAX> s_lds[W];

    const int w = uniform_i32(threadIdx.x / kWave);
    const int lane = lane_id();
    NumBmpLds<IdxT, NCMAX>& sh = s_lds[w];
    auto& st = sh.st;
    sh.pfx[kWaveBitsWords + lane] = 0xFF;   // dummy words: ranks out of range

    const int gb = xcd_contiguous_block(blockIdx.x, gridDim.x);
    const int q = TAB && bm.nprod > 1 ? find_product(bm.blk_start, bm.nprod, gb) : 0;
    const int blk = gb - (TAB && bm.nprod > 1 ? bm.blk_start[q] : 0);
    const NumArgs<T, IdxT, IdxC> p = TAB ? P[q] : p0;
    // the workgroup's rows rb .. rb + W * kRowsPerWave - 1, interleaved: row j
    // of wavefront w is rb + w + W * j, so that the wavefronts of a workgroup
    // work on neighbouring rows at the same time and share in L1 the B rows
    // those read
    const int64_t rb = (int64_t)blk * W * kRowsPerWave;
    const int64_t my_row = rb + w + (int64_t)W * lane;
    const uint64_t todo_all = ballot(lane < kRowsPerWave && my_row < p.m && p.cls[my_row] == want);
    if (!todo_all) return;
    const BReader<T, BUF> br(p.b_col, p.b_val, (int64_t)uniform(p.b_rp[p.k]));

    for (int h = 0; h < kRowsPerWave / kNumStageRows; ++h) {
        const int64_t row0 = rb + w + (int64_t)W * (h * kNumStageRows);
        uint64_t todo = (todo_all >> (h * kNumStageRows)) & ((1ull << kNumStageRows) - 1);
        if (!todo) continue;
        const int nrows = (int)max((int64_t)0, min((int64_t)kNumStageRows, (p.m - row0 + W - 1) / W));
        const bool staged = stage_rows_strided<T, IdxT, true>(st, row0, W, nrows, p.a_rp, p.a_col, p.a_val, p.b_rp);
        while (todo) {
            const int r = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const int64_t i = row0 + (int64_t)W * r;
            int nA, off;
            if (staged) {
                off = uniform_i32(st.rowoff[r]);
                nA = uniform_i32(st.rowoff[r + 1]) - off;
            } else {
                const IdxT rs = uniform(p.a_rp[i]);
                nA = (int)((int64_t)uniform(p.a_rp[i + 1]) - (int64_t)rs);
                off = 0;
                stage_row<T, IdxT, true>(st, rs, nA, p.a_col, p.a_val, p.b_rp);
            }
            const StEnt<IdxT, true>* ent = st.ent + off;
            const int L = dpp_reduce_max(lane < nA ? ent[lane].len : 0);
            const RowGeo rg = row_geo(L, nA);
            switch (rg.S) {
                case 1: num_row_bmp<1, T, IdxT, IdxC, NCMAX, BUF>(p, i, ent, nA, rg, br, sh); break;
                case 2: num_row_bmp<2, T, IdxT, IdxC, NCMAX, BUF>(p, i, ent, nA, rg, br, sh); break;
                case 3: num_row_bmp<3, T, IdxT, IdxC, NCMAX, BUF>(p, i, ent, nA, rg, br, sh); break;
                default: num_row_bmp<4, T, IdxT, IdxC, NCMAX, BUF>(p, i, ent, nA, rg, br, sh); break;
            }
        }
    }
}

// Numeric work of one hash-class row of S steps: an LDS hash table of HS
// slots keyed by column (rows of at most HS / 2 products), then the occupied
// slots are compacted to the front of the same table and each entry is
// placed by counting the smaller columns.
template <int S, int HS, typename T, typename IdxT, typename IdxC, bool BUF>
__device__ __forceinline__ void num_row_hash(const NumArgs<T, IdxT, IdxC>& p, int64_t i,
                                             const StEnt<IdxT, true>* ent, int nA, const RowGeo& rg,
                                             const BReader<T, BUF>& br, uint32_t* keys, double* hv) {
    constexpr int NC = HS / 2;
    constexpr int NCU = NC / kWave;
    constexpr int LOG = HS == 1024 ? 10 : 9;
    static_assert(HS == (1 << LOG), "512 or 1024 slots");
    constexpr uint32_t kEmpty = 0xFFFFFFFFu;
    const int lane = lane_id();
    int32_t c[S][kLaneEntries];
    T v[S][kLaneEntries];
    int rem[S];
    double a[S];
    row_loads<S, T, IdxT, true, BUF>(ent, nA, rg, br, c, v, rem, a);
    const int64_t cb = uniform((int64_t)p.c_rp[i]);
    for (int x = lane; x < HS; x += kWave) {
        keys[x] = kEmpty;
        hv[x] = 0.0;
    }
    wave_sync();
#pragma unroll
    for (int t = 0; t < S; ++t) {
#pragma unroll
        for (int u = 0; u < kLaneEntries; ++u) {
            if (u < rem[t]) {
                const uint32_t key = (uint32_t)c[t][u];
                uint32_t hs = hash_col((int)key) >> (32 - LOG);
                while (true) {
                    const uint32_t old = atomicCAS(&keys[hs], kEmpty, key);
                    if (old == kEmpty || old == key) break;
                    hs = (hs + 1) & (HS - 1);
                }
                atomicAdd(&hv[hs], a[t] * (double)v[t][u]);
            }
        }
    }
    wave_sync();
    // compaction in place: an entry moves to a slot at or before its own, and
    // every lane reads its slot before any lane writes
    int nc = 0;
    for (int x0 = 0; x0 < HS; x0 += kWave) {
        const int x = x0 + lane;
        const uint32_t kx = keys[x];
        const double vx = hv[x];
        const bool occ = kx != kEmpty;
        const uint64_t om = ballot(occ);
        wave_sync();
        if (occ && nc + mbcnt(om) < NC) {
            const int pos = nc + mbcnt(om);
            keys[pos] = kx;
            hv[pos] = vx;
        }
        nc += __popcll(om);
        wave_sync();
    }
    nc = min(nc, NC);
    int key[NCU];
    int rank[NCU];
#pragma unroll
    for (int u = 0; u < NCU; ++u) {
        const int e = u * kWave + lane;
        key[u] = (e < nc) ? (int)keys[e] : INT32_MAX;
        rank[u] = 0;
    }
    for (int j = 0; j < nc; ++j) {
        const int kj = (int)keys[j];
#pragma unroll
        for (int u = 0; u < NCU; ++u) rank[u] += (kj < key[u]) ? 1 : 0;
    }
#pragma unroll
    for (int u = 0; u < NCU; ++u) {
        const int e = u * kWave + lane;
        if (e < nc) {
            p.c_col[cb + rank[u]] = key[u];
            p.c_val[cb + rank[u]] = (T)hv[e];
        }
    }
    wave_sync();
}

// ---------------------------------------------------------------------------
// Numeric, one wavefront per row whose columns span too wide a window for the
// bitmap (at most HS / 2 products; HS = 512 or 1024 hash slots).
template <typename T, typename IdxT, typename IdxC, int W, bool TAB, bool BUF, int HS>
__global__ void __launch_bounds__(W * 64)
k_num_wave_hash(NumArgs<T, IdxT, IdxC> p0, const NumArgs<T, IdxT, IdxC>* __restrict__ P, BatchMap bm, uint8_t want) {
    __shared__ __align__(16) uint32_t s_keys[W][HS];
    __shared__ double s_hv[W][HS];
    __shared__ __align__(16) ChunkStage<IdxT, true, kNumStageRows, kNumStageCap> s_stage[W];

    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    auto& st = s_stage[w];

    const int gb = xcd_contiguous_block(blockIdx.x, gridDim.x);
    const int q = TAB && bm.nprod > 1 ? find_product(bm.blk_start, bm.nprod, gb) : 0;
    const int blk = gb - (TAB && bm.nprod > 1 ? bm.blk_start[q] : 0);
    const NumArgs<T, IdxT, IdxC> p = TAB ? P[q] : p0;
    const int64_t rowc = ((int64_t)blk * W + w) * kRowsPerWave;
    const int nall = (int)max((int64_t)0, min((int64_t)kRowsPerWave, p.m - rowc));
    const uint64_t todo_all = ballot(lane < nall && p.cls[rowc + lane] == want);
    if (!todo_all) return;
    const BReader<T, BUF> br(p.b_col, p.b_val, (int64_t)uniform(p.b_rp[p.k]));

    for (int h = 0; h < kRowsPerWave / kNumStageRows; ++h) {
        const int64_t row0 = rowc + h * kNumStageRows;
        uint64_t todo = (todo_all >> (h * kNumStageRows)) & ((1ull << kNumStageRows) - 1);
        if (!todo) continue;
        const int nrows = (int)max((int64_t)0, min((int64_t)kNumStageRows, p.m - row0));
        const bool staged = stage_chunk<T, IdxT, true>(st, row0, nrows, p.a_rp, p.a_col, p.a_val, p.b_rp);
        while (todo) {
            const int r = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const int64_t i = row0 + r;
            int nA, off;
            if (staged) {
                off = uniform_i32(st.rowoff[r]);
                nA = uniform_i32(st.rowoff[r + 1]) - off;
            } else {
                const IdxT rs = uniform(p.a_rp[i]);
                nA = (int)((int64_t)uniform(p.a_rp[i + 1]) - (int64_t)rs);
                off = 0;
                stage_row<T, IdxT, true>(st, rs, nA, p.a_col, p.a_val, p.b_rp);
            }
            const StEnt<IdxT, true>* ent = st.ent + off;
            const int L = dpp_reduce_max(lane < nA ? ent[lane].len : 0);
            const RowGeo rg = row_geo(L, nA);
            uint32_t* keys = s_keys[w];
            double* hv = s_hv[w];
            switch (rg.S) {
                case 1: num_row_hash<1, HS, T, IdxT, IdxC, BUF>(p, i, ent, nA, rg, br, keys, hv); break;
                case 2: num_row_hash<2, HS, T, IdxT, IdxC, BUF>(p, i, ent, nA, rg, br, keys, hv); break;
                case 3: num_row_hash<3, HS, T, IdxT, IdxC, BUF>(p, i, ent, nA, rg, br, keys, hv); break;
                default: num_row_hash<4, HS, T, IdxT, IdxC, BUF>(p, i, ent, nA, rg, br, keys, hv); break;
            }
        }
    }
}

}  // namespace reap
