// Host side of the C ABI declared in include/reap_spgemm.h: plan, workspace,
// argument checks and kernel launches on the plan's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "../../include/reap_spgemm.h"
#include "kernels_long.h"
#include "kernels_numeric.h"
#include "kernels_scan.h"
#include "kernels_symbolic.h"
#include "kernels_wave.h"
#include "spgemm_common.h"

using namespace reap;

namespace {

enum Phase { kPhSymbolic = 0, kPhScan, kPhNumWave, kPhNumHash, kPhNumGroup, kPhNumAll, kNumPhases };

struct Workspace {
    void* base = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct reap_spgemm_s {
    int device = 0;
    int num_cus = 256;
    hipStream_t stream = nullptr;
    reap_dtype_t dtype = REAP_F64;
    reap_index_t cidx = REAP_I32;
    Thresholds th{};
    bool validate = false;
    bool profile = false;
    bool debug_sync = false;  // REAP_DEBUG_SYNC=1: synchronise and log after every kernel

    Workspace ws;          // per-row arrays, counters, partials
    Workspace gvals;       // long-row FP64 accumulators (FP32 output only)
    int64_t ws_rows = -1;  // rows the per-row arrays were carved for

    uint8_t* cls = nullptr;
    int32_t* rnnz = nullptr;
    int2* win = nullptr;
    int32_t* group_rows = nullptr;
    Counters* ctr = nullptr;
    WGPart* parts = nullptr;
    long long* tiles = nullptr;
    int nparts = 0;
    int ntiles = 0;

    Counters* h_ctr = nullptr;  // pinned host mirror

    // state of the last symbolic pass
    bool have_symbolic = false;
    int64_t m = 0, k = 0, n = 0, a_nnz = 0, b_nnz = 0;
    reap_index_t in_idx = REAP_I32;
    int64_t c_nnz = 0;
    int group_grid = 0;
    int64_t gvals_stride = 0;

    hipEvent_t ev[2 * kNumPhases] = {};
    bool events_ok = false;
    bool phase_used[kNumPhases] = {};   // recorded and not yet folded into acc_ms
    double acc_ms[kNumPhases] = {};     // accumulated device time per phase
    long long acc_calls[kNumPhases] = {};
};

namespace {

constexpr int kSymWaves = 4;
constexpr int kNumWavesS = 4;
constexpr int kNumWavesH = 4;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }


#define REAP_HIP(call)                                   \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return REAP_ERR_HIP;       \
    } while (0)

#define REAP_LAUNCH_CHECK()                              \
    do {                                                 \
        hipError_t e_ = hipGetLastError();               \
        if (e_ != hipSuccess) return REAP_ERR_HIP;       \
    } while (0)

int clampi(int v, int lo, int hi, int dflt) {
    if (v == 0) return dflt;
    if (v < 0) return lo;
    return std::min(std::max(v, lo), hi);
}

reap_status_t check_csr(const reap_csr_t* M, reap_dtype_t dt) {
    (void)dt;
    if (!M) return REAP_ERR_INVALID_ARG;
    if (M->rows < 0 || M->cols < 0 || M->nnz < 0) return REAP_ERR_INVALID_ARG;
    if (M->cols > INT32_MAX) return REAP_ERR_INVALID_ARG;  // int32 column indices
    if (M->row_ptr_type != REAP_I32 && M->row_ptr_type != REAP_I64) return REAP_ERR_INVALID_ARG;
    if (M->row_ptr_type == REAP_I32 && M->nnz > INT32_MAX) return REAP_ERR_INVALID_ARG;
    if (!M->row_ptr) return REAP_ERR_INVALID_ARG;
    if (M->nnz > 0 && (!M->col_idx || !M->values)) return REAP_ERR_INVALID_ARG;
    return REAP_OK;
}

reap_status_t ensure_workspace(reap_spgemm_s* p, int64_t m) {
    if (p->ws_rows >= m && p->ws.base) return REAP_OK;
    const int64_t mm = std::max<int64_t>(m, 1);
    const int sym_blocks = (int)((mm + kSymWaves * kRowsPerWave - 1) / (kSymWaves * kRowsPerWave));
    const int ntiles = (int)((mm + kScanTile - 1) / kScanTile);
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t o_ctr = carve(sizeof(Counters));
    const size_t o_cls = carve((size_t)mm);
    const size_t o_rnnz = carve((size_t)mm * 4);
    const size_t o_win = carve((size_t)mm * 8);
    const size_t o_grp = carve((size_t)mm * 4);
    const size_t o_parts = carve((size_t)sym_blocks * sizeof(WGPart));
    const size_t o_tiles = carve((size_t)ntiles * 8);
    if (p->ws.base) {
        (void)hipFree(p->ws.base);
        p->ws.base = nullptr;
        p->ws.bytes = 0;
    }
    void* base = nullptr;
    if (hipMalloc(&base, off) != hipSuccess) {
        (void)hipGetLastError();
        p->ws_rows = -1;
        return REAP_ERR_OUT_OF_MEMORY;
    }
    char* b = static_cast<char*>(base);
    p->ws.base = base;
    p->ws.bytes = off;
    p->ctr = reinterpret_cast<Counters*>(b + o_ctr);
    p->cls = reinterpret_cast<uint8_t*>(b + o_cls);
    p->rnnz = reinterpret_cast<int32_t*>(b + o_rnnz);
    p->win = reinterpret_cast<int2*>(b + o_win);
    p->group_rows = reinterpret_cast<int32_t*>(b + o_grp);
    p->parts = reinterpret_cast<WGPart*>(b + o_parts);
    p->tiles = reinterpret_cast<long long*>(b + o_tiles);
    p->ws_rows = mm;
    return REAP_OK;
}

// With REAP_DEBUG_SYNC=1 in the environment every kernel launch is followed by
// a stream synchronisation and a line on stderr, so a failing kernel is named.
void debug_step(reap_spgemm_s* p, const char* kernel) {
    if (!p->debug_sync) return;
    fprintf(stderr, "[reap] %s launched\n", kernel);
    fflush(stderr);
    const hipError_t e = hipStreamSynchronize(p->stream);
    fprintf(stderr, "[reap] %s done (%s)\n", kernel, hipGetErrorString(e));
    fflush(stderr);
}

void ev_record(reap_spgemm_s* p, int phase, bool end) {
    if (p->profile && p->events_ok) {
        (void)hipEventRecord(p->ev[2 * phase + (end ? 1 : 0)], p->stream);
        if (end) p->phase_used[phase] = true;
    }
}

// Adds the elapsed time of every recorded phase to the totals.  Call only
// after the plan's stream has been synchronised.
void fold_events(reap_spgemm_s* p) {
    if (!p->profile || !p->events_ok) return;
    for (int i = 0; i < kNumPhases; ++i) {
        if (!p->phase_used[i]) continue;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]) == hipSuccess) {
            p->acc_ms[i] += ms;
            p->acc_calls[i] += 1;
        } else {
            (void)hipGetLastError();
        }
        p->phase_used[i] = false;
    }
}

template <typename IdxT>
reap_status_t run_symbolic(reap_spgemm_s* p, const reap_csr_t* A, const reap_csr_t* B, void* c_row_ptr) {
    const int64_t m = A->rows;
    SymArgs<IdxT> a;
    a.m = m;
    a.n = B->cols;
    a.a_rp = static_cast<const IdxT*>(A->row_ptr);
    a.a_col = A->col_idx;
    a.b_rp = static_cast<const IdxT*>(B->row_ptr);
    a.b_col = B->col_idx;
    a.cls = p->cls;
    a.rnnz = p->rnnz;
    a.win = p->win;
    a.group_rows = p->group_rows;
    a.ctr = p->ctr;
    a.parts = p->parts;
    a.th = p->th;

    const int sym_blocks = (int)((m + kSymWaves * kRowsPerWave - 1) / (kSymWaves * kRowsPerWave));
    const int ntiles = (int)((m + kScanTile - 1) / kScanTile);

    ev_record(p, kPhSymbolic, false);
    if (sym_blocks > 0) {
        hipLaunchKernelGGL(k_sym_wave<IdxT>, dim3(sym_blocks), dim3(kSymWaves * kWave), 0, p->stream, a);
        REAP_LAUNCH_CHECK();
        debug_step(p, "k_sym_wave");
        // the long-row count is known on the device only: a fixed grid walks the list
        const int lgrid = (int)std::max<int64_t>(1, std::min<int64_t>(m, (int64_t)p->num_cus * 2));
        hipLaunchKernelGGL(k_long_sym<IdxT>, dim3(lgrid), dim3(kLongThreads), 0, p->stream, a);
        REAP_LAUNCH_CHECK();
        debug_step(p, "k_long_sym");
    }
    ev_record(p, kPhSymbolic, true);
    ev_record(p, kPhScan, false);
    if (ntiles > 0) {
        hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(kScanThreads), 0, p->stream, p->rnnz, m, p->tiles);
        REAP_LAUNCH_CHECK();
        debug_step(p, "k_scan_tiles");
    }
    if (p->cidx == REAP_I32) {
        hipLaunchKernelGGL(k_scan_spine<int32_t>, dim3(1), dim3(1024), 0, p->stream, p->tiles, ntiles, p->parts,
                           sym_blocks, p->ctr, static_cast<int32_t*>(c_row_ptr), m);
        REAP_LAUNCH_CHECK();
        if (ntiles > 0) {
            hipLaunchKernelGGL(k_scan_apply<int32_t>, dim3(ntiles), dim3(kScanThreads), 0, p->stream, p->rnnz, m,
                               p->tiles, static_cast<int32_t*>(c_row_ptr));
            REAP_LAUNCH_CHECK();
        }
    } else {
        hipLaunchKernelGGL(k_scan_spine<int64_t>, dim3(1), dim3(1024), 0, p->stream, p->tiles, ntiles, p->parts,
                           sym_blocks, p->ctr, static_cast<int64_t*>(c_row_ptr), m);
        REAP_LAUNCH_CHECK();
        if (ntiles > 0) {
            hipLaunchKernelGGL(k_scan_apply<int64_t>, dim3(ntiles), dim3(kScanThreads), 0, p->stream, p->rnnz, m,
                               p->tiles, static_cast<int64_t*>(c_row_ptr));
            REAP_LAUNCH_CHECK();
        }
    }
    ev_record(p, kPhScan, true);
    return REAP_OK;
}

template <typename IdxT>
reap_status_t run_validate(reap_spgemm_s* p, const reap_csr_t* M, unsigned bit) {
    const int64_t n = M->rows + 1;
    const int blocks = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_validate<IdxT>, dim3(blocks), dim3(256), 0, p->stream, static_cast<const IdxT*>(M->row_ptr),
                       M->col_idx, M->rows, M->cols, M->nnz, p->ctr, bit);
    REAP_LAUNCH_CHECK();
    return REAP_OK;
}

template <typename T, typename IdxT, typename IdxC>
reap_status_t run_numeric(reap_spgemm_s* p, const reap_csr_t* A, const reap_csr_t* B, const void* c_row_ptr,
                          int32_t* c_col, void* c_val) {
    NumArgs<T, IdxT, IdxC> a;
    a.m = A->rows;
    a.n = B->cols;
    a.a_rp = static_cast<const IdxT*>(A->row_ptr);
    a.a_col = A->col_idx;
    a.a_val = static_cast<const T*>(A->values);
    a.b_rp = static_cast<const IdxT*>(B->row_ptr);
    a.b_col = B->col_idx;
    a.b_val = static_cast<const T*>(B->values);
    a.c_rp = static_cast<const IdxC*>(c_row_ptr);
    a.c_col = c_col;
    a.c_val = static_cast<T*>(c_val);
    a.cls = p->cls;
    a.win = p->win;
    a.group_rows = p->group_rows;
    a.ctr = p->ctr;
    a.gvals = static_cast<double*>(p->gvals.base);
    a.gvals_stride = p->gvals_stride;
    a.th = p->th;
    const int64_t m = A->rows;
    const Counters& h = *p->h_ctr;

    ev_record(p, kPhNumAll, false);
    ev_record(p, kPhNumWave, false);
    if (h.cls[kClsWaveBmpS] > 0) {
        const int blocks = (int)((m + kNumWavesS * kRowsPerWave - 1) / (kNumWavesS * kRowsPerWave));
        hipLaunchKernelGGL((k_num_wave_bmp<T, IdxT, IdxC, kWaveSmallNnz, kWaveSmallWords, kWaveSmallIt, kNumWavesS>), dim3(blocks),
                           dim3(kNumWavesS * kWave), 0, p->stream, a, (uint8_t)kClsWaveBmpS);
        REAP_LAUNCH_CHECK();
        debug_step(p, "k_num_wave_bmp (small)");
    }
    ev_record(p, kPhNumWave, true);
    ev_record(p, kPhNumHash, false);
    if (h.cls[kClsWaveHash] > 0) {
        const int blocks = (int)((m + kNumWavesH * kRowsPerWave - 1) / (kNumWavesH * kRowsPerWave));
        hipLaunchKernelGGL((k_num_wave_hash<T, IdxT, IdxC, kNumWavesH>), dim3(blocks), dim3(kNumWavesH * kWave), 0,
                           p->stream, a, (uint8_t)kClsWaveHash);
        REAP_LAUNCH_CHECK();
        debug_step(p, "k_num_wave_hash");
    }
    ev_record(p, kPhNumHash, true);
    ev_record(p, kPhNumGroup, false);
    if (h.n_group > 0) {
        hipLaunchKernelGGL((k_long_num<T, IdxT, IdxC>), dim3(p->group_grid), dim3(kLongThreads), 0, p->stream, a);
        REAP_LAUNCH_CHECK();
        debug_step(p, "k_long_num");
    }
    ev_record(p, kPhNumGroup, true);
    ev_record(p, kPhNumAll, true);
    return REAP_OK;
}

}  // namespace

extern "C" {

const char* reap_status_string(reap_status_t s) {
    switch (s) {
        case REAP_OK: return "ok";
        case REAP_ERR_INVALID_ARG: return "invalid argument";
        case REAP_ERR_BAD_CSR: return "malformed CSR operand";
        case REAP_ERR_INDEX_OVERFLOW: return "nnz(C) does not fit the C row-pointer type";
        case REAP_ERR_OUT_OF_MEMORY: return "out of device memory";
        case REAP_ERR_STATE: return "numeric call does not match a preceding symbolic call";
        case REAP_ERR_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char* reap_version(void) { return "0.1.0"; }

reap_status_t reap_spgemm_create(reap_spgemm_t* plan, reap_dtype_t dtype, reap_index_t c_row_ptr_type, void* stream,
                                 const reap_options_t* opts) {
    if (!plan) return REAP_ERR_INVALID_ARG;
    *plan = nullptr;
    if (dtype != REAP_F32 && dtype != REAP_F64) return REAP_ERR_INVALID_ARG;
    if (c_row_ptr_type != REAP_I32 && c_row_ptr_type != REAP_I64) return REAP_ERR_INVALID_ARG;
    reap_spgemm_s* p = new (std::nothrow) reap_spgemm_s();
    if (!p) return REAP_ERR_OUT_OF_MEMORY;
    p->dtype = dtype;
    p->cidx = c_row_ptr_type;
    p->stream = static_cast<hipStream_t>(stream);
    reap_options_t o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    p->validate = o.validate != 0;
    p->profile = o.profile != 0;
    const char* dbg = std::getenv("REAP_DEBUG_SYNC");
    p->debug_sync = dbg && dbg[0] == '1';
    p->th.wave_max_products = clampi(o.wave_max_products, 0, kWaveMaxProducts, kWaveMaxProducts);
    p->th.wave_max_span = clampi(o.wave_max_span, 0, 32 * kWaveBitsWords, 32 * kWaveBitsWords);
    p->th.wave_hash_products = clampi(o.wave_hash_products, 0, kWaveHashProducts, kWaveHashProducts);
    p->th.wave_small_nnz = clampi(o.wave_small_values, 0, kWaveSmallNnz, kWaveSmallNnz);
    p->th.group_lds_span = clampi(o.group_lds_span, 32, 32 * kGroupBitsWords, 32 * kGroupBitsWords) / 32 * 32;

    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&p->num_cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&p->h_ctr), sizeof(Counters), hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete p;
        return REAP_ERR_HIP;
    }
    std::memset(p->h_ctr, 0, sizeof(Counters));
    if (p->profile) {
        p->events_ok = true;
        for (int i = 0; i < 2 * kNumPhases; ++i)
            if (hipEventCreate(&p->ev[i]) != hipSuccess) p->events_ok = false;
    }
    *plan = p;
    return REAP_OK;
}

reap_status_t reap_spgemm_destroy(reap_spgemm_t p) {
    if (!p) return REAP_OK;
    (void)hipStreamSynchronize(p->stream);
    if (p->ws.base) (void)hipFree(p->ws.base);
    if (p->gvals.base) (void)hipFree(p->gvals.base);
    if (p->h_ctr) (void)hipHostFree(p->h_ctr);
    for (int i = 0; i < 2 * kNumPhases; ++i)
        if (p->ev[i]) (void)hipEventDestroy(p->ev[i]);
    delete p;
    return REAP_OK;
}

reap_status_t reap_spgemm_symbolic(reap_spgemm_t p, const reap_csr_t* A, const reap_csr_t* B, void* c_row_ptr,
                                   int64_t* c_nnz, int64_t* n_products, size_t* workspace_bytes) {
    if (!p || !c_nnz || !c_row_ptr) return REAP_ERR_INVALID_ARG;
    reap_status_t st;
    if ((st = check_csr(A, p->dtype)) != REAP_OK) return st;
    if ((st = check_csr(B, p->dtype)) != REAP_OK) return st;
    if (A->cols != B->rows) return REAP_ERR_INVALID_ARG;
    if (A->row_ptr_type != B->row_ptr_type) return REAP_ERR_INVALID_ARG;
    if (A->rows > INT32_MAX - 1) return REAP_ERR_INVALID_ARG;  // row ids are stored as int32
    p->have_symbolic = false;

    if ((st = ensure_workspace(p, A->rows)) != REAP_OK) return st;
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, p->stream, p->ctr);
    REAP_LAUNCH_CHECK();

    if (p->validate) {
        if (A->row_ptr_type == REAP_I32) {
            if ((st = run_validate<int32_t>(p, A, 1u)) != REAP_OK) return st;
            if ((st = run_validate<int32_t>(p, B, 2u)) != REAP_OK) return st;
        } else {
            if ((st = run_validate<int64_t>(p, A, 1u)) != REAP_OK) return st;
            if ((st = run_validate<int64_t>(p, B, 2u)) != REAP_OK) return st;
        }
        REAP_HIP(hipMemcpyAsync(p->h_ctr, p->ctr, sizeof(Counters), hipMemcpyDeviceToHost, p->stream));
        REAP_HIP(hipStreamSynchronize(p->stream));
        if (p->h_ctr->bad_csr) return REAP_ERR_BAD_CSR;
    }

    st = (A->row_ptr_type == REAP_I32) ? run_symbolic<int32_t>(p, A, B, c_row_ptr)
                                       : run_symbolic<int64_t>(p, A, B, c_row_ptr);
    if (st != REAP_OK) return st;
    REAP_HIP(hipMemcpyAsync(p->h_ctr, p->ctr, sizeof(Counters), hipMemcpyDeviceToHost, p->stream));
    REAP_HIP(hipStreamSynchronize(p->stream));
    fold_events(p);  // this call's symbolic phases and the previous numeric call's phases
    const Counters& h = *p->h_ctr;
    const int64_t nnz = (int64_t)h.nnz;

    // long rows: one workgroup per list entry up to two per CU; FP32 output
    // needs an FP64 accumulator per workgroup (one segment of the widest row)
    p->group_grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)h.n_group, (int64_t)p->num_cus * 2));
    p->gvals_stride = 0;
    if (p->dtype == REAP_F32 && h.n_group > 0) {
        const int64_t stride =
            std::max<int64_t>(1, std::min<int64_t>((int64_t)h.max_group_nnz, (int64_t)p->th.group_lds_span));
        const size_t need = (size_t)stride * (size_t)p->group_grid * sizeof(double);
        if (need > p->gvals.bytes) {
            if (p->gvals.base) (void)hipFree(p->gvals.base);
            p->gvals.base = nullptr;
            p->gvals.bytes = 0;
            if (hipMalloc(&p->gvals.base, need) != hipSuccess) {
                (void)hipGetLastError();
                return REAP_ERR_OUT_OF_MEMORY;
            }
            p->gvals.bytes = need;
        }
        p->gvals_stride = stride;
    }

    *c_nnz = nnz;
    if (n_products) *n_products = (int64_t)h.products;
    if (workspace_bytes) *workspace_bytes = p->ws.bytes + p->gvals.bytes;
    if (p->cidx == REAP_I32 && nnz > INT32_MAX) return REAP_ERR_INDEX_OVERFLOW;

    p->have_symbolic = true;
    p->m = A->rows;
    p->k = A->cols;
    p->n = B->cols;
    p->a_nnz = A->nnz;
    p->b_nnz = B->nnz;
    p->in_idx = A->row_ptr_type;
    p->c_nnz = nnz;
    return REAP_OK;
}

reap_status_t reap_spgemm_numeric(reap_spgemm_t p, const reap_csr_t* A, const reap_csr_t* B, const void* c_row_ptr,
                                  int32_t* c_col_idx, void* c_values) {
    if (!p) return REAP_ERR_INVALID_ARG;
    reap_status_t st;
    if ((st = check_csr(A, p->dtype)) != REAP_OK) return st;
    if ((st = check_csr(B, p->dtype)) != REAP_OK) return st;
    if (!c_row_ptr) return REAP_ERR_INVALID_ARG;
    if (!p->have_symbolic) return REAP_ERR_STATE;
    if (A->rows != p->m || A->cols != p->k || B->cols != p->n || A->nnz != p->a_nnz || B->nnz != p->b_nnz ||
        A->row_ptr_type != p->in_idx || B->row_ptr_type != p->in_idx)
        return REAP_ERR_STATE;
    if (p->c_nnz > 0 && (!c_col_idx || !c_values)) return REAP_ERR_INVALID_ARG;
    if (p->c_nnz == 0) return REAP_OK;
    const bool i32 = p->in_idx == REAP_I32, c32 = p->cidx == REAP_I32;
    if (p->dtype == REAP_F64) {
        if (i32 && c32) return run_numeric<double, int32_t, int32_t>(p, A, B, c_row_ptr, c_col_idx, c_values);
        if (i32 && !c32) return run_numeric<double, int32_t, int64_t>(p, A, B, c_row_ptr, c_col_idx, c_values);
        if (!i32 && c32) return run_numeric<double, int64_t, int32_t>(p, A, B, c_row_ptr, c_col_idx, c_values);
        return run_numeric<double, int64_t, int64_t>(p, A, B, c_row_ptr, c_col_idx, c_values);
    }
    if (i32 && c32) return run_numeric<float, int32_t, int32_t>(p, A, B, c_row_ptr, c_col_idx, c_values);
    if (i32 && !c32) return run_numeric<float, int32_t, int64_t>(p, A, B, c_row_ptr, c_col_idx, c_values);
    if (!i32 && c32) return run_numeric<float, int64_t, int32_t>(p, A, B, c_row_ptr, c_col_idx, c_values);
    return run_numeric<float, int64_t, int64_t>(p, A, B, c_row_ptr, c_col_idx, c_values);
}

reap_status_t reap_spgemm_bin_stats(reap_spgemm_t p, reap_bin_stats_t* out) {
    if (!p || !out) return REAP_ERR_INVALID_ARG;
    if (!p->have_symbolic) return REAP_ERR_STATE;
    const Counters& h = *p->h_ctr;
    out->empty = (int64_t)h.cls[kClsEmpty];
    out->wave_bitmap = (int64_t)(h.cls[kClsWaveBmpS] + h.cls[kClsWaveBmpL]);
    out->wave_hash = (int64_t)h.cls[kClsWaveHash];
    out->group = (int64_t)h.cls[kClsGroup];
    out->max_row_products = (int64_t)h.max_prod;
    out->max_row_nnz = (int64_t)h.max_nnz;
    return REAP_OK;
}

reap_status_t reap_spgemm_phase_times(reap_spgemm_t p, float* out, int n) {
    if (!p || !out || n <= 0) return REAP_ERR_INVALID_ARG;
    if (!p->profile || !p->events_ok) return REAP_ERR_STATE;
    REAP_HIP(hipStreamSynchronize(p->stream));
    fold_events(p);
    for (int i = 0; i < n && i < 8; ++i) {
        out[i] = 0.0f;
        if (i < kNumPhases && p->acc_calls[i] > 0) out[i] = (float)(p->acc_ms[i] / (double)p->acc_calls[i]);
    }
    if (n > 7) out[7] = (float)p->acc_calls[kPhNumAll];
    return REAP_OK;
}

reap_status_t reap_spgemm_phase_reset(reap_spgemm_t p) {
    if (!p) return REAP_ERR_INVALID_ARG;
    if (!p->profile || !p->events_ok) return REAP_ERR_STATE;
    REAP_HIP(hipStreamSynchronize(p->stream));
    for (int i = 0; i < kNumPhases; ++i) {
        p->phase_used[i] = false;
        p->acc_ms[i] = 0.0;
        p->acc_calls[i] = 0;
    }
    return REAP_OK;
}

}  // extern "C"
