// Host side of the C ABI declared in include/reap_spgemm.h: plan, workspace,
// argument checks and kernel launches on the plan's stream.  One engine serves
// the single-product calls and the batched calls: a batch of N products runs
// as one launch per kernel (a device table of per-product arguments and a
// block table map each workgroup to its product), and a single product is the
// batch of one with its arguments passed by value.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/reap_spgemm.h"
#include "kernels_long.h"
#include "kernels_numeric.h"
#include "kernels_scan.h"
#include "kernels_symbolic.h"
#include "kernels_transpose.h"
#include "kernels_wave.h"
#include "spgemm_common.h"

using namespace reap;

namespace {

enum Phase { kPhSymbolic = 0, kPhScan, kPhNumWave, kPhNumHash, kPhNumGroup, kPhNumAll, kNumPhases };

struct Workspace {
    void* base = nullptr;
    size_t bytes = 0;
};

// Host record of one product of the last symbolic call.
struct ProdState {
    int64_t m = 0, k = 0, n = 0, a_nnz = 0, b_nnz = 0;
    int32_t blocks = 0;   // workgroups of the wavefront kernels
    int32_t tiles = 0;    // scan tiles
    int64_t row_off = 0;  // first row in the per-row workspace arrays
    int32_t block_off = 0, tile_off = 0;
    int64_t c_nnz = 0, products = 0;
};

// Largest argument block of any instantiation (the device tables are sized by it).
constexpr size_t kArgBytes = std::max({sizeof(SymArgs<int64_t>), sizeof(NumArgs<double, int64_t, int64_t>),
                                       sizeof(NumArgs<float, int64_t, int64_t>)});
static_assert(sizeof(SymArgs<int32_t>) <= kArgBytes && sizeof(NumArgs<double, int32_t, int32_t>) <= kArgBytes,
              "argument table stride");

constexpr int kNumWavesS = kWaveKernelWaves;
constexpr int kNumWavesH = kWaveKernelWaves;

}  // namespace

// Workspace of reap_spgemm_symbolic_noalloc: one array per device, held for
// the life of the process.  Host code must not pass `scratch` itself to a
// kernel (in host code the name is a host-side stand-in); it uses the device
// address looked up by static_scratch() below.
static __device__ __align__(256) char scratch[REAP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up once per device (with
// that device current, as it is when a plan is created on it).
reap_status_t static_scratch(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return REAP_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return REAP_ERR_HIP;
        }
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return REAP_OK;
}

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
    bool use_graph = false;   // capture each pass into a HIP graph, replay while the shape repeats
    bool debug_sync = false;  // REAP_DEBUG_SYNC=1: synchronise and log after every kernel
    int long_wg_per_cu = 2;   // workgroups per CU walking the long-row list
    bool sym_narrow = true;   // narrow symbolic long-row workgroups when every product has <= 65536 columns
    int fail_alloc_at = 0;    // test hook: the n-th device allocation of the plan fails (0 = never)
    int scan_onepass = kScanOnePassTiles;  // most tiles per product for the one-launch scan
    int alloc_count = 0;      // device allocations attempted by the plan

    Workspace ws;      // counters, per-row arrays, tables
    Workspace gvals;   // long-row FP64 accumulators (FP32 output only)
    double* gvals_ptr = nullptr;   // accumulators in use: gvals.base, or inside the static scratch
    bool ws_static = false;        // the workspace pointers below point into the static scratch
    bool eager = false;            // this call runs its kernels directly (no tables, no graphs)
    bool buf_b = true;             // every B's values fit 2^31 bytes: buffer loads in the wavefront kernels
    Workspace tws;     // scratch of the device transpose
    int64_t cap_rows = -1, cap_prods = 0;
    int32_t cap_blocks = 0, cap_tiles = 0;
    uint64_t ws_generation = 0;

    Counters* ctr = nullptr;       // [nprod]
    unsigned int* n_long = nullptr;
    uint8_t* cls = nullptr;        // per row (all products)
    int32_t* rnnz = nullptr;
    int2* win = nullptr;
    int2* long_list = nullptr;
    int2* split_list = nullptr;    // long rows sorted into medium (from the start) and large (from the end)
    WGPart* parts = nullptr;       // per wavefront-kernel workgroup (all products)
    long long* tiles = nullptr;    // per scan tile (all products)
    int32_t* blk_start = nullptr;  // [nprod + 1]
    int32_t* tile_start = nullptr; // [nprod + 1]
    char* sym_args = nullptr;      // [nprod] SymArgs
    char* num_args = nullptr;      // [nprod] NumArgs
    ScanArgs* scan_args = nullptr; // [nprod]

    // pinned host memory: counters mirror (+ long-row count) and argument staging
    Counters* h_ctr = nullptr;
    Counters* h_ctr_dev = nullptr; // the same pinned memory as the device sees it
    TileStat* h_tiles = nullptr;   // per-tile statistics of the one-launch scan (pinned, device-mapped)
    TileStat* h_tiles_dev = nullptr;
    size_t h_tiles_cap = 0;        // tiles
    bool scan_onepass_used = false;
    size_t h_ctr_cap = 0;          // products
    char* h_stage = nullptr;       // symbolic tables
    char* h_stage_num = nullptr;   // numeric table
    size_t stage_cap = 0;          // products
    hipEvent_t ev_num_upload = nullptr;
    bool num_upload_recorded = false;

    // state of the last symbolic call
    bool have_symbolic = false;
    bool numeric_ran = false;          // a numeric call was enqueued since the last symbolic call
    int nprod = 0;
    std::vector<ProdState> prods;
    reap_index_t in_idx = REAP_I32;
    int64_t total_rows = 0;
    int32_t total_blocks = 0, total_tiles = 0;
    int32_t max_prod_tiles = 0;     // most scan tiles of one product in the batch
    unsigned int long_rows = 0;
    unsigned int mid_rows = 0, big_rows = 0;   // the split of the long rows (numeric shapes)
    int mid_grid = 1, big_grid = 1;
    int long_grid = 1;             // the wider of the two grids (FP64 accumulator slots)
    int64_t gvals_stride = 0;
    Counters agg{};                // summed / maxed over the products (bin statistics)

    // captured passes
    hipGraphExec_t g_sym = nullptr, g_num = nullptr;
    std::vector<uint64_t> g_sym_key, g_num_key;

    hipEvent_t ev[2 * kNumPhases] = {};
    bool events_ok = false;
    bool capturing = false;
    bool phase_used[kNumPhases] = {};   // recorded and not yet folded into acc_ms
    double acc_ms[kNumPhases] = {};     // accumulated device time per phase
    long long acc_calls[kNumPhases] = {};
};

namespace {

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

reap_status_t check_csr(const reap_csr_t* M) {
    if (!M) return REAP_ERR_INVALID_ARG;
    if (M->rows < 0 || M->cols < 0 || M->nnz < 0) return REAP_ERR_INVALID_ARG;
    if (M->cols > INT32_MAX) return REAP_ERR_INVALID_ARG;  // int32 column indices
    if (M->row_ptr_type != REAP_I32 && M->row_ptr_type != REAP_I64) return REAP_ERR_INVALID_ARG;
    if (M->row_ptr_type == REAP_I32 && M->nnz > INT32_MAX) return REAP_ERR_INVALID_ARG;
    if (!M->row_ptr) return REAP_ERR_INVALID_ARG;
    if (M->nnz > 0 && (!M->col_idx || !M->values)) return REAP_ERR_INVALID_ARG;
    return REAP_OK;
}

void release_graphs(reap_spgemm_s* p) {
    if (p->g_sym) (void)hipGraphExecDestroy(p->g_sym);
    if (p->g_num) (void)hipGraphExecDestroy(p->g_num);
    p->g_sym = p->g_num = nullptr;
    p->g_sym_key.clear();
    p->g_num_key.clear();
}

// Device allocation of the plan's own memory; the test hook makes the n-th
// attempt fail as an out-of-memory condition would.
hipError_t dev_malloc(reap_spgemm_s* p, void** ptr, size_t bytes) {
    ++p->alloc_count;
    if (p->fail_alloc_at > 0 && p->alloc_count == p->fail_alloc_at) {
        *ptr = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(ptr, bytes);
}

// Offsets of the workspace slices for R rows, Bk wavefront-kernel
// workgroups, Tl scan tiles and Q products (256-byte aligned).
struct WsLayout {
    size_t o_ctr, o_nlong, o_cls, o_rnnz, o_win, o_long, o_split, o_parts, o_tiles, o_bs, o_ts, o_sa, o_na, o_sc,
        total;
};

WsLayout ws_layout(int64_t R, int32_t Bk, int32_t Tl, int64_t Q) {
    WsLayout L{};
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    L.o_ctr = carve((size_t)Q * sizeof(Counters));
    L.o_nlong = carve(kLongCtrWords * sizeof(unsigned int));  // long-row counts and queue counters
    L.o_cls = carve((size_t)R);
    L.o_rnnz = carve((size_t)R * 4);
    L.o_win = carve((size_t)R * 8);
    L.o_long = carve((size_t)R * 8);
    L.o_split = carve((size_t)R * 8);
    L.o_parts = carve((size_t)Bk * sizeof(WGPart));
    L.o_tiles = carve((size_t)Tl * 8);
    L.o_bs = carve((size_t)(Q + 1) * 4);
    L.o_ts = carve((size_t)(Q + 1) * 4);
    L.o_sa = carve((size_t)Q * kArgBytes);
    L.o_na = carve((size_t)Q * kArgBytes);
    L.o_sc = carve((size_t)Q * sizeof(ScanArgs));
    L.total = off;
    return L;
}

// Pinned, device-mapped records of `ntiles` scan tiles for the one-launch scan.
reap_status_t ensure_host_tiles(reap_spgemm_s* p, size_t ntiles) {
    if (ntiles <= p->h_tiles_cap && p->h_tiles) return REAP_OK;
    (void)hipStreamSynchronize(p->stream);
    release_graphs(p);  // captured scans write the old records
    if (p->h_tiles) (void)hipHostFree(p->h_tiles);
    p->h_tiles = p->h_tiles_dev = nullptr;
    p->h_tiles_cap = 0;
    const size_t cap = std::max<size_t>(ntiles, kScanOnePassTiles);
    if (hipHostMalloc(reinterpret_cast<void**>(&p->h_tiles), cap * sizeof(TileStat),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer(reinterpret_cast<void**>(&p->h_tiles_dev), p->h_tiles, 0) != hipSuccess) {
        (void)hipGetLastError();
        if (p->h_tiles) (void)hipHostFree(p->h_tiles);
        p->h_tiles = p->h_tiles_dev = nullptr;
        return REAP_ERR_OUT_OF_MEMORY;
    }
    p->h_tiles_cap = cap;
    return REAP_OK;
}

// Pinned staging and counter mirror for `nprod` products.
reap_status_t ensure_host(reap_spgemm_s* p, int nprod) {
    if ((size_t)nprod <= p->stage_cap && p->h_ctr) return REAP_OK;
    if (p->ev_num_upload && p->num_upload_recorded) (void)hipEventSynchronize(p->ev_num_upload);
    (void)hipStreamSynchronize(p->stream);
    release_graphs(p);  // captured copies read the old staging buffers
    if (p->h_ctr) (void)hipHostFree(p->h_ctr);
    if (p->h_stage) (void)hipHostFree(p->h_stage);
    if (p->h_stage_num) (void)hipHostFree(p->h_stage_num);
    p->h_ctr = nullptr;
    p->h_ctr_dev = nullptr;
    p->h_stage = p->h_stage_num = nullptr;
    p->stage_cap = 0;
    const size_t cap = std::max<size_t>((size_t)nprod, 1);
    const size_t ctr_bytes = (cap + 1) * sizeof(Counters);  // the last slot holds the long-row count
    const size_t stage_bytes = cap * (kArgBytes + sizeof(ScanArgs)) + 2 * (cap + 1) * sizeof(int32_t) + 256;
    // the counter mirror is written by the scan kernel itself: coherent, device-mapped
    if (hipHostMalloc(reinterpret_cast<void**>(&p->h_ctr), ctr_bytes, hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer(reinterpret_cast<void**>(&p->h_ctr_dev), p->h_ctr, 0) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&p->h_stage), stage_bytes, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&p->h_stage_num), cap * kArgBytes + 256, hipHostMallocDefault) !=
            hipSuccess) {
        (void)hipGetLastError();
        return REAP_ERR_OUT_OF_MEMORY;
    }
    std::memset(p->h_ctr, 0, ctr_bytes);
    p->stage_cap = cap;
    p->h_ctr_cap = cap;
    return REAP_OK;
}

// Points the plan's workspace arrays into `b` laid out as L.
void bind_workspace(reap_spgemm_s* p, char* b, const WsLayout& L) {
    p->ctr = reinterpret_cast<Counters*>(b + L.o_ctr);
    p->n_long = reinterpret_cast<unsigned int*>(b + L.o_nlong);
    p->cls = reinterpret_cast<uint8_t*>(b + L.o_cls);
    p->rnnz = reinterpret_cast<int32_t*>(b + L.o_rnnz);
    p->win = reinterpret_cast<int2*>(b + L.o_win);
    p->long_list = reinterpret_cast<int2*>(b + L.o_long);
    p->split_list = reinterpret_cast<int2*>(b + L.o_split);
    p->parts = reinterpret_cast<WGPart*>(b + L.o_parts);
    p->tiles = reinterpret_cast<long long*>(b + L.o_tiles);
    p->blk_start = reinterpret_cast<int32_t*>(b + L.o_bs);
    p->tile_start = reinterpret_cast<int32_t*>(b + L.o_ts);
    p->sym_args = b + L.o_sa;
    p->num_args = b + L.o_na;
    p->scan_args = reinterpret_cast<ScanArgs*>(b + L.o_sc);
}

// Device workspace for the given totals (grows, never shrinks).
reap_status_t ensure_workspace(reap_spgemm_s* p, int64_t rows, int32_t blocks, int32_t tiles, int nprod) {
    if (p->ws.base && rows <= p->cap_rows && blocks <= p->cap_blocks && tiles <= p->cap_tiles &&
        (int64_t)nprod <= p->cap_prods) {
        if (p->ws_static) {  // the previous call ran in the static scratch: back to the plan's own
            bind_workspace(p, static_cast<char*>(p->ws.base),
                           ws_layout(p->cap_rows, p->cap_blocks, p->cap_tiles, p->cap_prods));
            p->ws_static = false;
            ++p->ws_generation;
        }
        return REAP_OK;
    }
    const int64_t R = std::max<int64_t>({rows, p->cap_rows, 1});
    const int32_t Bk = std::max({blocks, p->cap_blocks, 1});
    const int32_t Tl = std::max({tiles, p->cap_tiles, 1});
    const int64_t Q = std::max<int64_t>({(int64_t)nprod, p->cap_prods, 1});
    const WsLayout L = ws_layout(R, Bk, Tl, Q);
    (void)hipStreamSynchronize(p->stream);
    release_graphs(p);
    if (p->ws.base) {
        (void)hipFree(p->ws.base);
        p->ws.base = nullptr;
        p->ws.bytes = 0;
    }
    void* base = nullptr;
    if (dev_malloc(p, &base, L.total) != hipSuccess) {
        (void)hipGetLastError();
        p->cap_rows = -1;
        p->cap_blocks = p->cap_tiles = 0;
        p->cap_prods = 0;
        return REAP_ERR_OUT_OF_MEMORY;
    }
    p->ws.base = base;
    p->ws.bytes = L.total;
    bind_workspace(p, static_cast<char*>(base), L);
    p->ws_static = false;
    p->cap_rows = R;
    p->cap_blocks = Bk;
    p->cap_tiles = Tl;
    p->cap_prods = Q;
    ++p->ws_generation;
    return REAP_OK;
}

// Workspace of one product inside the device's static scratch (no
// allocation); *used receives the bytes taken.
reap_status_t bind_static(reap_spgemm_s* p, int64_t rows, int32_t blocks, int32_t tiles, size_t* used) {
    const WsLayout L = ws_layout(std::max<int64_t>(rows, 1), std::max(blocks, 1), std::max(tiles, 1), 1);
    if (L.total > (size_t)REAP_NOALLOC_SCRATCH_BYTES) return REAP_ERR_TOO_LARGE;
    void* base = nullptr;
    const reap_status_t st = static_scratch(p->device, &base);
    if (st != REAP_OK) return st;
    bind_workspace(p, static_cast<char*>(base), L);
    p->ws_static = true;
    ++p->ws_generation;
    *used = L.total;
    return REAP_OK;
}

// With REAP_DEBUG_SYNC=1 in the environment every kernel launch is followed by
// a stream synchronisation and a line on stderr, so a failing kernel is named.
void debug_step(reap_spgemm_s* p, const char* kernel) {
    if (!p->debug_sync || p->capturing) return;
    fprintf(stderr, "[reap] %s launched\n", kernel);
    fflush(stderr);
    const hipError_t e = hipStreamSynchronize(p->stream);
    fprintf(stderr, "[reap] %s done (%s)\n", kernel, hipGetErrorString(e));
    fflush(stderr);
}

void ev_record(reap_spgemm_s* p, int phase, bool end) {
    if (p->profile && p->events_ok && !p->capturing) {
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

BatchMap batch_map(const reap_spgemm_s* p) {
    BatchMap bm;
    bm.blk_start = p->blk_start;
    bm.nprod = p->nprod;
    bm.long_list = p->long_list;
    bm.n_long = p->n_long + kLongCtrCount;
    bm.queue = p->n_long + kLongCtrQueue;
    bm.split_list = p->split_list;
    bm.split_cap = (unsigned int)std::max<int64_t>(p->total_rows, 1);
    bm.n_split = p->n_long + kLongCtrSplit;
    return bm;
}

// Argument tables go through device memory for batches and captured passes;
// a single eager product passes its arguments by value.
bool use_tables(const reap_spgemm_s* p) { return p->nprod > 1 || (p->use_graph && !p->eager); }

// Runs `body` (which enqueues work on the plan's stream) eagerly, or captures
// it once per key into a graph and replays that graph.
template <typename Body>
reap_status_t run_pass(reap_spgemm_s* p, hipGraphExec_t& exec, std::vector<uint64_t>& key_store,
                       const std::vector<uint64_t>& key, Body&& body) {
    if (!p->use_graph) return body();
    if (!(exec && key_store == key)) {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
        key_store.clear();
        REAP_HIP(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
        p->capturing = true;
        const reap_status_t st = body();
        p->capturing = false;
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(p->stream, &graph);
        if (st != REAP_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return REAP_ERR_HIP;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            exec = nullptr;
            return REAP_ERR_HIP;
        }
        key_store = key;
    }
    REAP_HIP(hipGraphLaunch(exec, p->stream));
    return REAP_OK;
}

// ---------------------------------------------------------------------------
// C's row pointer from the tile sums: one launch when every product has at
// most p->scan_onepass tiles (and the tile records fit the host mirror), else
// the per-product spine and the row kernel.
template <typename IdxC>
reap_status_t launch_row_ptr_scan(reap_spgemm_s* p, const ScanArgs& s0, const ScanArgs* S, ScanMap sm) {
    if (p->scan_onepass_used) {
        hipLaunchKernelGGL(k_scan_onepass<IdxC>, dim3(p->total_tiles + 1), dim3(kScanThreads), 0, p->stream, s0, S,
                           sm, p->total_tiles);
        REAP_LAUNCH_CHECK();
        return REAP_OK;
    }
    hipLaunchKernelGGL(k_scan_spine<IdxC>, dim3(p->nprod), dim3(1024), 0, p->stream, s0, S);
    REAP_LAUNCH_CHECK();
    if (p->total_tiles > 0) {
        hipLaunchKernelGGL(k_scan_apply<IdxC>, dim3(p->total_tiles), dim3(kScanThreads), 0, p->stream, s0, S, sm);
        REAP_LAUNCH_CHECK();
    }
    return REAP_OK;
}

// Symbolic pass of the current batch (tables already in the staging buffer).

template <typename IdxT>
reap_status_t launch_symbolic(reap_spgemm_s* p, const SymArgs<IdxT>& a0, const ScanArgs& s0) {
    const bool tab = use_tables(p);
    const SymArgs<IdxT>* P = tab ? reinterpret_cast<const SymArgs<IdxT>*>(p->sym_args) : nullptr;
    const ScanArgs* S = tab ? p->scan_args : nullptr;
    const BatchMap bm = batch_map(p);
    ScanMap sm;
    sm.tile_start = p->tile_start;
    sm.nprod = p->nprod;

    if (tab) {
        char* h = p->h_stage;
        // layout in staging: [sym args][scan args][blk_start][tile_start]; copied piecewise
        REAP_HIP(hipMemcpyAsync(p->sym_args, h, (size_t)p->nprod * kArgBytes, hipMemcpyHostToDevice, p->stream));
        h += (size_t)p->nprod * kArgBytes;
        REAP_HIP(hipMemcpyAsync(p->scan_args, h, (size_t)p->nprod * sizeof(ScanArgs), hipMemcpyHostToDevice,
                                p->stream));
        h += (size_t)p->nprod * sizeof(ScanArgs);
        REAP_HIP(hipMemcpyAsync(p->blk_start, h, (size_t)(p->nprod + 1) * 4, hipMemcpyHostToDevice, p->stream));
        h += (size_t)(p->nprod + 1) * 4;
        REAP_HIP(hipMemcpyAsync(p->tile_start, h, (size_t)(p->nprod + 1) * 4, hipMemcpyHostToDevice, p->stream));
    }
    const int64_t zw = std::max<int64_t>((int64_t)p->nprod * (int64_t)(sizeof(Counters) / 4), p->total_tiles);
    const int zb = (int)std::min<int64_t>(1024, (zw + 255) / 256);
    hipLaunchKernelGGL(k_zero_counters, dim3(std::max(zb, 1)), dim3(256), 0, p->stream, p->ctr, p->nprod, p->n_long,
                       p->tiles, p->total_tiles);
    REAP_LAUNCH_CHECK();

    ev_record(p, kPhSymbolic, false);
    if (p->total_blocks > 0) {
        const dim3 grid(p->total_blocks), block(kWaveKernelWaves * kWave);
        if (tab && p->buf_b)
            hipLaunchKernelGGL((k_sym_wave<IdxT, true, true>), grid, block, 0, p->stream, a0, P, bm);
        else if (tab)
            hipLaunchKernelGGL((k_sym_wave<IdxT, true, false>), grid, block, 0, p->stream, a0, P, bm);
        else if (p->buf_b)
            hipLaunchKernelGGL((k_sym_wave<IdxT, false, true>), grid, block, 0, p->stream, a0, P, bm);
        else
            hipLaunchKernelGGL((k_sym_wave<IdxT, false, false>), grid, block, 0, p->stream, a0, P, bm);
        REAP_LAUNCH_CHECK();
        debug_step(p, "k_sym_wave");
        // the long-row count is known on the device only: a fixed grid takes rows
        // from the list; narrow workgroups (twice as many) when every product has
        // at most LongSymNarrow::SEGW * 32 columns
        bool narrow = p->sym_narrow;
        for (int q = 0; q < p->nprod && narrow; ++q) narrow = p->prods[(size_t)q].n <= LongSymNarrow::SEGW * 32;
        const int per_cu = p->long_wg_per_cu * (narrow ? 2 : 1);
        const int lgrid = (int)std::max<int64_t>(1, std::min<int64_t>(p->total_rows, (int64_t)p->num_cus * per_cu));
        if (narrow)
            hipLaunchKernelGGL((k_long_sym<IdxT, LongSymNarrow>), dim3(lgrid), dim3(LongSymNarrow::NT), 0, p->stream,
                               a0, P, bm);
        else
            hipLaunchKernelGGL((k_long_sym<IdxT, LongSymWide>), dim3(lgrid), dim3(LongSymWide::NT), 0, p->stream, a0,
                               P, bm);
        REAP_LAUNCH_CHECK();
        debug_step(p, "k_long_sym");
    }
    ev_record(p, kPhSymbolic, true);
    ev_record(p, kPhScan, false);
    // the symbolic kernels have summed every scan tile
    reap_status_t st = p->cidx == REAP_I32 ? launch_row_ptr_scan<int32_t>(p, s0, S, sm)
                                           : launch_row_ptr_scan<int64_t>(p, s0, S, sm);
    if (st != REAP_OK) return st;
    debug_step(p, "k_scan");
    ev_record(p, kPhScan, true);
    // the spine kernel has written every product's counters and the long-row
    // count into the pinned host mirror
    return REAP_OK;
}

template <typename IdxT>
reap_status_t run_validate(reap_spgemm_s* p, const reap_csr_t* M, Counters* ctr, unsigned bit) {
    const int64_t n = M->rows + 1;
    const int blocks = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_validate<IdxT>, dim3(blocks), dim3(256), 0, p->stream, static_cast<const IdxT*>(M->row_ptr),
                       M->col_idx, M->rows, M->cols, M->nnz, ctr, bit);
    REAP_LAUNCH_CHECK();
    return REAP_OK;
}

template <typename IdxT>
reap_status_t symbolic_typed(reap_spgemm_s* p, const reap_csr_t* A, const reap_csr_t* B, void* const* c_row_ptr) {
    const int nprod = p->nprod;
    // argument tables in the staging buffer
    char* h = p->h_stage;
    SymArgs<IdxT> a0{};
    ScanArgs s0{};
    for (int q = 0; q < nprod; ++q) {
        const ProdState& ps = p->prods[q];
        SymArgs<IdxT> a{};
        a.m = ps.m;
        a.n = ps.n;
        a.k = ps.k;
        a.a_rp = to_gptr(static_cast<const IdxT*>(A[q].row_ptr));
        a.a_col = to_gptr(A[q].col_idx);
        a.b_rp = to_gptr(static_cast<const IdxT*>(B[q].row_ptr));
        a.b_col = to_gptr(B[q].col_idx);
        a.cls = to_gptr(p->cls + ps.row_off);
        a.rnnz = to_gptr(p->rnnz + ps.row_off);
        a.win = to_gptr(p->win + ps.row_off);
        a.ctr = to_gptr(p->ctr + q);
        a.parts = to_gptr(p->parts + ps.block_off);
        a.tiles = to_gptr(reinterpret_cast<unsigned long long*>(p->tiles + ps.tile_off));
        a.th = p->th;
        ScanArgs s{};
        s.rnnz = p->rnnz + ps.row_off;
        s.m = ps.m;
        s.tiles = p->tiles + ps.tile_off;
        s.ntiles = ps.tiles;
        s.nparts = ps.blocks;
        s.parts = p->parts + ps.block_off;
        s.ctr = p->ctr + q;
        s.c_rp = c_row_ptr[q];
        s.h_ctr = p->h_ctr_dev + q;
        s.n_long = p->n_long;
        s.h_nlong = reinterpret_cast<unsigned int*>(p->h_ctr_dev + p->h_ctr_cap);
        s.h_tiles = p->scan_onepass_used ? p->h_tiles_dev + ps.tile_off : nullptr;
        // the kernels index the table as an array of this instantiation's type
        std::memcpy(h + (size_t)q * sizeof(a), &a, sizeof(a));
        std::memcpy(h + (size_t)nprod * kArgBytes + (size_t)q * sizeof(ScanArgs), &s, sizeof(s));
        if (q == 0) {
            a0 = a;
            s0 = s;
        }
    }
    int32_t* bs = reinterpret_cast<int32_t*>(h + (size_t)nprod * (kArgBytes + sizeof(ScanArgs)));
    int32_t* ts = bs + nprod + 1;
    for (int q = 0; q < nprod; ++q) {
        bs[q] = p->prods[q].block_off;
        ts[q] = p->prods[q].tile_off;
    }
    bs[nprod] = p->total_blocks;
    ts[nprod] = p->total_tiles;

    if (p->validate) {
        const int zb = (int)std::min<int64_t>(1024, ((int64_t)nprod * (int64_t)(sizeof(Counters) / 4) + 255) / 256);
        hipLaunchKernelGGL(k_zero_counters, dim3(std::max(zb, 1)), dim3(256), 0, p->stream, p->ctr, nprod, p->n_long,
                           p->tiles, 0);
        REAP_LAUNCH_CHECK();
        reap_status_t st;
        for (int q = 0; q < nprod; ++q) {
            if ((st = run_validate<IdxT>(p, &A[q], p->ctr + q, 1u)) != REAP_OK) return st;
            if ((st = run_validate<IdxT>(p, &B[q], p->ctr + q, 2u)) != REAP_OK) return st;
        }
        REAP_HIP(hipMemcpyAsync(p->h_ctr, p->ctr, (size_t)nprod * sizeof(Counters), hipMemcpyDeviceToHost, p->stream));
        REAP_HIP(hipStreamSynchronize(p->stream));
        for (int q = 0; q < nprod; ++q)
            if (p->h_ctr[q].bad_csr) return REAP_ERR_BAD_CSR;
    }

    if (!p->use_graph || p->eager) return launch_symbolic<IdxT>(p, a0, s0);
    std::vector<uint64_t> key = {p->ws_generation, (uint64_t)nprod, (uint64_t)p->total_blocks,
                                 (uint64_t)p->total_tiles, (uint64_t)p->total_rows, (uint64_t)p->cidx,
                                 (uint64_t)sizeof(IdxT), (uint64_t)p->buf_b,
                                 (uint64_t)p->scan_onepass_used};
    return run_pass(p, p->g_sym, p->g_sym_key, key, [&]() { return launch_symbolic<IdxT>(p, a0, s0); });
}

// Shape checks of a batch and its totals (rows, wavefront-kernel
// workgroups, scan tiles, widest B).
struct BatchTotals {
    int64_t rows = 0, blocks = 0, tiles = 0, max_n = 0;
};

reap_status_t batch_totals(int64_t count, const reap_csr_t* A, const reap_csr_t* B, BatchTotals* t) {
    if (count < 1 || count > INT32_MAX / 2 || !A || !B) return REAP_ERR_INVALID_ARG;
    reap_status_t st;
    const reap_index_t in_idx = A[0].row_ptr_type;
    for (int64_t q = 0; q < count; ++q) {
        if ((st = check_csr(&A[q])) != REAP_OK) return st;
        if ((st = check_csr(&B[q])) != REAP_OK) return st;
        if (A[q].cols != B[q].rows) return REAP_ERR_INVALID_ARG;
        if (A[q].row_ptr_type != in_idx || B[q].row_ptr_type != in_idx) return REAP_ERR_INVALID_ARG;
        if (A[q].rows > INT32_MAX - 1) return REAP_ERR_INVALID_ARG;  // row ids are stored as int32
        t->rows += A[q].rows;
        t->blocks += (A[q].rows + kRowsPerBlock - 1) / kRowsPerBlock;
        t->tiles += (A[q].rows + kScanTile - 1) / kScanTile;
        t->max_n = std::max(t->max_n, B[q].cols);
    }
    if (t->rows > INT32_MAX || t->blocks > INT32_MAX || t->tiles > INT32_MAX) return REAP_ERR_INVALID_ARG;
    return REAP_OK;
}

// Device bytes of the FP32 long-row accumulators at their largest: one
// segment of the widest row per numeric long-row workgroup.
size_t gvals_bound(const reap_spgemm_s* p, const BatchTotals& t) {
    if (p->dtype != REAP_F32) return 0;
    const int64_t stride = std::max<int64_t>(1, std::min<int64_t>(t.max_n, (int64_t)p->th.group_lds_span));
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(t.rows, (int64_t)p->num_cus));
    return (size_t)stride * (size_t)grid * sizeof(double);
}

// The symbolic pass of `count` products.  With `noalloc` (one product) the
// workspace is bound into the device's static scratch instead of the plan's
// own allocation, the kernels are launched directly, and nothing is
// allocated on the device or the host heap.
reap_status_t symbolic_batch(reap_spgemm_s* p, int64_t count, const reap_csr_t* A, const reap_csr_t* B,
                             void* const* c_row_ptr, int64_t* c_nnz, int64_t* n_products, size_t* workspace_bytes,
                             bool noalloc = false) {
    if (!p || count < 1 || count > INT32_MAX / 2 || !A || !B || !c_row_ptr || !c_nnz) return REAP_ERR_INVALID_ARG;
    if (noalloc && count != 1) return REAP_ERR_INVALID_ARG;
    reap_status_t st;
    const reap_index_t in_idx = A[0].row_ptr_type;
    BatchTotals bt;
    if ((st = batch_totals(count, A, B, &bt)) != REAP_OK) return st;
    for (int64_t q = 0; q < count; ++q)
        if (!c_row_ptr[q]) return REAP_ERR_INVALID_ARG;
    const int64_t rows = bt.rows, blocks = bt.blocks, tiles = bt.tiles;
    p->have_symbolic = false;
    if (p->ev_num_upload && p->num_upload_recorded) (void)hipEventSynchronize(p->ev_num_upload);
    size_t static_used = 0;
    if (noalloc) {
        // the pinned host mirror made at create holds one product's counters
        if ((st = bind_static(p, rows, (int32_t)blocks, (int32_t)tiles, &static_used)) != REAP_OK) return st;
    } else {
        if ((st = ensure_host(p, (int)count)) != REAP_OK) return st;
        if ((st = ensure_workspace(p, rows, (int32_t)blocks, (int32_t)tiles, (int)count)) != REAP_OK) return st;
    }
    p->eager = noalloc;

    p->nprod = (int)count;
    p->prods.assign((size_t)count, ProdState{});
    p->in_idx = in_idx;
    int64_t ro = 0;
    int32_t bo = 0, to = 0, mt = 0;
    for (int64_t q = 0; q < count; ++q) {
        ProdState& ps = p->prods[(size_t)q];
        ps.m = A[q].rows;
        ps.k = A[q].cols;
        ps.n = B[q].cols;
        ps.a_nnz = A[q].nnz;
        ps.b_nnz = B[q].nnz;
        ps.blocks = (int32_t)((ps.m + kRowsPerBlock - 1) / kRowsPerBlock);
        ps.tiles = (int32_t)((ps.m + kScanTile - 1) / kScanTile);
        ps.row_off = ro;
        ps.block_off = bo;
        ps.tile_off = to;
        ro += ps.m;
        bo += ps.blocks;
        to += ps.tiles;
        mt = std::max(mt, ps.tiles);
    }
    p->max_prod_tiles = mt;
    p->scan_onepass_used = false;
    if (mt <= p->scan_onepass) {
        // the allocation-free call uses the records made at create, if they suffice
        if (!noalloc && (st = ensure_host_tiles(p, (size_t)to)) != REAP_OK) return st;
        p->scan_onepass_used = (size_t)to <= p->h_tiles_cap;
    }
    p->total_rows = ro;
    p->total_blocks = bo;
    p->total_tiles = to;
    // buffer loads take 32-bit byte offsets: B's values must stay below 2^31 bytes
    p->buf_b = true;
    for (int64_t q = 0; q < count; ++q) p->buf_b &= B[q].nnz < ((int64_t)1 << 28);

    st = (in_idx == REAP_I32) ? symbolic_typed<int32_t>(p, A, B, c_row_ptr)
                              : symbolic_typed<int64_t>(p, A, B, c_row_ptr);
    if (st != REAP_OK) return st;
    REAP_HIP(hipStreamSynchronize(p->stream));
    fold_events(p);  // this call's symbolic phases and the previous numeric call's phases

    const unsigned int* hl =
        reinterpret_cast<const unsigned int*>(reinterpret_cast<const char*>(p->h_ctr) + p->h_ctr_cap * sizeof(Counters));
    const unsigned int nl = hl[0];
    p->long_rows = nl;
    p->mid_rows = hl[1];
    p->big_rows = hl[2];
    p->agg = Counters{};
    unsigned int max_group_nnz = 0;
    bool overflow = false;
    for (int q = 0; q < p->nprod; ++q) {
        Counters h = p->h_ctr[q];
        ProdState& ps = p->prods[(size_t)q];
        if (p->scan_onepass_used) {
            // the one-launch scan left the wavefront rows' statistics per tile
            for (int t = 0; t < ps.tiles; ++t) {
                const TileStat& ts = p->h_tiles[ps.tile_off + t];
                h.nnz += ts.nnz;
                h.products += ts.products;
                for (int c = 0; c < kNumClasses; ++c) h.cls[c] += ts.cls[c];
                h.max_prod = std::max(h.max_prod, ts.max_prod);
                h.max_nnz = std::max(h.max_nnz, ts.max_nnz);
            }
        }
        ps.c_nnz = (int64_t)h.nnz;
        ps.products = (int64_t)h.products;
        c_nnz[q] = ps.c_nnz;
        if (n_products) n_products[q] = ps.products;
        if (p->cidx == REAP_I32 && ps.c_nnz > INT32_MAX) overflow = true;
        p->agg.products += h.products;
        p->agg.nnz += h.nnz;
        for (int c = 0; c < kNumClasses; ++c) p->agg.cls[c] += h.cls[c];
        p->agg.max_prod = std::max(p->agg.max_prod, h.max_prod);
        p->agg.max_nnz = std::max(p->agg.max_nnz, h.max_nnz);
        max_group_nnz = std::max(max_group_nnz, h.max_group_nnz);
    }

    // long rows: one numeric workgroup per CU (its LDS takes most of the CU's).
    // FP32 output needs FP64 accumulators in device memory (one segment of the
    // widest row per workgroup) only where a long row reads a B row stored
    // out of column order (the rank-chunk walks need sorted rows)
    bool unsorted_long = false;
    for (int q = 0; q < p->nprod; ++q) unsorted_long |= (p->h_ctr[q].bad_csr & kUnsortedB) != 0u;
    p->mid_grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)p->mid_rows, (int64_t)p->num_cus * kMidPerCu));
    p->big_grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)p->big_rows, (int64_t)p->num_cus));
    p->long_grid = std::max(p->mid_grid, p->big_grid);
    p->gvals_stride = 0;
    p->gvals_ptr = nullptr;
    if (p->dtype == REAP_F32 && nl > 0 && unsorted_long) {
        const int64_t stride =
            std::max<int64_t>(1, std::min<int64_t>((int64_t)max_group_nnz, (int64_t)p->th.group_lds_span));
        const size_t need = (size_t)stride * (size_t)p->long_grid * sizeof(double);
        if (noalloc) {
            const size_t off = align_up(static_used, 256);
            if (off + need > (size_t)REAP_NOALLOC_SCRATCH_BYTES) return REAP_ERR_TOO_LARGE;
            void* base = nullptr;
            if ((st = static_scratch(p->device, &base)) != REAP_OK) return st;
            p->gvals_ptr = reinterpret_cast<double*>(static_cast<char*>(base) + off);
        } else {
            if (need > p->gvals.bytes) {
                (void)hipStreamSynchronize(p->stream);
                if (p->g_num) {
                    (void)hipGraphExecDestroy(p->g_num);
                    p->g_num = nullptr;
                    p->g_num_key.clear();
                }
                if (p->gvals.base) (void)hipFree(p->gvals.base);
                p->gvals.base = nullptr;
                p->gvals.bytes = 0;
                if (dev_malloc(p, &p->gvals.base, need) != hipSuccess) {
                    (void)hipGetLastError();
                    return REAP_ERR_OUT_OF_MEMORY;
                }
                p->gvals.bytes = need;
            }
            p->gvals_ptr = static_cast<double*>(p->gvals.base);
        }
        p->gvals_stride = stride;
    }
    if (workspace_bytes) *workspace_bytes = p->ws.bytes + p->gvals.bytes;
    if (overflow) return REAP_ERR_INDEX_OVERFLOW;
    p->have_symbolic = true;
    p->numeric_ran = false;
    return REAP_OK;
}

// ---------------------------------------------------------------------------
// Numeric pass.

// The hash-class numeric kernel with an HS-slot table.
template <typename T, typename IdxT, typename IdxC, int HS>
void launch_num_hash(reap_spgemm_s* p, bool tab, dim3 grid, dim3 block, const NumArgs<T, IdxT, IdxC>& a0,
                     const NumArgs<T, IdxT, IdxC>* P, const BatchMap& bm, uint8_t want) {
    if (tab && p->buf_b)
        hipLaunchKernelGGL((k_num_wave_hash<T, IdxT, IdxC, kNumWavesH, true, true, HS>), grid, block, 0, p->stream, a0,
                           P, bm, want);
    else if (tab)
        hipLaunchKernelGGL((k_num_wave_hash<T, IdxT, IdxC, kNumWavesH, true, false, HS>), grid, block, 0, p->stream,
                           a0, P, bm, want);
    else if (p->buf_b)
        hipLaunchKernelGGL((k_num_wave_hash<T, IdxT, IdxC, kNumWavesH, false, true, HS>), grid, block, 0, p->stream,
                           a0, P, bm, want);
    else
        hipLaunchKernelGGL((k_num_wave_hash<T, IdxT, IdxC, kNumWavesH, false, false, HS>), grid, block, 0, p->stream,
                           a0, P, bm, want);
}

template <typename T, typename IdxT, typename IdxC>
reap_status_t launch_numeric(reap_spgemm_s* p, const NumArgs<T, IdxT, IdxC>& a0) {
    const bool tab = use_tables(p);
    const NumArgs<T, IdxT, IdxC>* P = tab ? reinterpret_cast<const NumArgs<T, IdxT, IdxC>*>(p->num_args) : nullptr;
    const BatchMap bm = batch_map(p);
    if (tab) {
        REAP_HIP(hipMemcpyAsync(p->num_args, p->h_stage_num, (size_t)p->nprod * kArgBytes, hipMemcpyHostToDevice,
                                p->stream));
        if (!p->capturing) {
            REAP_HIP(hipEventRecord(p->ev_num_upload, p->stream));
            p->num_upload_recorded = true;
        }
    }
    ev_record(p, kPhNumAll, false);
    ev_record(p, kPhNumWave, false);
    if (p->agg.cls[kClsWaveBmpS] > 0) {
        const dim3 grid(p->total_blocks), block(kNumWavesS * kWave);
        const uint8_t want = kClsWaveBmpS;
        if (tab && p->buf_b)
            hipLaunchKernelGGL((k_num_wave_bmp<T, IdxT, IdxC, kWaveSmallNnz, kNumWavesS, true, true>), grid, block,
                               0, p->stream, a0, P, bm, want);
        else if (tab)
            hipLaunchKernelGGL((k_num_wave_bmp<T, IdxT, IdxC, kWaveSmallNnz, kNumWavesS, true, false>), grid, block,
                               0, p->stream, a0, P, bm, want);
        else if (p->buf_b)
            hipLaunchKernelGGL((k_num_wave_bmp<T, IdxT, IdxC, kWaveSmallNnz, kNumWavesS, false, true>), grid, block,
                               0, p->stream, a0, P, bm, want);
        else
            hipLaunchKernelGGL((k_num_wave_bmp<T, IdxT, IdxC, kWaveSmallNnz, kNumWavesS, false, false>), grid, block,
                               0, p->stream, a0, P, bm, want);
        REAP_LAUNCH_CHECK();
        debug_step(p, "k_num_wave_bmp");
    }
    ev_record(p, kPhNumWave, true);
    ev_record(p, kPhNumHash, false);
    if (p->agg.cls[kClsWaveHash] > 0) {
        const dim3 grid(p->total_blocks), block(kNumWavesH * kWave);
        const uint8_t want = kClsWaveHash;
        if (p->th.wave_hash_log2 == 10)
            launch_num_hash<T, IdxT, IdxC, kWaveHashSlotsMax>(p, tab, grid, block, a0, P, bm, want);
        else
            launch_num_hash<T, IdxT, IdxC, kWaveHashSlots>(p, tab, grid, block, a0, P, bm, want);
        REAP_LAUNCH_CHECK();
        debug_step(p, "k_num_wave_hash");
    }
    ev_record(p, kPhNumHash, true);
    ev_record(p, kPhNumGroup, false);
    if (p->mid_rows + p->big_rows > 0) {
        hipLaunchKernelGGL(k_long_rewind, dim3(1), dim3(64), 0, p->stream, bm.queue);
        REAP_LAUNCH_CHECK();
    }
    if (p->mid_rows > 0) {
        hipLaunchKernelGGL((k_long_num<T, IdxT, IdxC, LongNumMid>), dim3(p->mid_grid), dim3(LongNumMid::NT), 0,
                           p->stream, a0, P, bm);
        REAP_LAUNCH_CHECK();
        debug_step(p, "k_long_num<mid>");
    }
    if (p->big_rows > 0) {
        hipLaunchKernelGGL((k_long_num<T, IdxT, IdxC, LongNumLarge>), dim3(p->big_grid), dim3(LongNumLarge::NT), 0,
                           p->stream, a0, P, bm);
        REAP_LAUNCH_CHECK();
        debug_step(p, "k_long_num<large>");
    }
    ev_record(p, kPhNumGroup, true);
    ev_record(p, kPhNumAll, true);
    return REAP_OK;
}

template <typename T, typename IdxT, typename IdxC>
reap_status_t numeric_typed(reap_spgemm_s* p, const reap_csr_t* A, const reap_csr_t* B, const void* const* c_row_ptr,
                            int32_t* const* c_col, void* const* c_val) {
    if (p->ev_num_upload && p->num_upload_recorded) REAP_HIP(hipEventSynchronize(p->ev_num_upload));
    NumArgs<T, IdxT, IdxC> a0{};
    for (int q = 0; q < p->nprod; ++q) {
        const ProdState& ps = p->prods[(size_t)q];
        NumArgs<T, IdxT, IdxC> a{};
        a.m = ps.m;
        a.n = ps.n;
        a.k = ps.k;
        a.a_rp = to_gptr(static_cast<const IdxT*>(A[q].row_ptr));
        a.a_col = to_gptr(A[q].col_idx);
        a.a_val = to_gptr(static_cast<const T*>(A[q].values));
        a.b_rp = to_gptr(static_cast<const IdxT*>(B[q].row_ptr));
        a.b_col = to_gptr(B[q].col_idx);
        a.b_val = to_gptr(static_cast<const T*>(B[q].values));
        a.c_rp = to_gptr(static_cast<const IdxC*>(c_row_ptr[q]));
        a.c_col = to_gptr(c_col[q]);
        a.c_val = to_gptr(static_cast<T*>(c_val[q]));
        a.cls = to_gptr(p->cls + ps.row_off);
        a.win = to_gptr(p->win + ps.row_off);
        a.ctr = to_gptr(p->ctr + q);
        a.gvals = to_gptr(p->gvals_ptr);
        a.gvals_stride = p->gvals_stride;
        a.th = p->th;
        std::memcpy(p->h_stage_num + (size_t)q * sizeof(a), &a, sizeof(a));
        if (q == 0) a0 = a;
    }
    // after an allocation-free symbolic call the kernels run directly, so that
    // this call allocates nothing either
    if (!p->use_graph || p->eager) return launch_numeric<T, IdxT, IdxC>(p, a0);
    std::vector<uint64_t> key = {p->ws_generation, (uint64_t)p->nprod, (uint64_t)p->total_blocks,
                                 (uint64_t)p->long_rows, (uint64_t)p->long_grid, (uint64_t)p->mid_rows,
                                 (uint64_t)p->big_rows, (uint64_t)p->mid_grid, (uint64_t)p->big_grid,
                                 (uint64_t)(p->agg.cls[kClsWaveBmpS] > 0), (uint64_t)(p->agg.cls[kClsWaveHash] > 0),
                                 (uint64_t)sizeof(T), (uint64_t)sizeof(IdxT), (uint64_t)sizeof(IdxC),
                                 (uint64_t)(uintptr_t)p->gvals_ptr, (uint64_t)p->gvals_stride, (uint64_t)p->buf_b};
    const reap_status_t st =
        run_pass(p, p->g_num, p->g_num_key, key, [&]() { return launch_numeric<T, IdxT, IdxC>(p, a0); });
    if (st == REAP_OK && p->use_graph) {
        // a replayed graph reads the staging buffer when it runs: keep it until then
        REAP_HIP(hipEventRecord(p->ev_num_upload, p->stream));
        p->num_upload_recorded = true;
    }
    return st;
}

reap_status_t numeric_batch(reap_spgemm_s* p, int64_t count, const reap_csr_t* A, const reap_csr_t* B,
                            const void* const* c_row_ptr, int32_t* const* c_col, void* const* c_val) {
    if (!p || !A || !B || !c_row_ptr || !c_col || !c_val) return REAP_ERR_INVALID_ARG;
    if (!p->have_symbolic || count != p->nprod) return REAP_ERR_STATE;
    reap_status_t st;
    int64_t total_nnz = 0;
    for (int q = 0; q < p->nprod; ++q) {
        const ProdState& ps = p->prods[(size_t)q];
        if ((st = check_csr(&A[q])) != REAP_OK) return st;
        if ((st = check_csr(&B[q])) != REAP_OK) return st;
        if (!c_row_ptr[q]) return REAP_ERR_INVALID_ARG;
        if (A[q].rows != ps.m || A[q].cols != ps.k || B[q].cols != ps.n || A[q].nnz != ps.a_nnz ||
            B[q].nnz != ps.b_nnz || A[q].row_ptr_type != p->in_idx || B[q].row_ptr_type != p->in_idx)
            return REAP_ERR_STATE;
        if (ps.c_nnz > 0 && (!c_col[q] || !c_val[q])) return REAP_ERR_INVALID_ARG;
        total_nnz += ps.c_nnz;
    }
    if (total_nnz == 0) return REAP_OK;
    const bool i32 = p->in_idx == REAP_I32, c32 = p->cidx == REAP_I32;
    p->numeric_ran = true;
    if (p->dtype == REAP_F64) {
        if (i32 && c32) return numeric_typed<double, int32_t, int32_t>(p, A, B, c_row_ptr, c_col, c_val);
        if (i32 && !c32) return numeric_typed<double, int32_t, int64_t>(p, A, B, c_row_ptr, c_col, c_val);
        if (!i32 && c32) return numeric_typed<double, int64_t, int32_t>(p, A, B, c_row_ptr, c_col, c_val);
        return numeric_typed<double, int64_t, int64_t>(p, A, B, c_row_ptr, c_col, c_val);
    }
    if (i32 && c32) return numeric_typed<float, int32_t, int32_t>(p, A, B, c_row_ptr, c_col, c_val);
    if (i32 && !c32) return numeric_typed<float, int32_t, int64_t>(p, A, B, c_row_ptr, c_col, c_val);
    if (!i32 && c32) return numeric_typed<float, int64_t, int32_t>(p, A, B, c_row_ptr, c_col, c_val);
    return numeric_typed<float, int64_t, int64_t>(p, A, B, c_row_ptr, c_col, c_val);
}

// ---------------------------------------------------------------------------
// Device transpose.

template <typename IdxC>
reap_status_t launch_scan(reap_spgemm_s* p, const int32_t* counts, int64_t m, long long* tiles, Counters* dummy,
                          void* out) {
    ScanArgs s{};
    s.rnnz = counts;
    s.m = m;
    s.tiles = tiles;
    s.ntiles = (int32_t)((m + kScanTile - 1) / kScanTile);
    s.nparts = 0;
    s.parts = nullptr;
    s.ctr = dummy;
    s.c_rp = out;
    ScanMap sm;
    sm.tile_start = nullptr;
    sm.nprod = 1;
    if (s.ntiles > 0) {
        hipLaunchKernelGGL(k_scan_tiles, dim3(s.ntiles), dim3(kScanThreads), 0, p->stream, s, nullptr, sm);
        REAP_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_scan_spine<IdxC>, dim3(1), dim3(1024), 0, p->stream, s, nullptr);
    REAP_LAUNCH_CHECK();
    if (s.ntiles > 0) {
        hipLaunchKernelGGL(k_scan_apply<IdxC>, dim3(s.ntiles), dim3(kScanThreads), 0, p->stream, s, nullptr, sm);
        REAP_LAUNCH_CHECK();
    }
    return REAP_OK;
}

template <typename T, typename IdxT>
reap_status_t transpose_typed(reap_spgemm_s* p, const reap_csr_t* A, void* t_row_ptr, int32_t* t_col, void* t_val) {
    const int64_t m = A->rows, n = A->cols, nnz = A->nnz;
    const int64_t ntiles = (nnz + kRsTile - 1) / kRsTile;
    const int64_t nh = (int64_t)kRsBins * ntiles;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t o_row = carve((size_t)nnz * 4);
    const size_t o_k0 = carve((size_t)nnz * 4), o_v0 = carve((size_t)nnz * 4);
    const size_t o_k1 = carve((size_t)nnz * 4), o_v1 = carve((size_t)nnz * 4);
    const size_t o_cnt = carve((size_t)(n + 1) * 4);
    const size_t o_h = carve((size_t)(nh + 1) * 4), o_off = carve((size_t)(nh + 1) * 4);
    const size_t o_t1 = carve((size_t)((n + kScanTile) / kScanTile + 1) * 8);
    const size_t o_t2 = carve((size_t)((nh + kScanTile) / kScanTile + 1) * 8);
    const size_t o_c = carve(sizeof(Counters));
    if (off > p->tws.bytes) {
        (void)hipStreamSynchronize(p->stream);
        if (p->tws.base) (void)hipFree(p->tws.base);
        p->tws.base = nullptr;
        p->tws.bytes = 0;
        if (dev_malloc(p, &p->tws.base, off) != hipSuccess) {
            (void)hipGetLastError();
            return REAP_ERR_OUT_OF_MEMORY;
        }
        p->tws.bytes = off;
    }
    char* b = static_cast<char*>(p->tws.base);
    int32_t* rowid = reinterpret_cast<int32_t*>(b + o_row);
    int32_t* keys[2] = {reinterpret_cast<int32_t*>(b + o_k0), reinterpret_cast<int32_t*>(b + o_k1)};
    int32_t* vals[2] = {reinterpret_cast<int32_t*>(b + o_v0), reinterpret_cast<int32_t*>(b + o_v1)};
    int32_t* cnt = reinterpret_cast<int32_t*>(b + o_cnt);
    int32_t* hist = reinterpret_cast<int32_t*>(b + o_h);
    int32_t* offs = reinterpret_cast<int32_t*>(b + o_off);
    long long* t1 = reinterpret_cast<long long*>(b + o_t1);
    long long* t2 = reinterpret_cast<long long*>(b + o_t2);
    Counters* dummy = reinterpret_cast<Counters*>(b + o_c);
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((nnz + 255) / 256, (int64_t)p->num_cus * 16));

    // row pointer of the transpose: column counts, exclusive scan
    const int gz = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, (int64_t)p->num_cus * 16));
    hipLaunchKernelGGL(k_tr_zero, dim3(gz), dim3(256), 0, p->stream, cnt, n);
    REAP_LAUNCH_CHECK();
    if (nnz > 0) {
        hipLaunchKernelGGL(k_tr_colcount, dim3(g), dim3(256), 0, p->stream, A->col_idx, nnz, cnt);
        REAP_LAUNCH_CHECK();
    }
    reap_status_t st = launch_scan<IdxT>(p, cnt, n, t1, dummy, t_row_ptr);
    if (st != REAP_OK) return st;
    debug_step(p, "transpose row pointer");
    if (nnz == 0) return REAP_OK;

    // entries ordered by column (stable: A's row order is kept inside a column)
    if (m > 0) {
        hipLaunchKernelGGL(k_tr_rowid<IdxT>, dim3((unsigned)((m * kWave + 255) / 256)), dim3(256), 0, p->stream,
                           static_cast<const IdxT*>(A->row_ptr), m, rowid);
        REAP_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_tr_iota, dim3(g), dim3(256), 0, p->stream, vals[0], nnz);
    REAP_LAUNCH_CHECK();
    const int bits = n <= 1 ? 0 : 32 - __builtin_clz((unsigned)(n - 1));
    const int passes = (bits + 7) / 8;
    const int32_t* kin = A->col_idx;
    const int32_t* vin = vals[0];
    int cur = 1;
    for (int ps = 0; ps < passes; ++ps) {
        hipLaunchKernelGGL(k_rs_count, dim3((unsigned)ntiles), dim3(kRsThreads), 0, p->stream, kin, nnz, 8 * ps, hist);
        REAP_LAUNCH_CHECK();
        if ((st = launch_scan<int32_t>(p, hist, nh, t2, dummy, offs)) != REAP_OK) return st;
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)ntiles), dim3(kRsThreads), 0, p->stream, kin, vin, nnz,
                           8 * ps, offs, keys[cur], vals[cur]);
        REAP_LAUNCH_CHECK();
        kin = keys[cur];
        vin = vals[cur];
        cur ^= 1;
    }
    debug_step(p, "transpose sort");
    hipLaunchKernelGGL((k_tr_gather<T>), dim3(g), dim3(256), 0, p->stream, vin, nnz, rowid,
                       static_cast<const T*>(A->values), t_col, static_cast<T*>(t_val));
    REAP_LAUNCH_CHECK();
    debug_step(p, "transpose gather");
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
        case REAP_ERR_TOO_LARGE: return "product exceeds the static scratch of the allocation-free entry point";
    }
    return "unknown status";
}

const char* reap_version(void) { return "0.2.0"; }

reap_status_t reap_spgemm_create(reap_spgemm_t* plan, reap_dtype_t dtype, reap_index_t c_row_ptr_type, void* stream,
                                 const reap_options_t* opts) {
    if (!plan) return REAP_ERR_INVALID_ARG;
    *plan = nullptr;
    if (dtype != REAP_F32 && dtype != REAP_F64) return REAP_ERR_INVALID_ARG;
    if (c_row_ptr_type != REAP_I32 && c_row_ptr_type != REAP_I64) return REAP_ERR_INVALID_ARG;
    reap_options_t o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.graph && !stream) return REAP_ERR_INVALID_ARG;  // the legacy default stream cannot be captured
    reap_spgemm_s* p = new (std::nothrow) reap_spgemm_s();
    if (!p) return REAP_ERR_OUT_OF_MEMORY;
    p->dtype = dtype;
    p->cidx = c_row_ptr_type;
    p->stream = static_cast<hipStream_t>(stream);
    p->validate = o.validate != 0;
    p->profile = o.profile != 0;
    p->use_graph = o.graph != 0 && !p->validate;
    const char* dbg = std::getenv("REAP_DEBUG_SYNC");
    p->debug_sync = dbg && dbg[0] == '1';
    if (p->debug_sync) p->use_graph = false;
    p->th.wave_max_products = clampi(o.wave_max_products, 0, kWaveMaxProducts, kWaveMaxProducts);
    p->th.wave_max_span = clampi(o.wave_max_span, 0, 32 * kWaveBitsWords, 32 * kWaveBitsWords);
    p->th.wave_hash_log2 = o.wave_hash_slots == kWaveHashSlotsMax ? 10 : 9;
    p->th.wave_hash_products = clampi(o.wave_hash_products, 0, (1 << p->th.wave_hash_log2) / 2,
                                      (1 << p->th.wave_hash_log2) / 2);
    p->th.wave_small_nnz = clampi(o.wave_small_values, 0, kWaveSmallNnz, kWaveSmallNnz);
    p->th.group_lds_span = clampi(o.group_lds_span, 32, 32 * kGroupBitsWords, 32 * kGroupBitsWords) / 32 * 32;
    p->th.group_lds_values = clampi(o.group_lds_values, kLongMinVals, kLongVals, kLongVals);
    p->long_wg_per_cu = clampi(o.long_workgroups_per_cu, 1, 8, 2);
    p->th.mid_nnz = clampi(o.mid_values, 0, LongNumMid::VMAX, LongNumMid::VMAX);
    p->sym_narrow = o.long_sym_narrow >= 0;
    p->fail_alloc_at = std::max(0, o.test_fail_alloc);
    p->scan_onepass = clampi(o.scan_onepass_tiles, 0, kScanOnePassTiles, kScanOnePassTiles);

    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&p->num_cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_num_upload, hipEventDisableTiming);
    void* scratch_ptr = nullptr;
    if (e != hipSuccess || static_scratch(p->device, &scratch_ptr) != REAP_OK) {
        // the device address of the static scratch is looked up here, once per
        // device, with the plan's device current
        (void)hipGetLastError();
        if (p->ev_num_upload) (void)hipEventDestroy(p->ev_num_upload);
        delete p;
        return REAP_ERR_HIP;
    }
    p->prods.reserve(1);  // one product's record: the allocation-free call never grows it
    if (ensure_host(p, 1) != REAP_OK || ensure_host_tiles(p, kScanOnePassTiles) != REAP_OK) {
        if (p->h_ctr) (void)hipHostFree(p->h_ctr);
        if (p->h_stage) (void)hipHostFree(p->h_stage);
        if (p->h_stage_num) (void)hipHostFree(p->h_stage_num);
        (void)hipEventDestroy(p->ev_num_upload);
        delete p;
        return REAP_ERR_OUT_OF_MEMORY;
    }
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
    release_graphs(p);
    if (p->ws.base) (void)hipFree(p->ws.base);
    if (p->gvals.base) (void)hipFree(p->gvals.base);
    if (p->tws.base) (void)hipFree(p->tws.base);
    if (p->h_ctr) (void)hipHostFree(p->h_ctr);
    if (p->h_tiles) (void)hipHostFree(p->h_tiles);
    if (p->h_stage) (void)hipHostFree(p->h_stage);
    if (p->h_stage_num) (void)hipHostFree(p->h_stage_num);
    if (p->ev_num_upload) (void)hipEventDestroy(p->ev_num_upload);
    for (int i = 0; i < 2 * kNumPhases; ++i)
        if (p->ev[i]) (void)hipEventDestroy(p->ev[i]);
    delete p;
    return REAP_OK;
}

reap_status_t reap_spgemm_symbolic(reap_spgemm_t p, const reap_csr_t* A, const reap_csr_t* B, void* c_row_ptr,
                                   int64_t* c_nnz, int64_t* n_products, size_t* workspace_bytes) {
    if (!p || !A || !B || !c_nnz || !c_row_ptr) return REAP_ERR_INVALID_ARG;
    void* rp[1] = {c_row_ptr};
    return symbolic_batch(p, 1, A, B, rp, c_nnz, n_products, workspace_bytes);
}

reap_status_t reap_spgemm_symbolic_noalloc(reap_spgemm_t p, const reap_csr_t* A, const reap_csr_t* B, void* c_row_ptr,
                                           int64_t* c_nnz, int64_t* n_products) {
    if (!p || !A || !B || !c_nnz || !c_row_ptr) return REAP_ERR_INVALID_ARG;
    void* rp[1] = {c_row_ptr};
    return symbolic_batch(p, 1, A, B, rp, c_nnz, n_products, nullptr, true);
}

reap_status_t reap_spgemm_numeric(reap_spgemm_t p, const reap_csr_t* A, const reap_csr_t* B, const void* c_row_ptr,
                                  int32_t* c_col_idx, void* c_values) {
    if (!p || !A || !B || !c_row_ptr) return REAP_ERR_INVALID_ARG;
    if (p->have_symbolic && p->nprod != 1) return REAP_ERR_STATE;
    const void* rp[1] = {c_row_ptr};
    int32_t* cc[1] = {c_col_idx};
    void* cv[1] = {c_values};
    return numeric_batch(p, 1, A, B, rp, cc, cv);
}

reap_status_t reap_spgemm_batch_symbolic(reap_spgemm_t p, int64_t count, const reap_csr_t* A, const reap_csr_t* B,
                                         void* const* c_row_ptr, int64_t* c_nnz, int64_t* n_products,
                                         size_t* workspace_bytes) {
    return symbolic_batch(p, count, A, B, c_row_ptr, c_nnz, n_products, workspace_bytes);
}

reap_status_t reap_spgemm_batch_numeric(reap_spgemm_t p, int64_t count, const reap_csr_t* A, const reap_csr_t* B,
                                        const void* const* c_row_ptr, int32_t* const* c_col_idx,
                                        void* const* c_values) {
    return numeric_batch(p, count, A, B, c_row_ptr, c_col_idx, c_values);
}

reap_status_t reap_spgemm_workspace_query(reap_spgemm_t p, int64_t count, const reap_csr_t* A, const reap_csr_t* B,
                                          size_t* bytes) {
    if (!p || !bytes) return REAP_ERR_INVALID_ARG;
    BatchTotals bt;
    const reap_status_t st = batch_totals(count, A, B, &bt);
    if (st != REAP_OK) return st;
    // the workspace grows to the larger of its current and the needed sizes, never shrinks
    const int64_t R = std::max<int64_t>({bt.rows, p->cap_rows, 1});
    const int32_t Bk = std::max({(int32_t)bt.blocks, p->cap_blocks, 1});
    const int32_t Tl = std::max({(int32_t)bt.tiles, p->cap_tiles, 1});
    const int64_t Q = std::max<int64_t>({count, p->cap_prods, 1});
    const size_t ws = std::max(p->ws.bytes, ws_layout(R, Bk, Tl, Q).total);
    *bytes = ws + std::max(p->gvals.bytes, gvals_bound(p, bt));
    return REAP_OK;
}

reap_status_t reap_csr_transpose(reap_spgemm_t p, const reap_csr_t* A, void* t_row_ptr, int32_t* t_col_idx,
                                 void* t_values) {
    if (!p || !A || !t_row_ptr) return REAP_ERR_INVALID_ARG;
    reap_status_t st;
    if ((st = check_csr(A)) != REAP_OK) return st;
    if (A->nnz > INT32_MAX || A->rows > INT32_MAX) return REAP_ERR_INVALID_ARG;  // int32 entry and row ids
    if (A->nnz > 0 && (!t_col_idx || !t_values)) return REAP_ERR_INVALID_ARG;
    const bool i32 = A->row_ptr_type == REAP_I32;
    if (p->dtype == REAP_F64)
        return i32 ? transpose_typed<double, int32_t>(p, A, t_row_ptr, t_col_idx, t_values)
                   : transpose_typed<double, int64_t>(p, A, t_row_ptr, t_col_idx, t_values);
    return i32 ? transpose_typed<float, int32_t>(p, A, t_row_ptr, t_col_idx, t_values)
               : transpose_typed<float, int64_t>(p, A, t_row_ptr, t_col_idx, t_values);
}

reap_status_t reap_spgemm_bin_stats(reap_spgemm_t p, reap_bin_stats_t* out) {
    if (!p || !out) return REAP_ERR_INVALID_ARG;
    if (!p->have_symbolic) return REAP_ERR_STATE;
    const Counters& h = p->agg;
    out->empty = (int64_t)h.cls[kClsEmpty];
    out->wave_bitmap = (int64_t)(h.cls[kClsWaveBmpS] + h.cls[kClsWaveBmpL]);
    out->wave_hash = (int64_t)h.cls[kClsWaveHash];
    out->group = (int64_t)h.cls[kClsGroup];
    out->group_medium = (int64_t)p->mid_rows;
    out->max_row_products = (int64_t)h.max_prod;
    out->max_row_nnz = (int64_t)h.max_nnz;
    out->long_segments_lds = out->long_segments_chunked = out->long_segments_device = 0;
    if (p->numeric_ran && p->long_rows > 0) {
        // the numeric kernels count on the device: wait for them and read back
        REAP_HIP(hipStreamSynchronize(p->stream));
        REAP_HIP(hipMemcpy(p->h_ctr, p->ctr, (size_t)p->nprod * sizeof(Counters), hipMemcpyDeviceToHost));
        for (int q = 0; q < p->nprod; ++q) {
            out->long_segments_lds += p->h_ctr[q].seg_lds;
            out->long_segments_chunked += p->h_ctr[q].seg_chunked;
            out->long_segments_device += p->h_ctr[q].seg_device;
        }
    }
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
