// Types shared by the SpGEMM kernels and the host plan.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace reap {

// Pointer into device memory, typed as such for the device compiler.
// Argument structs read from a table in memory would otherwise hold generic
// pointers, accessed with FLAT instructions; those count against the LDS
// counter too, so every wait for an LDS result would also wait for the loads
// in flight.  The host pass sees plain pointers of the same size.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
#else
template <typename T>
using gptr = T*;
#endif

template <typename T>
__host__ __device__ inline gptr<T> to_gptr(T* p) {
    return (gptr<T>)p;
}

// Row classes, decided by the symbolic pass from the row's partial-product
// count P_i, its number of A entries, its column window and nnz(C_i).
enum RowClass : uint8_t {
    kClsEmpty = 0,     // P_i = 0: the row of C is empty
    kClsWaveBmpS = 1,  // one wavefront, circular LDS bitmap, at most kWaveSmallNnz entries of C
    kClsWaveBmpL = 2,  // not produced
    kClsWaveHash = 3,  // one wavefront, LDS hash table (window too wide for the bitmap)
    kClsGroup = 4,     // one workgroup: long rows
    kNumClasses = 5
};

constexpr int kWaveMaxProducts = 1024;   // product slots of a wavefront row (16 per lane)
constexpr int kWaveBitsWords = 1024;     // circular bitmap of the wavefront kernels: 32768 columns
constexpr int kWaveSmallNnz = 128;       // entries of C a wavefront numeric row holds
constexpr int kWaveHashProducts = 256;   // hash rows: at most 256 products (the default table)
constexpr int kWaveHashSlots = 512;      // default hash table: load factor <= 1/2
constexpr int kWaveHashSlotsMax = 1024;  // the larger table (rows of at most 512 products)
constexpr int kGroupBitsWords = 8192;    // 262144-column LDS bitmap segment of a long row
constexpr int kRowsPerWave = 8;          // consecutive rows a wavefront walks through
constexpr int kStageCap = 256;           // A entries of one chunk of rows staged in LDS (symbolic)

// Per-workgroup partial statistics of the wavefront symbolic kernel.
struct WGPart {
    unsigned long long products;
    unsigned int cls[kNumClasses];
    unsigned int max_prod;
    unsigned int max_nnz;
    unsigned int pad;
};

// Device-side counters, copied to the host at the end of the symbolic pass.
struct Counters {
    unsigned long long products;   // total partial products
    unsigned long long nnz;        // nnz(C)
    unsigned long long cls[8];     // rows per class
    unsigned int max_prod;         // max partial products in one row (saturating)
    unsigned int max_nnz;          // max nnz of one row of C
    unsigned int n_group;          // length of the long-row list
    unsigned int seg_lds;          // numeric: long-row window segments summed in LDS in one walk
    unsigned int seg_chunked;      // numeric: segments summed in LDS rank chunks
    unsigned int max_group_nnz;    // max nnz of a long row
    unsigned int bad_csr;          // validation flags (bit 0: A, bit 1: B)
    unsigned int seg_device;       // numeric: segments summed with device-memory atomics
    unsigned int pad[4];
};

// Statistics of one scan tile, written by the one-launch scan into pinned
// host memory; the host adds the tiles of each product to its counters.
struct TileStat {
    unsigned long long nnz;        // entries of C in the tile's rows
    unsigned long long products;   // partial products of the tile's wavefront rows
    unsigned int cls[kNumClasses]; // rows per class
    unsigned int max_prod;
    unsigned int max_nnz;
    unsigned int pad;
};

// Rows handled by one workgroup of the wavefront kernels (4 wavefronts of
// kRowsPerWave rows); the batch's block table is built for this many rows.
constexpr int kWaveKernelWaves = 4;
constexpr int kRowsPerBlock = kWaveKernelWaves * kRowsPerWave;

// Scan of the row counts into C's row pointer: tiles of kScanTile rows.  The
// symbolic kernels add each row's count into its tile's sum as they go, so a
// workgroup of a wavefront kernel (whose rows never straddle two tiles) adds
// once per launch.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // rows per tile
static_assert(kScanTile % kRowsPerBlock == 0, "a wavefront workgroup's rows lie in one scan tile");

// Several independent products in one launch.  Workgroup b of a wavefront
// kernel serves product q with blk_start[q] <= b < blk_start[q + 1]; its
// arguments are args[q] (or the kernel's by-value argument when nprod == 1).
// Long rows of every product are appended to one list of (product, row).
// The symbolic long-row pass sorts the list into medium rows (their window
// and nnz(C_i) fit the medium numeric workgroup) and large rows: split_list
// holds the medium ones from its start and the large ones from its end.
struct BatchMap {
    const int32_t* blk_start;  // [nprod + 1]
    int32_t nprod;
    int2* long_list;           // [sum of rows]
    unsigned int* n_long;      // length of long_list
    unsigned int* queue;       // next entry to take: [0] long_list (symbolic), [1] large rows, [2] medium rows
    int2* split_list;          // [split_cap]
    unsigned int split_cap;
    unsigned int* n_split;     // [0] medium rows, [1] large rows
};

// Layout of the plan's long-row counter block (unsigned ints).
constexpr int kLongCtrCount = 0;     // long_list length
constexpr int kLongCtrQueue = 1;     // three queue counters
constexpr int kLongCtrSplit = 4;     // medium and large row counts
constexpr int kLongCtrWords = 8;

// Thresholds of one plan (clamped to the kernel capacities above).
struct Thresholds {
    int wave_max_products;   // <= kWaveMaxProducts
    int wave_max_span;       // <= 32 * kWaveBitsWords
    int wave_hash_products;  // <= (1 << wave_hash_log2) / 2
    int wave_hash_log2;      // hash-class table: 9 (512 slots) or 10 (1024 slots)
    int wave_small_nnz;      // <= kWaveSmallNnz
    int group_lds_span;      // <= 32 * kGroupBitsWords, multiple of 32
    int group_lds_values;    // FP64 LDS slots per rank chunk of a long row, kLongMinVals..kLongVals
    int mid_nnz;             // long rows with at most this many entries of C (and a narrow window) are
                             // medium rows; 0: none
};

}  // namespace reap
