/*
 * reap_spgemm.h -- sparse general matrix-matrix product C = A * B on CSR
 * operands, computed on an AMD Instinct MI355X (gfx950) GPU.
 *
 * The operation is the paper's row-by-row sparse product (Section III-A,
 * Algorithm 1): each row i of C is formed from the rows of B selected by the
 * column indices of row i of A; every matching pair contributes one partial
 * product a_ik * b_kj, and products with the same column are summed into one
 * entry.  Rows of C are returned with strictly ascending column indices.
 * Entries whose products cancel to zero are kept (the algorithm emits every
 * column of the row's column set).
 *
 * The work is split in two calls, as the allocation of C requires:
 *   symbolic -- counts partial products and the number of entries of every row
 *               of C, writes C's row pointer, returns nnz(C) to the host;
 *   numeric  -- fills C's column indices and values.
 * Memory: every A, B and C array is owned by the caller and lives in device
 * memory.  The plan owns only its workspace (per-row counts and classes, long
 * row scratch), which it allocates in `symbolic`, reuses across calls and
 * releases in `destroy`.
 *
 * Errors: every entry point returns a reap_status_t; nothing throws or aborts.
 * After an error the plan may still be passed to reap_spgemm_destroy.  A plan
 * is not thread-safe; distinct plans are independent.
 */
#ifndef REAP_SPGEMM_H
#define REAP_SPGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct reap_spgemm_s* reap_spgemm_t;

typedef enum {
    REAP_OK = 0,
    REAP_ERR_INVALID_ARG = 1,    /* null pointer, negative size, A.cols != B.rows, dtype mismatch */
    REAP_ERR_BAD_CSR = 2,        /* validation found a malformed operand (opt-in check) */
    REAP_ERR_INDEX_OVERFLOW = 3, /* nnz(C) does not fit the requested C row-pointer type */
    REAP_ERR_OUT_OF_MEMORY = 4,  /* workspace allocation failed */
    REAP_ERR_STATE = 5,          /* numeric called without a matching symbolic */
    REAP_ERR_HIP = 6,            /* a HIP runtime call failed (includes earlier kernel faults) */
    REAP_ERR_TOO_LARGE = 7       /* the product exceeds the static scratch of reap_spgemm_symbolic_noalloc */
} reap_status_t;

/* Bytes of the per-device static scratch used by reap_spgemm_symbolic_noalloc. */
#define REAP_NOALLOC_SCRATCH_BYTES (64u << 20)

typedef enum { REAP_F32 = 0, REAP_F64 = 1 } reap_dtype_t;
typedef enum { REAP_I32 = 0, REAP_I64 = 1 } reap_index_t;

/*
 * One CSR operand in device memory (CSR as in the paper's Section I and
 * Section III-A: row pointer, column index, value).
 *   rows, cols    -- matrix shape (>= 0);
 *   nnz           -- number of stored entries; must equal row_ptr[rows];
 *   row_ptr_type  -- REAP_I32 or REAP_I64: element type of row_ptr;
 *   row_ptr       -- rows+1 entries, row_ptr[0] = 0, non-decreasing;
 *   col_idx       -- nnz int32 column indices in [0, cols); any order inside a
 *                    row; a repeated column adds;
 *   values        -- nnz values of the plan's dtype (float or double).
 * Pointers may be NULL only when the corresponding count is zero.
 */
typedef struct {
    int64_t rows, cols, nnz;
    reap_index_t row_ptr_type;
    const void* row_ptr;
    const int32_t* col_idx;
    const void* values;
} reap_csr_t;

/*
 * Tuning and test options.  Zero-initialise and set what you need, or pass
 * NULL for defaults.  Thresholds only change which kernel handles a row,
 * never the result.
 *   validate          -- non-zero: check both operands (row_ptr monotone, ends
 *                        at nnz, columns in range) before use; costs one pass.
 *   wave_max_products -- rows with at most this many partial products (and at
 *                        most 64 entries in A) are computed by one wavefront
 *                        (<= 1024; 0 = default 1024).
 *   wave_max_span     -- widest column window (max col - min col + 1) a
 *                        wavefront handles with a bitmap (<= 32768; 0 = default).
 *   wave_hash_products-- rows wider than that window but with at most this many
 *                        products use a wavefront hash table (<= half of
 *                        wave_hash_slots; 0 = default, that half).
 *   group_lds_span    -- columns per segment of a long row's window: a long
 *                        row's LDS bitmap covers this many columns at a time
 *                        and wider windows are processed segment by segment
 *                        (<= 262144, rounded down to a multiple of 32, at
 *                        least 32; 0 = default 262144).
 *   group_lds_values  -- FP64 accumulator slots in LDS for a long row (256 ..
 *                        8192; 0 = default 8192).  A long row's window
 *                        segment whose entries fit is summed in LDS in one
 *                        walk; a larger one in chunks of this many
 *                        consecutive entries, when the B rows it reads are
 *                        in column order, else in device memory.
 *   profile           -- non-zero: record per-phase device times (see
 *                        reap_spgemm_phase_times).
 *   wave_small_values -- rows of C with at most this many entries (and a
 *                        window of at most 20480 columns) use the compact
 *                        wavefront kernel (<= 128; 0 = default 128).
 *   graph             -- non-zero: each symbolic and numeric call is captured
 *                        into a HIP graph the first time its launch shape
 *                        occurs and replayed while the shape repeats (one
 *                        graph launch per call instead of one launch per
 *                        kernel).  Needs a stream other than the legacy
 *                        default stream; ignored with `validate` or with
 *                        REAP_DEBUG_SYNC=1 in the environment.
 *   long_workgroups_per_cu -- workgroups per compute unit that take rows
 *                        from the long-row list in the symbolic pass (1..8;
 *                        0 = default 2; the numeric pass runs one per CU).
 *   test_fail_alloc   -- test hook for callers' error handling: when n > 0,
 *                        the plan's n-th device allocation (workspace,
 *                        accumulators or transpose scratch, counted from 1)
 *                        fails as if the device were out of memory, so the
 *                        call returns REAP_ERR_OUT_OF_MEMORY; 0 = never.
 *   scan_onepass_tiles -- batches whose products all have at most this many
 *                        scan tiles (2048 rows each) build C's row pointer
 *                        with one kernel launch; larger ones with two (a
 *                        per-product spine over the tile sums, then the
 *                        rows).  <= 1024; 0 = default 1024; negative: always
 *                        two launches.
 *   mid_values        -- long rows with at most this many entries of C whose
 *                        columns span at most 65536 columns are summed by
 *                        medium workgroups (256 threads, three per CU)
 *                        instead of one 1024-thread workgroup per CU
 *                        (<= 2048; 0 = default 2048; negative: none).
 *   long_sym_narrow   -- the symbolic long-row pass runs 256-thread
 *                        workgroups with a 65536-column bitmap (twice as
 *                        many per CU) when every product of the call has at
 *                        most 65536 columns: 0 = yes (default), negative = no.
 *   wave_hash_slots   -- LDS hash-table slots of the wavefront hash class:
 *                        512 (default, any value other than 1024) or 1024;
 *                        rows of at most half as many products qualify
 *                        (wave_hash_products defaults to that half).
 * For every threshold, 0 selects the default and a negative value 0.
 */
typedef struct {
    int32_t validate;
    int32_t wave_max_products;
    int32_t wave_max_span;
    int32_t wave_hash_products;
    int32_t group_lds_span;
    int32_t group_lds_values;
    int32_t profile;
    int32_t wave_small_values;
    int32_t graph;
    int32_t long_workgroups_per_cu;
    int32_t test_fail_alloc;
    int32_t scan_onepass_tiles;
    int32_t mid_values;
    int32_t long_sym_narrow;
    int32_t wave_hash_slots;
    int32_t reserved[1];
} reap_options_t;

/*
 * Per-class row counts of the last symbolic pass (how rows were binned) and,
 * once a numeric call has followed it, how the long rows' window segments
 * were accumulated (summed over the numeric calls since that symbolic call).
 */
typedef struct {
    int64_t empty;        /* rows with no partial product */
    int64_t wave_bitmap;  /* one wavefront, LDS bitmap over the column window */
    int64_t wave_hash;    /* one wavefront, LDS hash table + sort */
    int64_t group;        /* one workgroup (long rows), LDS or device bitmap */
    int64_t max_row_products;
    int64_t max_row_nnz;
    int64_t long_segments_lds;      /* long-row window segments summed in LDS in one walk */
    int64_t long_segments_chunked;  /* ... summed in LDS rank chunks (B rows in column order) */
    int64_t long_segments_device;   /* ... summed with device-memory atomics */
    int64_t group_medium; /* long rows summed by medium workgroups (of `group`) */
} reap_bin_stats_t;

/*
 * Create a plan for products with values of type `dtype` and a C row pointer
 * of type `c_row_ptr_type`, enqueued on `stream` (a hipStream_t; NULL = the
 * default stream).  Binds to the current HIP device.  *plan is set to NULL on
 * failure.  Errors: INVALID_ARG, HIP.
 */
reap_status_t reap_spgemm_create(reap_spgemm_t* plan, reap_dtype_t dtype,
                                 reap_index_t c_row_ptr_type, void* stream,
                                 const reap_options_t* opts);

/*
 * Symbolic pass (the row product count, the binning of rows by their product
 * count, the per-row count of distinct columns -- the column set COLB of the
 * paper's Algorithm 1 -- and the prefix scan that places each row of C).
 *   c_row_ptr   -- device, A.rows+1 elements of the plan's C row-pointer type;
 *                  written with the exclusive scan of the row counts.
 *   c_nnz       -- host, required: receives nnz(C).
 *   n_products  -- host, optional: receives the number of partial products
 *                  (sum over i of sum over k in A_i of nnz(B_k)).
 *   workspace_bytes -- host, optional: device bytes the plan holds.
 * Blocks until c_nnz is known (the only host synchronisation of the pair).
 * Errors: INVALID_ARG (shapes, nulls, A.cols != B.rows), BAD_CSR (validate),
 * INDEX_OVERFLOW (c_row_ptr_type I32 and nnz(C) > INT32_MAX; c_row_ptr is then
 * unspecified), OUT_OF_MEMORY, HIP.
 */
reap_status_t reap_spgemm_symbolic(reap_spgemm_t plan, const reap_csr_t* A, const reap_csr_t* B,
                                   void* c_row_ptr, int64_t* c_nnz, int64_t* n_products,
                                   size_t* workspace_bytes);

/*
 * Allocation-free variant of reap_spgemm_symbolic, for callers that cannot
 * allocate memory during the call: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  Same arguments and
 * results as reap_spgemm_symbolic for one product (no workspace_bytes), and
 * the numeric call that follows is unchanged.  The plan's workspace for this
 * product (counters, per-row classes, counts and column windows, the
 * long-row list, scan partials, and for FP32 products the long-row FP64
 * accumulators when a long row reads a B row out of column order) is placed
 * in a static device array of REAP_NOALLOC_SCRATCH_BYTES (64 MiB) instead of
 * the plan's own allocation: about 29 bytes per row of A, so products up to
 * roughly 2.3 million rows.  Larger products return REAP_ERR_TOO_LARGE
 * before any device work.  The call and the numeric call after it launch
 * their kernels directly (not through captured graphs, whatever the plan's
 * `graph` option) and call no hipMalloc, hipFree or other allocating
 * routine; the plan itself must have been created beforehand.
 * Sharing: each device holds one such array from the plan creation that
 * first looked it up until the process ends, and every allocation-free call
 * on that device uses it, keeping the last call's contents (the counters are
 * cleared at the start of each call).  Calls that overlap on one device
 * race, and so does a numeric call whose allocation-free symbolic call was
 * followed by another one on the same device before it: serialise them (one
 * stream, or events).  A later reap_spgemm_symbolic on the plan returns it to
 * its own workspace.
 * Errors: as reap_spgemm_symbolic, plus TOO_LARGE (never OUT_OF_MEMORY).
 */
reap_status_t reap_spgemm_symbolic_noalloc(reap_spgemm_t plan, const reap_csr_t* A, const reap_csr_t* B,
                                           void* c_row_ptr, int64_t* c_nnz, int64_t* n_products);

/*
 * Numeric pass: multiply, accumulate and write C (Algorithm 1's products,
 * sort and merge).  A and B must have the same shapes and patterns as in the
 * preceding symbolic call on this plan (values may differ); c_row_ptr is the
 * array symbolic wrote.  c_col_idx and c_values are device arrays of nnz(C)
 * elements.  FP32 operands are multiplied and summed in FP64 and rounded once
 * on write.  Asynchronous on the plan's stream; a kernel fault surfaces as
 * REAP_ERR_HIP at a later call or stream synchronisation.
 * Errors: INVALID_ARG, STATE (no symbolic, or shapes differ from it), HIP.
 */
reap_status_t reap_spgemm_numeric(reap_spgemm_t plan, const reap_csr_t* A, const reap_csr_t* B,
                                  const void* c_row_ptr, int32_t* c_col_idx, void* c_values);

/*
 * Batched symbolic pass: `count` independent products C_q = A_q * B_q in one
 * launch per kernel (every product's rows share the wavefront kernels' grid;
 * the long rows of all products share one list).  A, B: host arrays of
 * `count` descriptors, all with the same row-pointer type; c_row_ptr: host
 * array of `count` device pointers (A_q.rows + 1 elements each).  c_nnz
 * (required) and n_products (optional): host arrays of `count` entries.
 * The per-product semantics are those of reap_spgemm_symbolic; a plan holds
 * the state of its last call, single or batched.  Blocks until every nnz(C_q)
 * is known.  Errors: as reap_spgemm_symbolic (INDEX_OVERFLOW if any product
 * overflows an int32 C row pointer).
 */
reap_status_t reap_spgemm_batch_symbolic(reap_spgemm_t plan, int64_t count, const reap_csr_t* A,
                                         const reap_csr_t* B, void* const* c_row_ptr, int64_t* c_nnz,
                                         int64_t* n_products, size_t* workspace_bytes);

/*
 * Batched numeric pass after reap_spgemm_batch_symbolic with the same count,
 * shapes and patterns (values may differ).  c_row_ptr, c_col_idx, c_values:
 * host arrays of `count` device pointers (nnz(C_q) column indices and values
 * each).  Asynchronous.  Errors: as reap_spgemm_numeric.
 */
reap_status_t reap_spgemm_batch_numeric(reap_spgemm_t plan, int64_t count, const reap_csr_t* A,
                                        const reap_csr_t* B, const void* const* c_row_ptr,
                                        int32_t* const* c_col_idx, void* const* c_values);

/*
 * Device memory the plan will hold once a (batched) symbolic call on these
 * operands has returned: its workspace, which only grows, plus the FP32
 * long-row accumulators counted at their largest (one window segment of the
 * widest B per compute unit).  A caller that admits work by its device
 * footprint adds this to C's arrays before calling symbolic (the serving
 * loop's admission, the analog of the paper's coarse-grained overlap of
 * CPU and accelerator work in Section II).  count, A, B as in
 * reap_spgemm_batch_symbolic (count = 1 for one product).  Host-only: no
 * device work, no allocation.  Errors: INVALID_ARG.
 */
reap_status_t reap_spgemm_workspace_query(reap_spgemm_t plan, int64_t count, const reap_csr_t* A,
                                          const reap_csr_t* B, size_t* bytes);

/*
 * Device transpose: T = A^T in CSR (A's compressed-column form), so that a
 * product A * A^T needs only A on the device.  T has A.cols rows and A.cols
 * + 1 row pointers of A's row-pointer type (t_row_ptr, device); t_col_idx
 * (int32) and t_values (the plan's dtype) are device arrays of A.nnz
 * elements.  Inside a row of T the entries keep A's row order, so T's
 * columns are ascending whenever A's rows are stored in order (every
 * canonical CSR input); entries of A that repeat a position stay separate
 * and keep their order.  The paper's row-reorganised input format reads the
 * second operand by columns (Section III-A); this is that change of
 * direction done on the device.  Asynchronous on the plan's stream; the plan
 * keeps scratch of about 20 bytes per entry of A.
 * Errors: INVALID_ARG (nulls, A.nnz or A.rows above INT32_MAX), OUT_OF_MEMORY, HIP.
 */
reap_status_t reap_csr_transpose(reap_spgemm_t plan, const reap_csr_t* A, void* t_row_ptr,
                                 int32_t* t_col_idx, void* t_values);

/* Release the plan's workspace and the plan (NULL is accepted). */
reap_status_t reap_spgemm_destroy(reap_spgemm_t plan);

/*
 * Row classes of the last symbolic pass and, after a numeric call, the long-row
 * segment counts (reading those synchronises the plan's stream).
 * Errors: INVALID_ARG, STATE, HIP.
 */
reap_status_t reap_spgemm_bin_stats(reap_spgemm_t plan, reap_bin_stats_t* out);

/*
 * Device milliseconds per call of each phase, averaged over the calls made
 * since the plan was created or last reset, when the plan was created with
 * opts->profile set (HIP events recorded on the plan's stream around each
 * phase; no extra host synchronisation is added to symbolic or numeric).
 *   out[0] symbolic kernels (row product counts, binning, per-row column
 *          counts), out[1] scan, out[2] numeric wavefront-bitmap kernels,
 *   out[3] numeric wavefront-hash kernel, out[4] numeric workgroup kernel,
 *   out[5] whole numeric call, out[6] 0, out[7] number of numeric calls
 *   averaged.  A phase that did not run reads 0.
 *   n = capacity of out (<= 8 is read).
 * Synchronises the plan's stream.  Errors: INVALID_ARG, STATE (no profile).
 */
reap_status_t reap_spgemm_phase_times(reap_spgemm_t plan, float* out, int n);

/* Clears the accumulated phase times.  Errors: INVALID_ARG, STATE (no profile). */
reap_status_t reap_spgemm_phase_reset(reap_spgemm_t plan);

/* Static description of a status code. */
const char* reap_status_string(reap_status_t s);

/* Library version, "major.minor.patch". */
const char* reap_version(void);

#ifdef __cplusplus
}
#endif

#endif /* REAP_SPGEMM_H */
