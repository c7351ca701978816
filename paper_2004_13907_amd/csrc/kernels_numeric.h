// Numeric pass: partial products a_ik * b_kj, their accumulation by column and
// the ascending-column write of each row of C (the multiply, sort and merge
// steps of the paper's Algorithm 1).  Sorting is replaced by ranking: a bitmap
// over the row's column window, with a prefix count per 32-bit word, gives
// every column its position in the sorted row directly.  This file holds the
// argument block; the wavefront kernels are in kernels_wave.h and the
// long-row kernels in kernels_long.h.
#pragma once
#include "device_utils.h"
#include "kernels_symbolic.h"
#include "spgemm_common.h"

namespace reap {

template <typename T, typename IdxT, typename IdxC>
struct NumArgs {
    int64_t m;
    int64_t n;
    int64_t k;                 // rows of B (B's row pointer has k + 1 entries)
    gptr<const IdxT> a_rp;
    gptr<const int32_t> a_col;
    gptr<const T> a_val;
    gptr<const IdxT> b_rp;
    gptr<const int32_t> b_col;
    gptr<const T> b_val;
    gptr<const IdxC> c_rp;
    gptr<int32_t> c_col;
    gptr<T> c_val;
    gptr<const uint8_t> cls;
    gptr<const int2> win;
    gptr<Counters> ctr;
    gptr<double> gvals;     // per-workgroup FP64 accumulators of long rows with FP32 output
    int64_t gvals_stride;   // doubles per workgroup slot
    Thresholds th;
};

}  // namespace reap
