// Row kernels on sliced ELL (64-row slices, column-major inside a slice).
#pragma once

#include "vag_internal.h"

namespace vag {

// sum_q A[row, q] * f(col_q), four independent accumulation chains so that
// several gathers are in flight per lane.  The summation order is fixed.
template <class V, class Acc, class F>
__device__ inline Acc sell_row_apply(const Sell<V> &A, int32_t row, F f) {
    const int64_t b1 = A.ptr[(row >> 6) + 1];
    int64_t q = A.ptr[row >> 6] + (row & 63);
    Acc s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (; q + 192 < b1; q += 256) {
        s0 += (Acc)A.val[q] * f(A.col[q]);
        s1 += (Acc)A.val[q + 64] * f(A.col[q + 64]);
        s2 += (Acc)A.val[q + 128] * f(A.col[q + 128]);
        s3 += (Acc)A.val[q + 192] * f(A.col[q + 192]);
    }
    for (; q < b1; q += 64) s0 += (Acc)A.val[q] * f(A.col[q]);
    return (s0 + s1) + (s2 + s3);
}

}  // namespace vag
