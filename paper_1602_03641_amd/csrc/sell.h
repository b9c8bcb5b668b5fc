// Row kernels on sliced ELL (64-row slices, column-major inside a slice).
#pragma once

#include "vag_internal.h"

namespace vag {

// sum_q A[row, q] * f(col_q), kChains independent accumulation chains so that
// several gathers are in flight per lane.  The summation order is fixed.
constexpr int kChains = 4;
template <bool NT, class V, class Acc, class F, class Col>
__device__ inline void sell_row_chains(const Sell<V> &A, int64_t q, int64_t b1, Acc *s, F f, Col col) {
    for (; q + (kChains - 1) * 64 < b1; q += kChains * 64) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) s[c] += (Acc)ld_matrix<NT>(&A.val[q + c * 64]) * f(col(q + c * 64));
    }
#pragma unroll
    for (int c = 0; c < kChains - 1; ++c)
        if (q + c * 64 < b1) s[c] += (Acc)ld_matrix<NT>(&A.val[q + c * 64]) * f(col(q + c * 64));
}

template <class V, class Acc, class F>
__device__ inline Acc sell_row_apply(const Sell<V> &A, int32_t row, F f) {
    const int64_t b0 = A.ptr[row >> 6], b1 = A.ptr[(row >> 6) + 1];
    const int64_t q = b0 + (row & 63);
    Acc s[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) s[c] = 0;
    // the slice's first group says whether its columns are 16-bit; p / 64 is
    // the same for every lane of the wavefront (the slice's level)
    const int32_t cb = A.col16 && b1 > b0 ? A.cbase[b0 >> 6] : -1;
    if (cb >= 0) {
        if (A.nt)
            sell_row_chains<true, V, Acc>(A, q, b1, s, f, [&](int64_t p) {
                return A.cbase[p >> 6] + (int32_t)ld_matrix<true>(&A.col16[p]);
            });
        else
            sell_row_chains<false, V, Acc>(A, q, b1, s, f, [&](int64_t p) { return A.cbase[p >> 6] + (int32_t)A.col16[p]; });
    } else {
        if (A.nt)
            sell_row_chains<true, V, Acc>(A, q, b1, s, f, [&](int64_t p) { return ld_matrix<true>(&A.col[p]); });
        else
            sell_row_chains<false, V, Acc>(A, q, b1, s, f, [&](int64_t p) { return A.col[p]; });
    }
#pragma unroll
    for (int w = kChains / 2; w > 0; w >>= 1)
#pragma unroll
        for (int c = 0; c < w; ++c) s[c] += s[c + w];
    if (A.dg) s[0] += (Acc)A.dg[row] * f(row);
    return s[0];
}

}  // namespace vag
