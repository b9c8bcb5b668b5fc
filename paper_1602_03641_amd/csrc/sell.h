// Row kernels on sliced ELL (64-row slices, column-major inside a slice).
#pragma once

#include "vag_internal.h"

namespace vag {

// sum over the levels k of the slice of A[row, k] * f(col(k)), kChains
// independent accumulation chains (chain c takes the levels k = c mod
// kChains) so that several gathers are in flight per lane.  The summation
// order is fixed.  The level index k, the slice's start b0 and its width w are
// the same for every lane (the wavefront holds the slice's 64 rows), so the
// loop control and the per-level column bases stay in scalar registers.
constexpr int kChains = 4;
template <bool NT, class V, class Acc, class F, class Col>
__device__ inline void sell_row_chains(const Sell<V> &A, int64_t b0, int32_t w, int lane, Acc *s, F f, Col col) {
    int32_t k = 0;
    for (; k + kChains <= w; k += kChains) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            const int64_t p = b0 + 64 * (int64_t)(k + c) + lane;
            s[c] += (Acc)ld_matrix<NT>(&A.val[p]) * f(col(p, k + c));
        }
    }
#pragma unroll
    for (int c = 0; c < kChains - 1; ++c)
        if (k + c < w) {
            const int64_t p = b0 + 64 * (int64_t)(k + c) + lane;
            s[c] += (Acc)ld_matrix<NT>(&A.val[p]) * f(col(p, k + c));
        }
}

// Row `row` of A applied to f.  Every caller runs one thread per row in blocks
// of whole wavefronts, so the active lanes of a wavefront are rows of one
// slice and lane = row mod 64.
template <class V, class Acc, class F>
__device__ inline Acc sell_row_apply(const Sell<V> &A, int32_t row, F f) {
    const int32_t sl = __builtin_amdgcn_readfirstlane(row >> 6);
    const int64_t b0 = A.ptr[sl], b1 = A.ptr[sl + 1];
    const int32_t w = (int32_t)((b1 - b0) >> 6);
    const int lane = row & 63;
    Acc s[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) s[c] = 0;
    // 16-bit columns where the slice's first level has a base: level k's base
    // is cbase[b0 / 64 + k]
    const int32_t *cb = A.col16 && w > 0 && A.cbase[b0 >> 6] >= 0 ? A.cbase + (b0 >> 6) : nullptr;
    if (cb) {
        if (A.nt)
            sell_row_chains<true, V, Acc>(A, b0, w, lane, s, f, [&](int64_t p, int32_t k) {
                return cb[k] + (int32_t)ld_matrix<true>(&A.col16[p]);
            });
        else
            sell_row_chains<false, V, Acc>(A, b0, w, lane, s, f,
                                           [&](int64_t p, int32_t k) { return cb[k] + (int32_t)A.col16[p]; });
    } else {
        if (A.nt)
            sell_row_chains<true, V, Acc>(A, b0, w, lane, s, f,
                                          [&](int64_t p, int32_t) { return ld_matrix<true>(&A.col[p]); });
        else
            sell_row_chains<false, V, Acc>(A, b0, w, lane, s, f, [&](int64_t p, int32_t) { return A.col[p]; });
    }
#pragma unroll
    for (int w2 = kChains / 2; w2 > 0; w2 >>= 1)
#pragma unroll
        for (int c = 0; c < w2; ++c) s[c] += s[c + w2];
    if (A.dg) s[0] += (Acc)A.dg[row] * f(row);
    return s[0];
}

}  // namespace vag
