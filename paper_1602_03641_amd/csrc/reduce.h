// Deterministic grid-wide reductions for wave64 devices.
//
// Each block reduces its threads' values (wave shuffles, then LDS across the
// block's waves), writes one partial per block, and the last block to finish
// (ticket counter) sums the partials in block order.  The summation order
// depends only on the launch shape, never on timing, so results are bitwise
// reproducible run to run.
#pragma once

#include "vag_internal.h"

namespace vag {

struct OpSum {
    __device__ static double id() { return 0.0; }
    __device__ static double op(double a, double b) { return a + b; }
};
struct OpMin {
    __device__ static double id() { return __builtin_inf(); }
    __device__ static double op(double a, double b) { return a < b ? a : b; }
};

template <class Op>
__device__ inline double wave_reduce(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = Op::op(v, __shfl_down(v, o, 64));
    return v;  // valid in lane 0
}

// Reduces NV values per thread over the block; results valid in thread 0.
template <class Op, int NV, int NT>
__device__ inline void block_reduce(double (&v)[NV]) {
    __shared__ double lds[NV][NT / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = wave_reduce<Op>(v[k]);
        if (lane == 0) lds[k][w] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double t = lds[k][0];
            for (int i = 1; i < NT / 64; ++i) t = Op::op(t, lds[k][i]);
            v[k] = t;
        }
    }
    __syncthreads();
}

// Grid reduction; returns true in the block that holds the final values
// (valid in its thread 0).  Uses ticket slot `slot`; resets it for reuse.
template <class Op, int NV, int NT>
__device__ inline bool grid_reduce(double (&v)[NV], ReduceScratch rs, int slot) {
    __shared__ bool is_last;
    block_reduce<Op, NV, NT>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k)
            __hip_atomic_store(&rs.parts[(size_t)blockIdx.x * NV + k], v[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned t = atomicAdd(&rs.ticket[slot], 1u);
        is_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = Op::id();
    for (unsigned i = threadIdx.x; i < gridDim.x; i += NT)
#pragma unroll
        for (int k = 0; k < NV; ++k)
            acc[k] = Op::op(acc[k], __hip_atomic_load(&rs.parts[(size_t)i * NV + k], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT));
    block_reduce<Op, NV, NT>(acc);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = acc[k];
        rs.ticket[slot] = 0u;
    }
    return true;
}

inline unsigned reduce_grid(int64_t n_items, int threads) {
    int64_t b = (n_items + threads - 1) / threads;
    if (b > kReduceBlocks) b = kReduceBlocks;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace vag
