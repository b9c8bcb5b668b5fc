// Deterministic reductions for wave64 devices without grid-wide fences.
//
// A reducing kernel writes one partial per block (block_partials).  The total
// is formed later, after a kernel boundary has made the partials visible: either
// redundantly by every block of the consuming kernel (sum_parts, all blocks
// read the same partials in the same order and get the same bits), or by a
// one-block finishing kernel.  The summation order depends only on the launch
// shape, never on timing, so results are bitwise reproducible.
#pragma once

#include "vag_internal.h"

namespace vag {

// The workgroups of a launch are dealt to the 8 XCDs in turn (block b to XCD
// b mod 8), each XCD with its own L2.  xcd_block() renumbers the blocks so
// that every XCD receives one contiguous run of block indices: neighbouring
// rows then share an L2, and the gathers of a row's neighbours (and of an
// aggregate's members) hit lines that the same XCD has already fetched.  A
// bijection of [0, gridDim.x).
__device__ inline unsigned xcd_block() {
    const unsigned nb = gridDim.x, b = blockIdx.x, q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

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

// Reduces NV values per thread over the block; results valid in every thread.
template <class Op, int NV, int NT>
__device__ inline void block_reduce(double (&v)[NV]) {
    __shared__ double lds[NV][NT / 64];
    __shared__ double res[NV];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = wave_reduce<Op>(v[k]);
        if (lane == 0) lds[k][w] = t;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = lds[threadIdx.x][0];
        for (int i = 1; i < NT / 64; ++i) t = Op::op(t, lds[threadIdx.x][i]);
        res[threadIdx.x] = t;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = res[k];
    __syncthreads();
}

// Writes the block's reduction of NV values to parts[k * stride + blockIdx.x].
template <class Op, int NV, int NT>
__device__ inline void block_partials(double (&v)[NV], double *parts, int stride) {
    block_reduce<Op, NV, NT>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) parts[(size_t)k * stride + blockIdx.x] = v[k];
    }
}

// Total of nparts partials, identical in every thread of every block.
template <class Op, int NT>
__device__ inline double sum_parts(const double *parts, int nparts) {
    double v[1] = {Op::id()};
    for (int i = threadIdx.x; i < nparts; i += NT) v[0] = Op::op(v[0], parts[i]);
    block_reduce<Op, 1, NT>(v);
    return v[0];
}

inline unsigned reduce_grid(int64_t n_items, int threads) {
    int64_t b = (n_items + threads - 1) / threads;
    if (b > kReduceBlocks) b = kReduceBlocks;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// one-block kernel: out[k] = Op-total of parts[k*stride .. k*stride+nparts)
void launch_finalize_sum(hipStream_t s, const double *parts, int stride, int nparts, int nv, double *out);
void launch_finalize_min(hipStream_t s, const double *parts, int stride, int nparts, int nv, double *out);

}  // namespace vag
