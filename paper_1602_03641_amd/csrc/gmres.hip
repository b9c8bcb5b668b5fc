// Kernels of restarted flexible GMRES with classical Gram-Schmidt
// applied twice (CGS2).  The Krylov basis V is stored as (m+1) vectors of
// length ld, one after the other.  Every reduction goes through per-block
// partials summed in a fixed order (deterministic); the Hessenberg column is
// reduced on the device and read by the host once per iteration.
#include "reduce.h"
#include "sell.h"

namespace vag {

namespace {

constexpr int kT = 256;
constexpr int kDots = 8;  // basis vectors per block in the multi-dot kernel

#define GS(i, n) \
    for (int64_t i = (int64_t)xcd_block() * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

template <class V, class T>
__global__ __launch_bounds__(kT) void gm_spmv_kernel(Sell<V> A, const T *__restrict__ x, T *__restrict__ y) {
    GS(i, A.n) y[i] = (T)sell_row_apply<V, double>(A, (int32_t)i, [&](int32_t j) { return (double)x[j]; });
}

// parts[(c*kDots + i) * G + bx] = partial of <V_{c*kDots+i}, w> over block bx
template <class T>
__global__ __launch_bounds__(kT) void gm_multidot_kernel(int32_t n, int k, const T *__restrict__ V, int64_t ld,
                                                         const T *__restrict__ w, double *__restrict__ parts) {
    const int c0 = blockIdx.y * kDots;
    double v[kDots];
#pragma unroll
    for (int i = 0; i < kDots; ++i) v[i] = 0.0;
    GS(r, n) {
        const double wr = (double)w[r];
#pragma unroll
        for (int i = 0; i < kDots; ++i)
            if (c0 + i < k) v[i] += (double)V[(int64_t)(c0 + i) * ld + r] * wr;
    }
    block_reduce<OpSum, kDots, kT>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kDots; ++i)
            if (c0 + i < k) parts[(size_t)(c0 + i) * gridDim.x + blockIdx.x] = v[i];
    }
}

// h[i] = sum of the G partials of dot i (one block per dot)
__global__ __launch_bounds__(kT) void gm_hreduce_kernel(const double *__restrict__ parts, int G,
                                                        double *__restrict__ h) {
    const double t = sum_parts<OpSum, kT>(parts + (size_t)blockIdx.x * G, G);
    if (threadIdx.x == 0) h[blockIdx.x] = t;
}

// w -= sum_{i<k} h[i] V_i, and partials of ||w||^2
template <class T>
__global__ __launch_bounds__(kT) void gm_multiaxpy_kernel(int32_t n, int k, const T *__restrict__ V, int64_t ld,
                                                          const double *__restrict__ h, T *__restrict__ w,
                                                          double *__restrict__ parts) {
    double v[1] = {0.0};
    GS(r, n) {
        double t = (double)w[r];
        for (int i = 0; i < k; ++i) t -= h[i] * (double)V[(int64_t)i * ld + r];
        const T tw = (T)t;
        w[r] = tw;
        v[0] += (double)tw * (double)tw;
    }
    block_partials<OpSum, 1, kT>(v, parts, gridDim.x);
}

// out = s * (the vector w), s = 1 / sqrt(sum of the partials); hn = sqrt(...)
template <class T>
__global__ __launch_bounds__(kT) void gm_normalize_kernel(int32_t n, const double *__restrict__ parts, int G,
                                                          const T *__restrict__ w, T *__restrict__ out,
                                                          double *__restrict__ hn) {
    const double nrm = sqrt(sum_parts<OpSum, kT>(parts, G));
    if (blockIdx.x == 0 && threadIdx.x == 0) *hn = nrm;
    const double s = nrm > 0.0 ? 1.0 / nrm : 0.0;
    GS(r, n) out[r] = (T)(s * (double)w[r]);
}

// t = sum_{i<k} y[i] V_i
template <class T>
__global__ __launch_bounds__(kT) void gm_combine_kernel(int32_t n, int k, const T *__restrict__ V, int64_t ld,
                                                        const double *__restrict__ y, T *__restrict__ t) {
    GS(r, n) {
        double s = 0.0;
        for (int i = 0; i < k; ++i) s += y[i] * (double)V[(int64_t)i * ld + r];
        t[r] = (T)s;
    }
}

// x += z
template <class T>
__global__ __launch_bounds__(kT) void gm_add_kernel(int32_t n, const T *__restrict__ z, T *__restrict__ x) {
    GS(r, n) x[r] = (T)((double)x[r] + (double)z[r]);
}

// r = b - A x, partials of ||r||^2
template <class V, class T>
__global__ __launch_bounds__(kT) void gm_residual_kernel(Sell<V> A, const T *__restrict__ b, const T *__restrict__ x,
                                                         T *__restrict__ r, double *__restrict__ parts) {
    double v[1] = {0.0};
    GS(i, A.n) {
        const double t =
            (double)b[i] - sell_row_apply<V, double>(A, (int32_t)i, [&](int32_t j) { return (double)x[j]; });
        const T tr = (T)t;
        r[i] = tr;
        v[0] += (double)tr * (double)tr;
    }
    block_partials<OpSum, 1, kT>(v, parts, gridDim.x);
}

}  // namespace

int gmres_grid(int64_t n) { return (int)reduce_grid(n, kT); }

template <class V, class T>
void launch_gm_spmv(hipStream_t s, Sell<V> A, const T *x, T *y) {
    if (A.n <= 0) return;
    hipLaunchKernelGGL((gm_spmv_kernel<V, T>), dim3(gmres_grid(A.n)), dim3(kT), 0, s, A, x, y);
    VAG_HIP(hipGetLastError());
}

template <class T>
void launch_gm_orthogonalize(hipStream_t s, int32_t n, int k, const T *V, int64_t ld, T *w, double *parts,
                             double *h, double *nparts) {
    const int G = gmres_grid(n);
    const dim3 grid(G, (k + kDots - 1) / kDots);
    hipLaunchKernelGGL((gm_multidot_kernel<T>), grid, dim3(kT), 0, s, n, k, V, ld, w, parts);
    VAG_HIP(hipGetLastError());
    hipLaunchKernelGGL(gm_hreduce_kernel, dim3(k), dim3(kT), 0, s, parts, G, h);
    VAG_HIP(hipGetLastError());
    hipLaunchKernelGGL((gm_multiaxpy_kernel<T>), dim3(G), dim3(kT), 0, s, n, k, V, ld, h, w, nparts);
    VAG_HIP(hipGetLastError());
}

template <class T>
void launch_gm_normalize(hipStream_t s, int32_t n, const double *nparts, const T *w, T *out, double *hn) {
    const int G = gmres_grid(n);
    hipLaunchKernelGGL((gm_normalize_kernel<T>), dim3(G), dim3(kT), 0, s, n, nparts, G, w, out, hn);
    VAG_HIP(hipGetLastError());
}

template <class T>
void launch_gm_combine(hipStream_t s, int32_t n, int k, const T *V, int64_t ld, const double *y, T *t) {
    hipLaunchKernelGGL((gm_combine_kernel<T>), dim3(gmres_grid(n)), dim3(kT), 0, s, n, k, V, ld, y, t);
    VAG_HIP(hipGetLastError());
}

template <class T>
void launch_gm_add(hipStream_t s, int32_t n, const T *z, T *x) {
    hipLaunchKernelGGL((gm_add_kernel<T>), dim3(gmres_grid(n)), dim3(kT), 0, s, n, z, x);
    VAG_HIP(hipGetLastError());
}

template <class V, class T>
void launch_gm_residual(hipStream_t s, Sell<V> A, const T *b, const T *x, T *r, double *nparts) {
    hipLaunchKernelGGL((gm_residual_kernel<V, T>), dim3(gmres_grid(A.n)), dim3(kT), 0, s, A, b, x, r, nparts);
    VAG_HIP(hipGetLastError());
}

#define GM_INST(T)                                                                                               \
    template void launch_gm_spmv<T, T>(hipStream_t, Sell<T>, const T *, T *);                                    \
    template void launch_gm_orthogonalize<T>(hipStream_t, int32_t, int, const T *, int64_t, T *, double *,      \
                                             double *, double *);                                               \
    template void launch_gm_normalize<T>(hipStream_t, int32_t, const double *, const T *, T *, double *);        \
    template void launch_gm_combine<T>(hipStream_t, int32_t, int, const T *, int64_t, const double *, T *);      \
    template void launch_gm_add<T>(hipStream_t, int32_t, const T *, T *);                                        \
    template void launch_gm_residual<T, T>(hipStream_t, Sell<T>, const T *, const T *, T *, double *);
GM_INST(double)
GM_INST(float)

}  // namespace vag
