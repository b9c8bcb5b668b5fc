// Krylov kernels for the SPD system of eq eqschur.
//
// SpMV on sliced ELL: one row per lane, a wavefront = one 64-row slice, so
// every value/column load of a wave is one contiguous 512/256-byte segment.
//
// Preconditioned CG keeps its scalars on the device.  An iteration k is
//   direction(k): convergence test on ||r_k||^2, p = z + beta p
//   spmv:         q = A p, partials of p.q
//   update(k):    alpha = (r.z)/(p.q), x += alpha p, r -= alpha q,
//                 z = M^-1 r, partials of r.z and r.r
// Each kernel forms the totals it needs from the previous kernels' block
// partials (redundantly in every block, in a fixed order), so no grid-wide
// fence or atomic is needed and the arithmetic is reproducible bit for bit.
// Partials are double-buffered by iteration parity.  Once the test succeeds the
// `done` flag makes every later kernel return at once: the host queues many
// iterations and reads the flag only now and then.
#include "reduce.h"
#include "sell.h"

namespace vag {

constexpr int kThreads = kKrylovThreads;

int pcg_grid(int64_t n) { return (int)reduce_grid(n, kThreads); }

template <class V, class X>
__device__ inline double sell_row(const Sell<V> &A, const X *__restrict__ x, int32_t row) {
    return sell_row_apply<V, double>(A, row, [&](int32_t j) { return (double)x[j]; });
}

#define GRID_STRIDE(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

__global__ __launch_bounds__(kThreads) void spmv_kernel(Sell<double> A, const double *__restrict__ x,
                                                        double *__restrict__ y) {
    GRID_STRIDE(i, A.n) y[i] = sell_row(A, x, (int32_t)i);
}

__global__ __launch_bounds__(kThreads) void residual_kernel(Sell<double> A, const double *__restrict__ x,
                                                            const double *__restrict__ b, double *__restrict__ r,
                                                            double *__restrict__ parts) {
    double v[2] = {0.0, 0.0};
    GRID_STRIDE(i, A.n) {
        const double t = b[i] - sell_row(A, x, (int32_t)i);
        r[i] = t;
        v[0] += t * t;
        v[1] += b[i] * b[i];
    }
    block_partials<OpSum, 2, kThreads>(v, parts, gridDim.x);
}

template <class Op>
__global__ __launch_bounds__(kThreads) void finalize_kernel(const double *__restrict__ parts, int stride, int nparts,
                                                            int nv, double *__restrict__ out) {
    for (int k = 0; k < nv; ++k) {
        const double t = sum_parts<Op, kThreads>(parts + (size_t)k * stride, nparts);
        if (threadIdx.x == 0) out[k] = t;
    }
}

__global__ __launch_bounds__(kThreads) void fill_kernel(int64_t n, double v, double *__restrict__ x) {
    GRID_STRIDE(i, n) x[i] = v;
}
__global__ __launch_bounds__(kThreads) void copy_kernel(int64_t n, const double *__restrict__ s,
                                                        double *__restrict__ d) {
    GRID_STRIDE(i, n) d[i] = s[i];
}
__global__ __launch_bounds__(kThreads) void jacobi_kernel(int64_t n, const double *__restrict__ dinv,
                                                          const double *__restrict__ r, double *__restrict__ z) {
    GRID_STRIDE(i, n) z[i] = dinv[i] * r[i];
}

// ---------------------------------------------------------------------------
// preconditioned CG, x0 = 0
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void pcg_init_kernel(int32_t n, const double *__restrict__ b,
                                                            const double *__restrict__ dinv,
                                                            double *__restrict__ x, double *__restrict__ r,
                                                            double *__restrict__ z, PcgParts P) {
    double v[2] = {0.0, 0.0};
    GRID_STRIDE(i, n) {
        const double bi = b[i];
        x[i] = 0.0;
        r[i] = bi;
        if (dinv) {
            const double zi = dinv[i] * bi;
            z[i] = zi;
            v[0] += bi * zi;
        }
        v[1] += bi * bi;
    }
    block_reduce<OpSum, 2, kThreads>(v);
    if (threadIdx.x == 0) {
        if (dinv) P.rz(-1)[blockIdx.x] = v[0];
        P.rr(-1)[blockIdx.x] = v[1];
    }
}

__global__ __launch_bounds__(kThreads) void pcg_start_kernel(PcgParts P, PcgState *st, double rtol, int k0) {
    const double bb = sum_parts<OpSum, kThreads>(P.rr(k0 - 1), P.G);
    if (threadIdx.x == 0) {
        st->bnorm2 = bb;
        st->tol2 = rtol * rtol * bb;
        st->rr = bb;
        st->iter = k0;
        st->done = (bb == 0.0);
        st->converged = (bb == 0.0);
    }
}

template <class T>
__global__ __launch_bounds__(kThreads) void pcg_direction_kernel(int32_t n, int k, int k0, const T *__restrict__ z,
                                                                 T *__restrict__ p, PcgParts P, PcgState *st,
                                                                 int update, int flexible) {
    if (st->done) return;
    const double rr = sum_parts<OpSum, kThreads>(P.rr(k - 1), P.G);
    if (rr <= st->tol2) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->done = 1;
            st->converged = 1;
            st->rr = rr;
        }
        return;
    }
    if (!update) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->rr = rr;
        return;
    }
    double beta = 0.0;
    if (k > k0) {
        if (flexible)
            beta = -sum_parts<OpSum, kThreads>(P.zq(), P.G) / sum_parts<OpSum, kThreads>(P.pq(), P.G);
        else
            beta = sum_parts<OpSum, kThreads>(P.rz(k - 1), P.G) / sum_parts<OpSum, kThreads>(P.rz(k), P.G);
    }
    if (k == k0) {
        GRID_STRIDE(i, n) p[i] = z[i];
    } else {
        const T b = (T)beta;
        GRID_STRIDE(i, n) p[i] = z[i] + b * p[i];
    }
}

template <class V, class T>
__global__ __launch_bounds__(kThreads) void pcg_spmv_kernel(Sell<V> A, const T *__restrict__ p, T *__restrict__ q,
                                                            PcgParts P, const PcgState *st) {
    if (st->done) return;
    double v[1] = {0.0};
    GRID_STRIDE(i, A.n) {
        const double s = sell_row(A, p, (int32_t)i);
        q[i] = (T)s;
        v[0] += (double)p[i] * s;
    }
    block_partials<OpSum, 1, kThreads>(v, P.pq(), P.G);
}

__global__ __launch_bounds__(kThreads) void pcg_update_kernel(int32_t n, int k, double *__restrict__ x,
                                                              double *__restrict__ r, double *__restrict__ z,
                                                              const double *__restrict__ p,
                                                              const double *__restrict__ q,
                                                              const double *__restrict__ dinv, PcgParts P,
                                                              PcgState *st) {
    if (st->done) return;
    const double alpha = sum_parts<OpSum, kThreads>(P.rz(k - 1), P.G) / sum_parts<OpSum, kThreads>(P.pq(), P.G);
    double v[2] = {0.0, 0.0};
    GRID_STRIDE(i, n) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        const double zi = dinv[i] * ri;
        r[i] = ri;
        z[i] = zi;
        v[0] += ri * zi;
        v[1] += ri * ri;
    }
    block_reduce<OpSum, 2, kThreads>(v);
    if (threadIdx.x == 0) {
        P.rz(k)[blockIdx.x] = v[0];
        P.rr(k)[blockIdx.x] = v[1];
        if (blockIdx.x == 0) st->iter = k + 1;
    }
}

template <class T>
__global__ __launch_bounds__(kThreads) void pcg_update_xr_kernel(int32_t n, int k, T *__restrict__ x,
                                                                 T *__restrict__ r, const T *__restrict__ p,
                                                                 const T *__restrict__ q, PcgParts P, PcgState *st,
                                                                 const T *__restrict__ dinv, T *__restrict__ x0) {
    if (st->done) return;
    const double alpha = sum_parts<OpSum, kThreads>(P.rz(k - 1), P.G) / sum_parts<OpSum, kThreads>(P.pq(), P.G);
    const T a = (T)alpha;
    double v[1] = {0.0};
    GRID_STRIDE(i, n) {
        x[i] += a * p[i];
        const T ri = r[i] - a * q[i];
        r[i] = ri;
        if (x0) x0[i] = dinv[i] * ri;  // first smoothing iterate of the preconditioner
        v[0] += (double)ri * (double)ri;
    }
    block_reduce<OpSum, 1, kThreads>(v);
    if (threadIdx.x == 0) {
        P.rr(k)[blockIdx.x] = v[0];
        if (blockIdx.x == 0) st->iter = k + 1;
    }
}

template <class T>
__global__ __launch_bounds__(kThreads) void pcg_dot_rz_kernel(int32_t n, int k, const T *__restrict__ r,
                                                              const T *__restrict__ z, PcgParts P,
                                                              const PcgState *st) {
    if (st && st->done) return;
    double v[1] = {0.0};
    GRID_STRIDE(i, n) v[0] += (double)r[i] * (double)z[i];
    block_reduce<OpSum, 1, kThreads>(v);
    if (threadIdx.x == 0) P.rz(k)[blockIdx.x] = v[0];
}

// warm start at iteration k0: r = b - A x, partials rr(k0-1); with dinv also
// z = D^-1 r and partials rz(k0-1)
__global__ __launch_bounds__(kThreads) void pcg_init_warm_kernel(Sell<double> A, int k0, const double *__restrict__ b,
                                                                 const double *__restrict__ x, double *__restrict__ r,
                                                                 const double *__restrict__ dinv, double *__restrict__ z,
                                                                 PcgParts P) {
    double v[2] = {0.0, 0.0};
    GRID_STRIDE(i, A.n) {
        const double ri = b[i] - sell_row(A, x, (int32_t)i);
        r[i] = ri;
        if (dinv) {
            const double zi = dinv[i] * ri;
            z[i] = zi;
            v[0] += ri * zi;
        }
        v[1] += ri * ri;
    }
    block_reduce<OpSum, 2, kThreads>(v);
    if (threadIdx.x == 0) {
        if (dinv) P.rz(k0 - 1)[blockIdx.x] = v[0];
        P.rr(k0 - 1)[blockIdx.x] = v[1];
    }
}

// x = 0, r = b (no preconditioner applied), partials of b.b
template <class T>
__global__ __launch_bounds__(kThreads) void pcg_init_plain_kernel(int32_t n, const T *__restrict__ b,
                                                                  T *__restrict__ x, T *__restrict__ r, PcgParts P) {
    double v[1] = {0.0};
    GRID_STRIDE(i, n) {
        x[i] = (T)0;
        r[i] = b[i];
        v[0] += (double)b[i] * (double)b[i];
    }
    block_reduce<OpSum, 1, kThreads>(v);
    if (threadIdx.x == 0) P.rr(-1)[blockIdx.x] = v[0];
}

// FP64 refinement around an FP32 inner solve:
//   partials of ||r||^2; r32 = r / ||r||; x += ||r|| d32
__global__ __launch_bounds__(kThreads) void norm2_kernel(int32_t n, const double *__restrict__ r,
                                                         double *__restrict__ parts) {
    double v[1] = {0.0};
    GRID_STRIDE(i, n) v[0] += r[i] * r[i];
    block_partials<OpSum, 1, kThreads>(v, parts, gridDim.x);
}
__global__ __launch_bounds__(kThreads) void normalize_to_float_kernel(int32_t n, const double *__restrict__ r,
                                                                      const double *__restrict__ nrm2,
                                                                      float *__restrict__ r32) {
    const double s = nrm2[0] > 0.0 ? 1.0 / sqrt(nrm2[0]) : 0.0;
    GRID_STRIDE(i, n) r32[i] = (float)(r[i] * s);
}
__global__ __launch_bounds__(kThreads) void correct_kernel(int32_t n, double *__restrict__ x,
                                                           const float *__restrict__ d32,
                                                           const double *__restrict__ nrm2) {
    const double s = sqrt(nrm2[0]);
    GRID_STRIDE(i, n) x[i] += s * (double)d32[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned vec_grid(int64_t n) { return reduce_grid(n, kThreads); }
#define LAUNCH(kern, grid, ...)                                                          \
    do {                                                                                 \
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), 0, s, __VA_ARGS__);         \
        VAG_HIP(hipGetLastError());                                                      \
    } while (0)

void launch_fill(hipStream_t s, int64_t n, double v, double *x) {
    if (n > 0) LAUNCH(fill_kernel, vec_grid(n), n, v, x);
}
void launch_copy(hipStream_t s, int64_t n, const double *src, double *dst) {
    if (n > 0) LAUNCH(copy_kernel, vec_grid(n), n, src, dst);
}
void launch_jacobi(hipStream_t s, int64_t n, const double *dinv, const double *r, double *z) {
    if (n > 0) LAUNCH(jacobi_kernel, vec_grid(n), n, dinv, r, z);
}
void launch_spmv(hipStream_t s, Sell<double> A, const double *x, double *y) {
    if (A.n > 0) LAUNCH(spmv_kernel, vec_grid(A.n), A, x, y);
}
void launch_finalize_sum(hipStream_t s, const double *parts, int stride, int nparts, int nv, double *out) {
    LAUNCH(finalize_kernel<OpSum>, 1, parts, stride, nparts, nv, out);
}
void launch_finalize_min(hipStream_t s, const double *parts, int stride, int nparts, int nv, double *out) {
    LAUNCH(finalize_kernel<OpMin>, 1, parts, stride, nparts, nv, out);
}
void launch_residual_norm(hipStream_t s, Sell<double> A, const double *x, const double *b, double *r,
                          double *parts, double *out2) {
    const unsigned g = vec_grid(A.n);
    LAUNCH(residual_kernel, g, A, x, b, r, parts);
    launch_finalize_sum(s, parts, (int)g, (int)g, 2, out2);
}
void launch_pcg_init(hipStream_t s, int32_t n, const double *b, const double *dinv, double *x, double *r,
                     double *z, PcgParts P) {
    LAUNCH(pcg_init_kernel, P.G, n, b, dinv, x, r, z, P);
}
void launch_pcg_start(hipStream_t s, PcgParts P, PcgState *st, double rtol, int k0) {
    LAUNCH(pcg_start_kernel, 1, P, st, rtol, k0);
}
void launch_pcg_init_warm(hipStream_t s, Sell<double> A, int k0, const double *b, const double *x, double *r,
                          const double *dinv, double *z, PcgParts P) {
    LAUNCH(pcg_init_warm_kernel, P.G, A, k0, b, x, r, dinv, z, P);
}
template <class T>
void launch_pcg_direction(hipStream_t s, int32_t n, int k, int k0, const T *z, T *p, PcgParts P, PcgState *st,
                          bool update, bool flexible) {
    LAUNCH(pcg_direction_kernel<T>, P.G, n, k, k0, z, p, P, st, update ? 1 : 0, flexible ? 1 : 0);
}
template <class V, class T>
void launch_pcg_spmv(hipStream_t s, Sell<V> A, const T *p, T *q, PcgParts P, const PcgState *st) {
    LAUNCH((pcg_spmv_kernel<V, T>), P.G, A, p, q, P, st);
}
void launch_pcg_update(hipStream_t s, int32_t n, int k, double *x, double *r, double *z, const double *p,
                       const double *q, const double *dinv, PcgParts P, PcgState *st) {
    LAUNCH(pcg_update_kernel, P.G, n, k, x, r, z, p, q, dinv, P, st);
}
template <class T>
void launch_pcg_update_xr(hipStream_t s, int32_t n, int k, T *x, T *r, const T *p, const T *q, PcgParts P,
                          PcgState *st, const T *dinv, T *x0) {
    LAUNCH(pcg_update_xr_kernel<T>, P.G, n, k, x, r, p, q, P, st, dinv, x0);
}
template <class T>
void launch_pcg_dot_rz(hipStream_t s, int32_t n, int k, const T *r, const T *z, PcgParts P, const PcgState *st) {
    LAUNCH(pcg_dot_rz_kernel<T>, P.G, n, k, r, z, P, st);
}
template <class T>
void launch_pcg_init_plain(hipStream_t s, int32_t n, const T *b, T *x, T *r, PcgParts P) {
    LAUNCH(pcg_init_plain_kernel<T>, P.G, n, b, x, r, P);
}
void launch_norm2(hipStream_t s, int32_t n, const double *r, double *parts, double *out) {
    const unsigned g = vec_grid(n);
    LAUNCH(norm2_kernel, g, n, r, parts);
    launch_finalize_sum(s, parts, (int)g, (int)g, 1, out);
}
void launch_normalize_to_float(hipStream_t s, int32_t n, const double *r, const double *nrm2, float *r32) {
    if (n > 0) LAUNCH(normalize_to_float_kernel, vec_grid(n), n, r, nrm2, r32);
}
void launch_correct(hipStream_t s, int32_t n, double *x, const float *d32, const double *nrm2) {
    if (n > 0) LAUNCH(correct_kernel, vec_grid(n), n, x, d32, nrm2);
}

#define INST(T)                                                                                                   \
    template void launch_pcg_direction<T>(hipStream_t, int32_t, int, int, const T *, T *, PcgParts, PcgState *,   \
                                          bool, bool);                                                            \
    template void launch_pcg_spmv<T, T>(hipStream_t, Sell<T>, const T *, T *, PcgParts, const PcgState *);        \
    template void launch_pcg_update_xr<T>(hipStream_t, int32_t, int, T *, T *, const T *, const T *, PcgParts,   \
                                          PcgState *, const T *, T *);                                            \
    template void launch_pcg_dot_rz<T>(hipStream_t, int32_t, int, const T *, const T *, PcgParts,                 \
                                       const PcgState *);                                                         \
    template void launch_pcg_init_plain<T>(hipStream_t, int32_t, const T *, T *, T *, PcgParts);
INST(double)
INST(float)

}  // namespace vag
