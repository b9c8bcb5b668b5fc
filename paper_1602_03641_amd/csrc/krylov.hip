// Krylov kernels for the SPD system of eq eqschur: CSR SpMV (a group of LPR
// lanes per row, row entries read contiguously), and preconditioned CG whose
// scalars stay on the device.  Every kernel of an iteration first reads the
// `done` flag and returns at once when the solve has converged, so the host
// can queue many iterations and check convergence only now and then.
#include "reduce.h"

namespace vag {

constexpr int kLPR = 8;       // lanes per CSR row (rows have ~27 entries)
constexpr int kThreads = 256;

template <int LPR>
__device__ inline double row_dot(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                 const double *__restrict__ val, const double *__restrict__ x, int32_t row,
                                 int lane) {
    double s = 0.0;
    const int32_t e = rp[row + 1];
    for (int32_t k = rp[row] + lane; k < e; k += LPR) s += val[k] * x[col[k]];
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, LPR);
    return s;
}

__global__ __launch_bounds__(kThreads) void spmv_kernel(int32_t n, const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col,
                                                        const double *__restrict__ val,
                                                        const double *__restrict__ x, double *__restrict__ y) {
    const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kLPR;
    const int lane = threadIdx.x % kLPR;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x / kLPR;
    for (int64_t row = g; row < n; row += stride) {
        const double s = row_dot<kLPR>(rp, col, val, x, (int32_t)row, lane);
        if (lane == 0) y[row] = s;
    }
}

// r = b - A x; parts: ||r||^2, ||b||^2
__global__ __launch_bounds__(kThreads) void residual_kernel(int32_t n, const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ col,
                                                            const double *__restrict__ val,
                                                            const double *__restrict__ x,
                                                            const double *__restrict__ b, double *__restrict__ r,
                                                            ReduceScratch rs, double *__restrict__ out) {
    const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kLPR;
    const int lane = threadIdx.x % kLPR;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x / kLPR;
    double v[2] = {0.0, 0.0};
    for (int64_t row = g; row < n; row += stride) {
        const double s = row_dot<kLPR>(rp, col, val, x, (int32_t)row, lane);
        if (lane == 0) {
            const double t = b[row] - s;
            r[row] = t;
            v[0] += t * t;
            v[1] += b[row] * b[row];
        }
    }
    if (grid_reduce<OpSum, 2, kThreads>(v, rs, 0) && threadIdx.x == 0) {
        out[0] = v[0];
        out[1] = v[1];
    }
}

__global__ __launch_bounds__(kThreads) void fill_kernel(int64_t n, double v, double *__restrict__ x) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}
__global__ __launch_bounds__(kThreads) void copy_kernel(int64_t n, const double *__restrict__ s,
                                                        double *__restrict__ d) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = s[i];
}

__global__ __launch_bounds__(kThreads) void jacobi_kernel(int64_t n, const double *__restrict__ dinv,
                                                          const double *__restrict__ r, double *__restrict__ z) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        z[i] = dinv[i] * r[i];
}

// ---------------------------------------------------------------------------
// Jacobi-preconditioned CG, x0 = 0
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void pcg_init_kernel(int32_t n, const double *__restrict__ b,
                                                            const double *__restrict__ dinv,
                                                            double *__restrict__ x, double *__restrict__ r,
                                                            double *__restrict__ z, double *__restrict__ p,
                                                            ReduceScratch rs, PcgState *st, double rtol,
                                                            int max_iter) {
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double bi = b[i];
        const double zi = dinv[i] * bi;
        x[i] = 0.0;
        r[i] = bi;
        z[i] = zi;
        p[i] = zi;
        v[0] += bi * zi;
        v[1] += bi * bi;
    }
    if (grid_reduce<OpSum, 2, kThreads>(v, rs, 0) && threadIdx.x == 0) {
        st->rz = v[0];
        st->rr = v[1];
        st->bnorm2 = v[1];
        st->tol2 = rtol * rtol * v[1];
        st->iter = 0;
        st->max_iter = max_iter;
        const bool conv = (v[1] == 0.0);
        st->done = conv || max_iter <= 0;
        st->converged = conv;
        st->alpha = st->beta = st->pq = 0.0;
    }
}

// q = A p, alpha = rz / (p . q)
__global__ __launch_bounds__(kThreads) void pcg_spmv_kernel(int32_t n, const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ col,
                                                            const double *__restrict__ val,
                                                            const double *__restrict__ p, double *__restrict__ q,
                                                            ReduceScratch rs, PcgState *st) {
    if (st->done) return;
    const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kLPR;
    const int lane = threadIdx.x % kLPR;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x / kLPR;
    double v[1] = {0.0};
    for (int64_t row = g; row < n; row += stride) {
        const double s = row_dot<kLPR>(rp, col, val, p, (int32_t)row, lane);
        if (lane == 0) {
            q[row] = s;
            v[0] += p[row] * s;
        }
    }
    if (grid_reduce<OpSum, 1, kThreads>(v, rs, 1) && threadIdx.x == 0) {
        st->pq = v[0];
        st->alpha = st->rz / v[0];
    }
}

// x += alpha p, r -= alpha q, z = D^-1 r, beta = (r.z)_new / (r.z)_old
__global__ __launch_bounds__(kThreads) void pcg_update_kernel(int32_t n, double *__restrict__ x,
                                                              double *__restrict__ r, double *__restrict__ z,
                                                              const double *__restrict__ p,
                                                              const double *__restrict__ q,
                                                              const double *__restrict__ dinv,
                                                              ReduceScratch rs, PcgState *st) {
    if (st->done) return;
    const double alpha = st->alpha;
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        const double zi = dinv[i] * ri;
        r[i] = ri;
        z[i] = zi;
        v[0] += ri * zi;
        v[1] += ri * ri;
    }
    if (grid_reduce<OpSum, 2, kThreads>(v, rs, 2) && threadIdx.x == 0) {
        st->beta = v[0] / st->rz;
        st->rz = v[0];
        st->rr = v[1];
        st->iter += 1;
        if (v[1] <= st->tol2) {
            st->done = 1;
            st->converged = 1;
        } else if (st->iter >= st->max_iter) {
            st->done = 1;
        }
    }
}

__global__ __launch_bounds__(kThreads) void pcg_direction_kernel(int32_t n, const double *__restrict__ z,
                                                                 double *__restrict__ p, const PcgState *st) {
    if (st->done) return;
    const double beta = st->beta;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + beta * p[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned rows_grid(int64_t n) { return reduce_grid(n * kLPR, kThreads); }
static inline unsigned vec_grid(int64_t n) { return reduce_grid(n, kThreads); }

void launch_fill(hipStream_t s, int64_t n, double v, double *x) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_kernel, dim3(vec_grid(n)), dim3(kThreads), 0, s, n, v, x);
    VAG_HIP(hipGetLastError());
}
void launch_copy(hipStream_t s, int64_t n, const double *src, double *dst) {
    if (n <= 0) return;
    hipLaunchKernelGGL(copy_kernel, dim3(vec_grid(n)), dim3(kThreads), 0, s, n, src, dst);
    VAG_HIP(hipGetLastError());
}
void launch_jacobi(hipStream_t s, int64_t n, const double *dinv, const double *r, double *z) {
    if (n <= 0) return;
    hipLaunchKernelGGL(jacobi_kernel, dim3(vec_grid(n)), dim3(kThreads), 0, s, n, dinv, r, z);
    VAG_HIP(hipGetLastError());
}
void launch_spmv(hipStream_t s, int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                 const double *x, double *y) {
    if (n <= 0) return;
    hipLaunchKernelGGL(spmv_kernel, dim3(rows_grid(n)), dim3(kThreads), 0, s, n, rp, col, val, x, y);
    VAG_HIP(hipGetLastError());
}
void launch_residual_norm(hipStream_t s, int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                          const double *x, const double *b, double *r, ReduceScratch rs, double *out2) {
    hipLaunchKernelGGL(residual_kernel, dim3(rows_grid(n)), dim3(kThreads), 0, s, n, rp, col, val, x, b, r, rs,
                       out2);
    VAG_HIP(hipGetLastError());
}
void launch_pcg_init(hipStream_t s, int32_t n, const double *b, const double *dinv, double *x, double *r,
                     double *z, double *p, ReduceScratch rs, PcgState *st, double rtol, int max_iter) {
    hipLaunchKernelGGL(pcg_init_kernel, dim3(vec_grid(n)), dim3(kThreads), 0, s, n, b, dinv, x, r, z, p, rs, st,
                       rtol, max_iter);
    VAG_HIP(hipGetLastError());
}
void launch_pcg_iter(hipStream_t s, int32_t n, const int32_t *rp, const int32_t *col, const double *val,
                     const double *dinv, double *x, double *r, double *z, double *p, double *q,
                     ReduceScratch rs, PcgState *st) {
    hipLaunchKernelGGL(pcg_spmv_kernel, dim3(rows_grid(n)), dim3(kThreads), 0, s, n, rp, col, val, p, q, rs, st);
    hipLaunchKernelGGL(pcg_update_kernel, dim3(vec_grid(n)), dim3(kThreads), 0, s, n, x, r, z, p, q, dinv, rs,
                       st);
    hipLaunchKernelGGL(pcg_direction_kernel, dim3(vec_grid(n)), dim3(kThreads), 0, s, n, z, p, st);
    VAG_HIP(hipGetLastError());
}

}  // namespace vag
