// Kernels of right-preconditioned BiCGStab (van der Vorst's stabilised
// bi-conjugate gradients, the alternative Krylov method of the paper's solver
// study, §5.3) with every scalar kept on the device: each kernel forms the
// scalars it needs from the per-block partials of the previous kernels
// (summed in a fixed order by every block, so the result is bitwise
// reproducible), and the host only queues iterations and reads the state
// every few iterations, as for CG.
//
// Iteration k (rhat = r_0 fixed; p, v, s, t as in the method):
//   rho_k   = rhat . r_k
//   beta    = (rho_k / rho_{k-1}) (alpha_{k-1} / omega_{k-1})
//   p       = r + beta (p - omega_{k-1} v)          (p = r at the start)
//   phat    = M^-1 p,   v = A phat,   alpha_k = rho_k / (rhat . v)
//   s       = r - alpha_k v                           (done if |s| is small)
//   shat    = M^-1 s,   t = A shat,   omega_k = (t . s) / (t . t)
//   x      += alpha_k phat + omega_k shat,   r = s - omega_k t
#include "reduce.h"
#include "sell.h"

namespace vag {

namespace {

constexpr int kT = kKrylovThreads;

#define GSB(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// partial slots: rho(k) parity 0/1, rhat.v, t.s, t.t, r.r parity 0/1, s.s
struct BcgParts {
    double *base;
    int G;
    __device__ double *rho(int k) const { return base + (size_t)(k & 1) * G; }
    __device__ double *rv() const { return base + (size_t)2 * G; }
    __device__ double *ts() const { return base + (size_t)3 * G; }
    __device__ double *tt() const { return base + (size_t)4 * G; }
    __device__ double *rr(int k) const { return base + (size_t)(5 + (k & 1)) * G; }
    __device__ double *ss() const { return base + (size_t)7 * G; }
};

__device__ inline double total(const double *p, int G) { return sum_parts<OpSum, kT>(p, G); }

// x0 given: r = b - A x (or r = b when x is zero: A == null), rhat = r;
// partials r.r and rhat.r for iteration k0 - 1
__global__ __launch_bounds__(kT) void bcg_init_kernel(Sell<double> A, int zero_x, int k0, const double *__restrict__ b,
                                                      double *__restrict__ x, double *__restrict__ r,
                                                      double *__restrict__ rhat, BcgParts P) {
    double v[1] = {0.0};
    GSB(i, A.n) {
        double ri;
        if (zero_x) {
            x[i] = 0.0;
            ri = b[i];
        } else {
            ri = b[i] - sell_row_apply<double, double>(A, (int32_t)i, [&](int32_t j) { return x[j]; });
        }
        r[i] = ri;
        rhat[i] = ri;
        v[0] += ri * ri;
    }
    block_reduce<OpSum, 1, kT>(v);
    if (threadIdx.x == 0) {
        P.rr(k0 - 1)[blockIdx.x] = v[0];
        P.rho(k0 - 1)[blockIdx.x] = v[0];
    }
}

__global__ __launch_bounds__(kT) void bcg_start_kernel(BcgParts P, PcgState *st, double rtol, int k0) {
    const double rr = total(P.rr(k0 - 1), P.G);
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (k0 == 0) st->bnorm2 = rr;
        st->tol2 = rtol * rtol * rr;
        st->rr = rr;
        st->iter = k0;
        st->done = (rr == 0.0);
        st->converged = (rr == 0.0);
    }
}

// convergence test on r_{k-1}, then the search direction p
__global__ __launch_bounds__(kT) void bcg_direction_kernel(int32_t n, int k, int k0, const double *__restrict__ r,
                                                           double *__restrict__ p, const double *__restrict__ v,
                                                           BcgParts P, PcgState *st, int update) {
    if (st->done) return;
    const double rr = total(P.rr(k - 1), P.G);
    const double rho = total(P.rho(k - 1), P.G);
    const bool conv = rr <= st->tol2;
    if (conv || rho == 0.0 || !(rr == rr)) {  // converged, breakdown (rhat orthogonal to r) or NaN
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->done = 1;
            st->converged = conv ? 1 : 0;
            st->rr = rr;
        }
        return;
    }
    if (!update) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->rr = rr;
        return;
    }
    if (k == k0) {
        GSB(i, n) p[i] = r[i];
        return;
    }
    const double rho_prev = total(P.rho(k - 2), P.G);
    const double alpha = rho_prev / total(P.rv(), P.G);
    const double omega = total(P.ts(), P.G) / total(P.tt(), P.G);
    const double beta = (rho / rho_prev) * (alpha / omega);
    GSB(i, n) p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

// y = A x with the partials of w . y into parts (and of y . y into parts2)
__global__ __launch_bounds__(kT) void bcg_spmv_dot_kernel(Sell<double> A, const double *__restrict__ x,
                                                          double *__restrict__ y, const double *__restrict__ w,
                                                          double *__restrict__ parts, double *__restrict__ parts2,
                                                          const PcgState *st) {
    if (st->done) return;
    double v[2] = {0.0, 0.0};
    GSB(i, A.n) {
        const double yi = sell_row_apply<double, double>(A, (int32_t)i, [&](int32_t j) { return x[j]; });
        y[i] = yi;
        v[0] += w[i] * yi;
        v[1] += yi * yi;
    }
    block_reduce<OpSum, 2, kT>(v);
    if (threadIdx.x == 0) {
        parts[blockIdx.x] = v[0];
        if (parts2) parts2[blockIdx.x] = v[1];
    }
}

// s = r - alpha v; if |s| already meets the tolerance, x += alpha phat and stop
__global__ __launch_bounds__(kT) void bcg_s_kernel(int32_t n, int k, const double *__restrict__ r,
                                                   const double *__restrict__ v, double *__restrict__ s, BcgParts P,
                                                   const PcgState *st) {
    if (st->done) return;
    const double alpha = total(P.rho(k - 1), P.G) / total(P.rv(), P.G);
    double w[1] = {0.0};
    GSB(i, n) {
        const double si = r[i] - alpha * v[i];
        s[i] = si;
        w[0] += si * si;
    }
    block_reduce<OpSum, 1, kT>(w);
    if (threadIdx.x == 0) P.ss()[blockIdx.x] = w[0];
}

// the half step: when |s|^2 <= tol2, x += alpha phat and the solve is done
__global__ __launch_bounds__(kT) void bcg_half_kernel(int32_t n, int k, const double *__restrict__ phat,
                                                      double *__restrict__ x, BcgParts P, PcgState *st) {
    if (st->done) return;
    const double ss = total(P.ss(), P.G);
    if (!(ss <= st->tol2)) return;
    const double alpha = total(P.rho(k - 1), P.G) / total(P.rv(), P.G);
    GSB(i, n) x[i] += alpha * phat[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->done = 1;
        st->converged = 1;
        st->rr = ss;
        st->iter = k + 1;
    }
}

// x += alpha phat + omega shat, r = s - omega t; partials r.r and rhat.r
__global__ __launch_bounds__(kT) void bcg_update_kernel(int32_t n, int k, const double *__restrict__ phat,
                                                        const double *__restrict__ shat,
                                                        const double *__restrict__ s, const double *__restrict__ t,
                                                        const double *__restrict__ rhat, double *__restrict__ x,
                                                        double *__restrict__ r, BcgParts P, PcgState *st) {
    if (st->done) return;
    const double alpha = total(P.rho(k - 1), P.G) / total(P.rv(), P.G);
    const double tt = total(P.tt(), P.G);
    const double omega = tt > 0.0 ? total(P.ts(), P.G) / tt : 0.0;
    double v[2] = {0.0, 0.0};
    GSB(i, n) {
        x[i] += alpha * phat[i] + omega * shat[i];
        const double ri = s[i] - omega * t[i];
        r[i] = ri;
        v[0] += ri * ri;
        v[1] += rhat[i] * ri;
    }
    block_reduce<OpSum, 2, kT>(v);
    if (threadIdx.x == 0) {
        P.rr(k)[blockIdx.x] = v[0];
        P.rho(k)[blockIdx.x] = v[1];
        if (blockIdx.x == 0) st->iter = k + 1;
    }
}

}  // namespace

int bcg_grid(int64_t n) { return (int)reduce_grid(n, kT); }

#define BLAUNCH(kern, G, ...)                                                      \
    do {                                                                           \
        hipLaunchKernelGGL(kern, dim3(G), dim3(kT), 0, s, __VA_ARGS__);            \
        VAG_HIP(hipGetLastError());                                                \
    } while (0)

void launch_bcg_init(hipStream_t s, Sell<double> A, bool zero_x, int k0, const double *b, double *x, double *r,
                     double *rhat, double *parts) {
    const int G = bcg_grid(A.n);
    BLAUNCH(bcg_init_kernel, G, A, zero_x ? 1 : 0, k0, b, x, r, rhat, BcgParts{parts, G});
}
void launch_bcg_start(hipStream_t s, int32_t n, double *parts, PcgState *st, double rtol, int k0) {
    BLAUNCH(bcg_start_kernel, 1, BcgParts{parts, bcg_grid(n)}, st, rtol, k0);
}
void launch_bcg_direction(hipStream_t s, int32_t n, int k, int k0, const double *r, double *p, const double *v,
                          double *parts, PcgState *st, bool update) {
    const int G = bcg_grid(n);
    BLAUNCH(bcg_direction_kernel, G, n, k, k0, r, p, v, BcgParts{parts, G}, st, update ? 1 : 0);
}
void launch_bcg_spmv_v(hipStream_t s, Sell<double> A, const double *phat, double *v, const double *rhat,
                       double *parts, const PcgState *st) {
    const int G = bcg_grid(A.n);
    BLAUNCH(bcg_spmv_dot_kernel, G, A, phat, v, rhat, parts + (size_t)2 * G, (double *)nullptr, st);
}
void launch_bcg_s(hipStream_t s, int32_t n, int k, const double *r, const double *v, const double *phat, double *sv,
                  double *x, double *parts, PcgState *st) {
    const int G = bcg_grid(n);
    BLAUNCH(bcg_s_kernel, G, n, k, r, v, sv, BcgParts{parts, G}, st);
    BLAUNCH(bcg_half_kernel, G, n, k, phat, x, BcgParts{parts, G}, st);
}
void launch_bcg_spmv_t(hipStream_t s, Sell<double> A, const double *shat, double *t, const double *sv, double *parts,
                       const PcgState *st) {
    const int G = bcg_grid(A.n);
    BLAUNCH(bcg_spmv_dot_kernel, G, A, shat, t, sv, parts + (size_t)3 * G, parts + (size_t)4 * G, st);
}
void launch_bcg_update(hipStream_t s, int32_t n, int k, const double *phat, const double *shat, const double *sv,
                       const double *t, const double *rhat, double *x, double *r, double *parts, PcgState *st) {
    const int G = bcg_grid(n);
    BLAUNCH(bcg_update_kernel, G, n, k, phat, shat, sv, t, rhat, x, r, BcgParts{parts, G}, st);
}

}  // namespace vag
