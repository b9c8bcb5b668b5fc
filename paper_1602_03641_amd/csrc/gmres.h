// Restarted flexible GMRES(m) (right preconditioning) with CGS2
// orthogonalisation (host driver; kernels in gmres.hip).  The preconditioned
// vectors z_j = M^-1 v_j are kept, and each cycle ends with x += Z y, so the
// update satisfies A Z = V H exactly as the Arnoldi step built it, even when
// M^-1 is not exactly linear (an FP32 V-cycle, whose rounding on
// ill-conditioned coarse levels would otherwise cap the attainable residual;
// a K-cycle).  The small Hessenberg least-squares problem is solved on the
// host with Givens rotations, one device read per iteration.
#pragma once

#include <cmath>
#include <vector>

#include "vag_internal.h"

namespace vag {

int gmres_grid(int64_t n);
template <class V, class T>
void launch_gm_spmv(hipStream_t s, Sell<V> A, const T *x, T *y);
// w -= V h with h = V^T w (k basis vectors), then partials of ||w||^2 in nparts
template <class T>
void launch_gm_orthogonalize(hipStream_t s, int32_t n, int k, const T *V, int64_t ld, T *w, double *parts,
                             double *h, double *nparts);
template <class T>
void launch_gm_normalize(hipStream_t s, int32_t n, const double *nparts, const T *w, T *out, double *hn);
template <class T>
void launch_gm_combine(hipStream_t s, int32_t n, int k, const T *V, int64_t ld, const double *y, T *t);
template <class T>
void launch_gm_add(hipStream_t s, int32_t n, const T *z, T *x);
template <class V, class T>
void launch_gm_residual(hipStream_t s, Sell<V> A, const T *b, const T *x, T *r, double *nparts);

// Device and pinned scratch of one GMRES(m) solve on vectors of type T.
template <class T>
struct GmresWork {
    T *V = nullptr;          // (m+1) * n basis
    T *Z = nullptr;          // m * n preconditioned basis vectors
    T *w = nullptr, *t = nullptr;
    double *parts = nullptr;  // (m+1) * gmres_grid(n)
    double *nparts = nullptr; // gmres_grid(n)
    double *hd = nullptr;     // device: h1[m+1], h2[m+1], hn, y[m+1]
    double *hh = nullptr;     // pinned host copy of hd
};

struct GmresResult {
    int iterations = 0;
    bool converged = false;
    double rnorm = 0.0;  // final true residual norm
};

// Solves A x = b from the given x until ||b - A x|| <= tol (absolute) or
// max_iter iterations.  prec(in, out): out = M^-1 in.
template <class V, class T, class Prec>
GmresResult gmres_solve(hipStream_t s, Sell<V> A, const T *b, T *x, double tol, int m, int max_iter,
                        const GmresWork<T> &W, Prec prec) {
    const int32_t n = A.n;
    const int64_t ld = n;
    double *h1 = W.hd, *h2 = W.hd + (m + 1), *hn = W.hd + 2 * (m + 1), *yd = W.hd + 2 * (m + 1) + 1;
    double *H1 = W.hh, *H2 = W.hh + (m + 1), *HN = W.hh + 2 * (m + 1), *Y = W.hh + 2 * (m + 1) + 1;
    std::vector<double> R((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m);
    GmresResult res;
    // r0 = b - A x, v0 = r0 / ||r0||
    launch_gm_residual<V, T>(s, A, b, x, W.w, W.nparts);
    launch_gm_normalize<T>(s, n, W.nparts, W.w, W.V, hn);
    VAG_HIP(hipMemcpyAsync(HN, hn, sizeof(double), hipMemcpyDeviceToHost, s));
    VAG_HIP(hipStreamSynchronize(s));
    double beta = *HN;
    res.rnorm = beta;
    if (beta <= tol) {
        res.converged = true;
        return res;
    }
    int it = 0;
    while (it < max_iter) {
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int j = 0;
        double est = beta;
        for (; j < m && it < max_iter; ++j, ++it) {
            T *vj = W.V + (int64_t)j * ld;
            T *zj = W.Z + (int64_t)j * ld;
            prec(vj, zj);
            launch_gm_spmv<V, T>(s, A, zj, W.w);
            launch_gm_orthogonalize<T>(s, n, j + 1, W.V, ld, W.w, W.parts, h1, W.nparts);
            launch_gm_orthogonalize<T>(s, n, j + 1, W.V, ld, W.w, W.parts, h2, W.nparts);
            launch_gm_normalize<T>(s, n, W.nparts, W.w, W.V + (int64_t)(j + 1) * ld, hn);
            VAG_HIP(hipMemcpyAsync(W.hh, W.hd, (2 * (m + 1) + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
            VAG_HIP(hipStreamSynchronize(s));
            double *col = &R[(size_t)j * (m + 1)];
            for (int i = 0; i <= j; ++i) col[i] = H1[i] + H2[i];
            col[j + 1] = *HN;
            for (int i = 0; i < j; ++i) {  // previous rotations
                const double a = cs[i] * col[i] + sn[i] * col[i + 1];
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                col[i] = a;
            }
            const double rr = std::hypot(col[j], col[j + 1]);
            cs[j] = rr > 0 ? col[j] / rr : 1.0;
            sn[j] = rr > 0 ? col[j + 1] / rr : 0.0;
            col[j] = rr;
            col[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            est = std::fabs(g[j + 1]);
            if (est <= tol || *HN == 0.0) {
                ++j;
                ++it;
                break;
            }
        }
        // y = R^-1 g, x += Z y
        for (int i = j - 1; i >= 0; --i) {
            double v = g[i];
            for (int k = i + 1; k < j; ++k) v -= R[(size_t)k * (m + 1) + i] * Y[k];
            Y[i] = v / R[(size_t)i * (m + 1) + i];
        }
        VAG_HIP(hipMemcpyAsync(yd, Y, j * sizeof(double), hipMemcpyHostToDevice, s));
        launch_gm_combine<T>(s, n, j, W.Z, ld, yd, W.t);
        launch_gm_add<T>(s, n, W.t, x);
        // true residual; restart from it
        launch_gm_residual<V, T>(s, A, b, x, W.w, W.nparts);
        launch_gm_normalize<T>(s, n, W.nparts, W.w, W.V, hn);
        VAG_HIP(hipMemcpyAsync(HN, hn, sizeof(double), hipMemcpyDeviceToHost, s));
        VAG_HIP(hipStreamSynchronize(s));
        beta = *HN;
        res.rnorm = beta;
        res.iterations = it;
        if (beta <= tol) {
            res.converged = true;
            break;
        }
    }
    res.iterations = it;
    return res;
}

}  // namespace vag
