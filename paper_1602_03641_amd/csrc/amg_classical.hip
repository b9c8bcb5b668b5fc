// Classical (Ruge-Stueben type) AMG hierarchy: the kernels (host side in
// amg_host.cpp).  The paper's solver study (§5.3) uses a classical AMG
// (BoomerAMG) beside aggregation AMG; this is the GPU form used here:
//
// * strength: j strongly influences i when -a_ij >= theta max_{k != i}(-a_ik)
//   (negative couplings only).  The matrices are symmetric, so whether i
//   strongly influences j is read from the same entry with j's row maximum,
//   and the measure lambda_i (how many points i influences) needs no
//   transpose;
// * coarse/fine splitting by PMIS (De Sterck, Yang, Heys): a point is coarse
//   when its key (lambda, then a bijective hash of the index) exceeds those
//   of all undecided strong neighbours; undecided points that strongly
//   depend on a new coarse point become fine; points that influence no one
//   start fine;
// * direct interpolation (Stueben's review of AMG): w_ij = -alpha_i a_ij / a~_ii
//   over the strong coarse neighbours, alpha_i = sum of all negative
//   couplings / sum of the strong coarse ones, a~_ii = a_ii + the positive
//   couplings;
// * R = P^T row by row (a coarse point's row lists the fine neighbours that
//   interpolate from it, in the order of its own matrix row: no atomics);
// * Galerkin product R (A P) by two sparse products, one thread per output
//   row accumulating into its own open-addressing table in a scratch buffer,
//   in a fixed order: bitwise reproducible.
#include <algorithm>

#include "amg.h"
#include "reduce.h"

namespace vag {

namespace {

constexpr int kCT = 256;
constexpr int8_t kU = 0, kC = 1, kF = 2;

#define CL_GS(i, n) \
    for (int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x); i < (n); i += (int32_t)(gridDim.x * blockDim.x))

int cgrid(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kCT - 1) / kCT, 16384)); }

__device__ inline int sell_w(const int64_t *ptr, int32_t i) { return (int)((ptr[(i >> 6) + 1] - ptr[i >> 6]) >> 6); }
__device__ inline int64_t sell_at(const int64_t *ptr, int32_t i) { return ptr[i >> 6] + (i & 63); }

// bijective mixing of a 32-bit index (xorshift-multiply rounds, each invertible)
__device__ inline uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

}  // namespace

// m_i = max over off-diagonal entries of -a_ij (0 when none is negative)
__global__ __launch_bounds__(kCT) void cl_negmax_kernel(Sell<double> A, double *m) {
    CL_GS(i, A.n) {
        const int64_t b = sell_at(A.ptr, i);
        const int w = sell_w(A.ptr, i);
        double mx = 0.0;
        for (int j = 0; j < w; ++j) {
            const int64_t p = b + (int64_t)j * 64;
            if (A.col[p] != i) mx = fmax(mx, -A.val[p]);
        }
        m[i] = mx;
    }
}

// per stored entry: bit 0 = i depends strongly on j, bit 1 = j depends
// strongly on i; keys and initial states
__global__ __launch_bounds__(kCT) void cl_strength_kernel(Sell<double> A, const double *m, double theta, uint8_t *sf,
                                                          uint64_t *key, int8_t *state) {
    CL_GS(i, A.n) {
        const int64_t b = sell_at(A.ptr, i);
        const int w = sell_w(A.ptr, i);
        const double mi = m[i];
        uint32_t lam = 0;
        for (int j = 0; j < w; ++j) {
            const int64_t p = b + (int64_t)j * 64;
            const int32_t c = A.col[p];
            const double v = -A.val[p];
            uint8_t f = 0;
            if (c != i && v > 0.0) {
                if (v >= theta * mi) f |= 1;
                if (v >= theta * m[c]) f |= 2;
            }
            sf[p] = f;
            lam += f >> 1;
        }
        key[i] = ((uint64_t)lam << 32) | mix32((uint32_t)i);
        state[i] = lam == 0 ? kF : kU;
    }
}

// undecided points whose key beats every undecided strong neighbour become coarse
__global__ __launch_bounds__(kCT) void cl_pmis_select_kernel(Sell<double> A, const uint8_t *sf, const uint64_t *key,
                                                             const int8_t *in, int8_t *out) {
    CL_GS(i, A.n) {
        int8_t s = in[i];
        if (s == kU) {
            const int64_t b = sell_at(A.ptr, i);
            const int w = sell_w(A.ptr, i);
            const uint64_t ki = key[i];
            bool top = true;
            for (int j = 0; j < w && top; ++j) {
                const int64_t p = b + (int64_t)j * 64;
                const int32_t c = A.col[p];
                if (sf[p] && in[c] == kU && key[c] > ki) top = false;
            }
            if (top) s = kC;
        }
        out[i] = s;
    }
}

// undecided points that depend strongly on a coarse point become fine; the
// remaining undecided points are counted (one atomic per block)
__global__ __launch_bounds__(kCT) void cl_pmis_fine_kernel(Sell<double> A, const uint8_t *sf, int8_t *st, int *cnt) {
    int mine = 0;
    CL_GS(i, A.n) {
        if (st[i] != kU) continue;
        const int64_t b = sell_at(A.ptr, i);
        const int w = sell_w(A.ptr, i);
        bool fine = false;
        for (int j = 0; j < w && !fine; ++j) {
            const int64_t p = b + (int64_t)j * 64;
            if ((sf[p] & 1) && st[A.col[p]] == kC) fine = true;
        }
        if (fine)
            st[i] = kF;
        else
            ++mine;
    }
    const int total = __syncthreads_count(mine > 0) > 0 ? 1 : 0;
    if (threadIdx.x == 0 && total) atomicAdd(cnt, 1);
}

// points still undecided after the last round become coarse
__global__ __launch_bounds__(kCT) void cl_pmis_close_kernel(int32_t n, int8_t *st) {
    CL_GS(i, n) if (st[i] == kU) st[i] = kC;
}

// interpolation row lengths and coarse flags
__global__ __launch_bounds__(kCT) void cl_interp_count_kernel(Sell<double> A, const uint8_t *sf, const int8_t *st,
                                                              int32_t *plen, int32_t *cflag) {
    CL_GS(i, A.n) {
        if (st[i] == kC) {
            plen[i] = 1;
            cflag[i] = 1;
            continue;
        }
        cflag[i] = 0;
        const int64_t b = sell_at(A.ptr, i);
        const int w = sell_w(A.ptr, i);
        int32_t c = 0;
        for (int j = 0; j < w; ++j) {
            const int64_t p = b + (int64_t)j * 64;
            c += (sf[p] & 1) && st[A.col[p]] == kC;
        }
        plen[i] = c;
    }
}

__global__ __launch_bounds__(kCT) void cl_interp_fill_kernel(Sell<double> A, const uint8_t *sf, const int8_t *st,
                                                             const int32_t *cidx, const int32_t *pptr, int32_t *pcol,
                                                             double *pval, int32_t *cfine) {
    CL_GS(i, A.n) {
        int32_t q = pptr[i];
        if (st[i] == kC) {
            pcol[q] = cidx[i];
            pval[q] = 1.0;
            cfine[cidx[i]] = i;
            continue;
        }
        if (pptr[i + 1] == q) continue;
        const int64_t b = sell_at(A.ptr, i);
        const int w = sell_w(A.ptr, i);
        double aii = 0.0, neg = 0.0, pos = 0.0, negc = 0.0;
        for (int j = 0; j < w; ++j) {
            const int64_t p = b + (int64_t)j * 64;
            const int32_t c = A.col[p];
            const double v = A.val[p];
            if (c == i) {
                aii += v;  // padding entries hold 0
            } else {
                neg += fmin(v, 0.0);
                pos += fmax(v, 0.0);
                if ((sf[p] & 1) && st[c] == kC) negc += v;
            }
        }
        const double scale = -(neg / negc) / (aii + pos);
        for (int j = 0; j < w; ++j) {
            const int64_t p = b + (int64_t)j * 64;
            const int32_t c = A.col[p];
            if (c != i && (sf[p] & 1) && st[c] == kC) {
                pcol[q] = cidx[c];
                pval[q] = scale * A.val[p];
                ++q;
            }
        }
    }
}

// R = P^T: coarse point c (fine point f) takes (f, 1) and, for each fine
// neighbour i of f in A's row order, P's weight of c in row i
template <bool FILL>
__global__ __launch_bounds__(kCT) void cl_transpose_kernel(Sell<double> A, int32_t nc, const int32_t *cfine,
                                                           const int8_t *st, const int32_t *pptr, const int32_t *pcol,
                                                           const double *pval, int32_t *rlen, const int32_t *rptr,
                                                           int32_t *rcol, double *rval) {
    CL_GS(c, nc) {
        const int32_t f = cfine[c];
        int32_t q = FILL ? rptr[c] : 0;
        if (FILL) {
            rcol[q] = f;
            rval[q] = 1.0;
        }
        ++q;
        const int64_t b = sell_at(A.ptr, f);
        const int w = sell_w(A.ptr, f);
        for (int j = 0; j < w; ++j) {
            const int32_t i = A.col[b + (int64_t)j * 64];
            if (i == f || st[i] == kC) continue;
            for (int32_t t = pptr[i]; t < pptr[i + 1]; ++t)
                if (pcol[t] == c) {
                    if (FILL) {
                        rcol[q] = i;
                        rval[q] = pval[t];
                    }
                    ++q;
                    break;
                }
        }
        if (!FILL) rlen[c] = q;
    }
}

// Table sizes of a product row: cap = the power of two >= 2 x (number of
// contributions), at least 8, at most kClCapMax (a row with more distinct
// columns than its table holds sets *overflow).
__device__ inline int32_t cl_cap(int64_t bound) {
    int64_t c = 8;
    while (c < 2 * bound && c < kClCapMax) c <<= 1;
    return (int32_t)c;
}

// contributions of row i of A P: sum over A's nonzero entries of |P row|
__global__ __launch_bounds__(kCT) void cl_ap_cap_kernel(Sell<double> A, const int32_t *pptr, int32_t *cap) {
    CL_GS(i, A.n) {
        const int64_t b = sell_at(A.ptr, i);
        const int w = sell_w(A.ptr, i);
        int64_t s = 0;
        for (int j = 0; j < w; ++j) {
            const int64_t p = b + (int64_t)j * 64;
            if (A.val[p] != 0.0) s += pptr[A.col[p] + 1] - pptr[A.col[p]];
        }
        cap[i] = cl_cap(s);
    }
}

// contributions of row c of R (A P)
__global__ __launch_bounds__(kCT) void cl_rap_cap_kernel(int32_t nc, const int32_t *rptr, const int32_t *rcol,
                                                         const int32_t *apptr, int32_t *cap) {
    CL_GS(c, nc) {
        int64_t s = 0;
        for (int32_t q = rptr[c]; q < rptr[c + 1]; ++q) s += apptr[rcol[q] + 1] - apptr[rcol[q]];
        cap[c] = cl_cap(s);
    }
}

// sum of the table sizes of each chunk of kClChunk rows
__global__ __launch_bounds__(kCT) void cl_chunk_sum_kernel(int32_t n, const int32_t *cap, int64_t *sums) {
    const int32_t r0 = blockIdx.x * kClChunk, r1 = min(n, r0 + kClChunk);
    int64_t s = 0;
    for (int32_t i = r0 + threadIdx.x; i < r1; i += kCT) s += cap[i];
    __shared__ int64_t red[kCT];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kCT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

// One output row per thread: accumulate sum_t x_it * (row t of Y) into the
// row's own table (slots hoff[i - r0] .. + cap[i]), then either count the
// distinct columns (rowlen) or write them in slot order.  X is A in sliced
// ELL (SELL_X) or R in CSR; the output is CSR (optr) or sliced ELL (SELL_OUT).
template <bool SELL_X, bool SELL_OUT>
__global__ __launch_bounds__(kCT) void cl_product_kernel(int32_t r0, int32_t r1, Sell<double> AX, const int32_t *xptr,
                                                         const int32_t *xcol, const double *xval, const int32_t *yptr,
                                                         const int32_t *ycol, const double *yval, const int32_t *cap,
                                                         const int32_t *hoff, int32_t *hkey, double *hval, int fill,
                                                         int32_t *rowlen, const int64_t *optr, int32_t *ocol,
                                                         double *oval, int *overflow) {
    for (int32_t i = r0 + (int32_t)(blockIdx.x * blockDim.x + threadIdx.x); i < r1;
         i += (int32_t)(gridDim.x * blockDim.x)) {
        const int32_t C = cap[i];
        int32_t *K = hkey + hoff[i - r0];
        double *V = hval + hoff[i - r0];
        for (int32_t s = 0; s < C; ++s) K[s] = -1;
        const int lg = 31 - __builtin_clz((unsigned)C);
        bool over = false;
        auto add = [&](int32_t m, double v) {
            uint32_t h = (mix32((uint32_t)m) >> (32 - lg));
            for (int32_t probe = 0; probe < C; ++probe) {
                const int32_t k = K[h];
                if (k == m) {
                    V[h] += v;
                    return;
                }
                if (k == -1) {
                    K[h] = m;
                    V[h] = v;
                    return;
                }
                h = (h + 1) & (uint32_t)(C - 1);
            }
            over = true;
        };
        if (SELL_X) {
            const int64_t b = sell_at(AX.ptr, i);
            const int w = sell_w(AX.ptr, i);
            for (int j = 0; j < w && !over; ++j) {
                const int64_t p = b + (int64_t)j * 64;
                const double x = AX.val[p];
                if (x == 0.0) continue;
                const int32_t t = AX.col[p];
                for (int32_t q = yptr[t]; q < yptr[t + 1]; ++q) add(ycol[q], x * yval[q]);
            }
        } else {
            for (int32_t a = xptr[i]; a < xptr[i + 1] && !over; ++a) {
                const double x = xval[a];
                const int32_t t = xcol[a];
                for (int32_t q = yptr[t]; q < yptr[t + 1]; ++q) add(ycol[q], x * yval[q]);
            }
        }
        if (over) {
            *overflow = 1;
            if (!fill) rowlen[i] = 0;
            continue;
        }
        if (!fill) {
            int32_t n = 0;
            for (int32_t s = 0; s < C; ++s) n += K[s] != -1;
            rowlen[i] = n;
        } else {
            int32_t j = 0;
            for (int32_t s = 0; s < C; ++s) {
                if (K[s] == -1) continue;
                const int64_t p = SELL_OUT ? optr[i >> 6] + (int64_t)j * 64 + (i & 63) : optr[i] + j;
                ocol[p] = K[s];
                oval[p] = V[s];
                ++j;
            }
            if (SELL_OUT) {  // padding of the slice: the row itself with value 0
                const int w = (int)((optr[(i >> 6) + 1] - optr[i >> 6]) >> 6);
                for (; j < w; ++j) {
                    const int64_t p = optr[i >> 6] + (int64_t)j * 64 + (i & 63);
                    ocol[p] = i;
                    oval[p] = 0.0;
                }
            }
        }
    }
}

// int32 row pointers from row lengths (64-bit sizes checked by the host)
__global__ __launch_bounds__(kCT) void cl_widen_kernel(int32_t n, const int32_t *in, int64_t *out) {
    CL_GS(i, n + 1) out[i] = in[i];
}

// cycle: bc = R r (and xc = D_c^-1 bc); y = x + P e
template <class X>
__global__ __launch_bounds__(kCT) void cl_restrict_kernel(int32_t nc, const int32_t *rptr, const int32_t *rcol,
                                                          const double *rval, const X *r, X *bc, const X *dinv_c,
                                                          X *xc, const PcgState *st) {
    if (st && st->done) return;
    CL_GS(c, nc) {
        double s = 0.0;
        for (int32_t q = rptr[c]; q < rptr[c + 1]; ++q) s += rval[q] * (double)r[rcol[q]];
        bc[c] = (X)s;
        if (xc) xc[c] = dinv_c[c] * (X)s;
    }
}

template <class X>
__global__ __launch_bounds__(kCT) void cl_prolong_kernel(int32_t n, const int32_t *pptr, const int32_t *pcol,
                                                         const double *pval, const X *x, const X *e, X *y,
                                                         const PcgState *st) {
    if (st && st->done) return;
    CL_GS(i, n) {
        double s = (double)x[i];
        for (int32_t q = pptr[i]; q < pptr[i + 1]; ++q) s += pval[q] * (double)e[pcol[q]];
        y[i] = (X)s;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define CLAUNCH(kern, grid, ...)                                                  \
    do {                                                                          \
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kCT), 0, s, __VA_ARGS__);       \
        VAG_HIP(hipGetLastError());                                               \
    } while (0)

void cl_launch_strength(hipStream_t s, Sell<double> A, double theta, double *m, uint8_t *sf, uint64_t *key,
                        int8_t *state) {
    if (A.n <= 0) return;
    CLAUNCH(cl_negmax_kernel, cgrid(A.n), A, m);
    CLAUNCH(cl_strength_kernel, cgrid(A.n), A, m, theta, sf, key, state);
}
void cl_launch_pmis_round(hipStream_t s, Sell<double> A, const uint8_t *sf, const uint64_t *key, int8_t *st,
                          int8_t *tmp, int *cnt) {
    if (A.n <= 0) return;
    CLAUNCH(cl_pmis_select_kernel, cgrid(A.n), A, sf, key, st, tmp);
    CLAUNCH(cl_pmis_fine_kernel, cgrid(A.n), A, sf, tmp, cnt);
    VAG_HIP(hipMemcpyAsync(st, tmp, (size_t)A.n, hipMemcpyDeviceToDevice, s));
}
void cl_launch_pmis_close(hipStream_t s, int32_t n, int8_t *st) {
    if (n > 0) CLAUNCH(cl_pmis_close_kernel, cgrid(n), n, st);
}
void cl_launch_interp_count(hipStream_t s, Sell<double> A, const uint8_t *sf, const int8_t *st, int32_t *plen,
                            int32_t *cflag) {
    if (A.n > 0) CLAUNCH(cl_interp_count_kernel, cgrid(A.n), A, sf, st, plen, cflag);
}
void cl_launch_interp_fill(hipStream_t s, Sell<double> A, const uint8_t *sf, const int8_t *st, const int32_t *cidx,
                           const int32_t *pptr, int32_t *pcol, double *pval, int32_t *cfine) {
    if (A.n > 0) CLAUNCH(cl_interp_fill_kernel, cgrid(A.n), A, sf, st, cidx, pptr, pcol, pval, cfine);
}
void cl_launch_transpose(hipStream_t s, Sell<double> A, int32_t nc, const int32_t *cfine, const int8_t *st,
                         const int32_t *pptr, const int32_t *pcol, const double *pval, int32_t *rlen,
                         const int32_t *rptr, int32_t *rcol, double *rval) {
    if (nc <= 0) return;
    if (!rptr)
        CLAUNCH(cl_transpose_kernel<false>, cgrid(nc), A, nc, cfine, st, pptr, pcol, pval, rlen, rptr, rcol, rval);
    else
        CLAUNCH(cl_transpose_kernel<true>, cgrid(nc), A, nc, cfine, st, pptr, pcol, pval, rlen, rptr, rcol, rval);
}
void cl_launch_ap_cap(hipStream_t s, Sell<double> A, const int32_t *pptr, int32_t *cap) {
    if (A.n > 0) CLAUNCH(cl_ap_cap_kernel, cgrid(A.n), A, pptr, cap);
}
void cl_launch_rap_cap(hipStream_t s, int32_t nc, const int32_t *rptr, const int32_t *rcol, const int32_t *apptr,
                       int32_t *cap) {
    if (nc > 0) CLAUNCH(cl_rap_cap_kernel, cgrid(nc), nc, rptr, rcol, apptr, cap);
}
void cl_launch_chunk_sums(hipStream_t s, int32_t n, const int32_t *cap, int64_t *sums) {
    if (n > 0) CLAUNCH(cl_chunk_sum_kernel, (n + kClChunk - 1) / kClChunk, n, cap, sums);
}
void cl_launch_product(hipStream_t s, int32_t r0, int32_t r1, const Sell<double> *AX, const int32_t *xptr,
                       const int32_t *xcol, const double *xval, const int32_t *yptr, const int32_t *ycol,
                       const double *yval, const int32_t *cap, const int32_t *hoff, int32_t *hkey, double *hval,
                       bool fill, int32_t *rowlen, const int64_t *optr, bool sell_out, int32_t *ocol, double *oval,
                       int *overflow) {
    if (r1 <= r0) return;
    const int g = cgrid(r1 - r0);
    const Sell<double> ax = AX ? *AX : Sell<double>{};
    if (AX && !sell_out)
        CLAUNCH((cl_product_kernel<true, false>), g, r0, r1, ax, xptr, xcol, xval, yptr, ycol, yval, cap, hoff, hkey,
                hval, fill ? 1 : 0, rowlen, optr, ocol, oval, overflow);
    else if (!AX && sell_out)
        CLAUNCH((cl_product_kernel<false, true>), g, r0, r1, ax, xptr, xcol, xval, yptr, ycol, yval, cap, hoff, hkey,
                hval, fill ? 1 : 0, rowlen, optr, ocol, oval, overflow);
    else
        throw Error(VAG_ERR_ARG, "internal: unsupported sparse product layout");
}
void cl_launch_widen(hipStream_t s, int32_t n, const int32_t *in, int64_t *out) {
    CLAUNCH(cl_widen_kernel, cgrid((int64_t)n + 1), n, in, out);
}
template <class X>
void cl_launch_restrict(hipStream_t s, int32_t nc, const int32_t *rptr, const int32_t *rcol, const double *rval,
                        const X *r, X *bc, const X *dinv_c, X *xc, const PcgState *st) {
    if (nc > 0) CLAUNCH(cl_restrict_kernel<X>, cgrid(nc), nc, rptr, rcol, rval, r, bc, dinv_c, xc, st);
}
template <class X>
void cl_launch_prolong(hipStream_t s, int32_t n, const int32_t *pptr, const int32_t *pcol, const double *pval,
                       const X *x, const X *e, X *y, const PcgState *st) {
    if (n > 0) CLAUNCH(cl_prolong_kernel<X>, cgrid(n), n, pptr, pcol, pval, x, e, y, st);
}
template void cl_launch_restrict<double>(hipStream_t, int32_t, const int32_t *, const int32_t *, const double *,
                                         const double *, double *, const double *, double *, const PcgState *);
template void cl_launch_restrict<float>(hipStream_t, int32_t, const int32_t *, const int32_t *, const double *,
                                        const float *, float *, const float *, float *, const PcgState *);
template void cl_launch_prolong<double>(hipStream_t, int32_t, const int32_t *, const int32_t *, const double *,
                                        const double *, const double *, double *, const PcgState *);
template void cl_launch_prolong<float>(hipStream_t, int32_t, const int32_t *, const int32_t *, const double *,
                                       const float *, const float *, float *, const PcgState *);

}  // namespace vag
