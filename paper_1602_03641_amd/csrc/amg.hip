// Aggregation AMG for the SPD system of eq eqschur, set up on the device at
// every solve (the matrix values change with the permeabilities).
//
// Coarsening (one level):
//   strength   j is a strong neighbour of i if |a_ij| >= theta sqrt(|a_ii a_jj|)
//   roots      a distance-2 maximal independent set of the strength graph,
//              found by rounds of 2-hop max propagation of (state, hash, index)
//              keys; a fixed number of rounds, later rounds exit at once when
//              nothing is left undecided (no host synchronisation)
//   aggregates each root starts one; other nodes join their strongest root
//              neighbour, then the strongest already-aggregated neighbour
//   P          piecewise-constant interpolation (one 1 per row)
//   A_c        = P^T A P, one wavefront per coarse row: the (coarse column,
//              fine position) keys of the aggregate's rows are bitonic-sorted
//              in LDS and each coarse entry sums its fine entries in position
//              order, so the coarse matrix is bitwise reproducible
// Smoother: l1-Jacobi, M = diag(sum_j |a_ij|), convergent for any SPD matrix.
// Cycle: symmetric V-cycle (one pre- and one post-sweep), the coarsest level
// solved by a dense inverse formed on the device by Gauss-Jordan elimination.
#include <algorithm>

#include "amg.h"
#include "reduce.h"
#include "sell.h"

namespace vag {

constexpr int kAT = 256;
constexpr int kRzThreads = kKrylovThreads;  // the r.z sweep writes Krylov partials
constexpr int kCap = 8192;  // candidate entries per coarse row held in LDS

#define GS(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// full grid for the grid-stride kernels (no reduction partials)
static inline unsigned gridv(int64_t n) {
    const int64_t b = (n + kAT - 1) / kAT;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 20));
}

__device__ inline uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
__device__ inline int rank_of(uint64_t t) { return (int)(t >> 62); }

template <class V>
__device__ inline bool strong(const V *val, const int32_t *col, int64_t q, int32_t i, double di,
                              const double *diag, double theta, int32_t &j, double &s) {
    j = col[q];
    const double a = fabs((double)val[q]);
    if (j == i || a == 0.0) return false;
    const double dd = sqrt(fabs(di * diag[j]));
    s = a / dd;
    return a >= theta * dd;
}

// diag and l1-Jacobi inverse
__global__ __launch_bounds__(kAT) void amg_diag_kernel(Sell<double> A, double *__restrict__ diag,
                                                       double *__restrict__ dinv) {
    GS(i, A.n) {
        const int64_t b0 = A.ptr[i >> 6], b1 = A.ptr[(i >> 6) + 1];
        double d = 0.0, l1 = 0.0;
        for (int64_t q = b0 + (i & 63); q < b1; q += 64) {
            const double v = A.val[q];
            if (A.col[q] == i) d += v;
            l1 += fabs(v);
        }
        diag[i] = d;
        dinv[i] = 1.0 / l1;
    }
}

// strong[q] = 1 if entry q is a strong off-diagonal coupling
__global__ __launch_bounds__(kAT) void strength_kernel(Sell<double> A, const double *__restrict__ diag, double theta,
                                                       uint8_t *__restrict__ strongq) {
    GS(i, A.n) {
        const int64_t b0 = A.ptr[i >> 6], b1 = A.ptr[(i >> 6) + 1];
        const double di = diag[i];
        for (int64_t q = b0 + (i & 63); q < b1; q += 64) {
            int32_t j;
            double s;
            strongq[q] = strong(A.val, A.col, q, (int32_t)i, di, diag, theta, j, s) ? 1 : 0;
        }
    }
}

__global__ __launch_bounds__(kAT) void mis_init_kernel(int32_t n, uint64_t *__restrict__ T) {
    GS(i, n) T[i] = (1ull << 62) | ((uint64_t)(mix32((uint32_t)i) & 0x3fffffffu) << 32) | (uint64_t)(uint32_t)i;
}

// Tout[i] = max of T over {i} and its strong neighbours
__global__ __launch_bounds__(kAT) void mis_max_kernel(Sell<double> A, const uint8_t *__restrict__ strongq,
                                                      const uint64_t *__restrict__ Tin, uint64_t *__restrict__ Tout,
                                                      const int *__restrict__ active) {
    if (active && *active == 0) return;
    GS(i, A.n) {
        const int64_t b0 = A.ptr[i >> 6], b1 = A.ptr[(i >> 6) + 1];
        uint64_t m = Tin[i];
        for (int64_t q = b0 + (i & 63); q < b1; q += 64)
            if (strongq[q]) m = max(m, Tin[A.col[q]]);
        Tout[i] = m;
    }
}

// second hop, then the decision of undecided nodes
__global__ __launch_bounds__(kAT) void mis_select_kernel(Sell<double> A, const uint8_t *__restrict__ strongq,
                                                         const uint64_t *__restrict__ T1, uint64_t *__restrict__ T,
                                                         int *__restrict__ undecided, const int *__restrict__ active) {
    if (active && *active == 0) return;
    int cnt = 0;
    GS(i, A.n) {
        const uint64_t own = T[i];
        if (rank_of(own) != 1) continue;
        const int64_t b0 = A.ptr[i >> 6], b1 = A.ptr[(i >> 6) + 1];
        uint64_t m = T1[i];
        for (int64_t q = b0 + (i & 63); q < b1; q += 64)
            if (strongq[q]) m = max(m, T1[A.col[q]]);
        if (m == own)
            T[i] = (own & ~(3ull << 62)) | (2ull << 62);  // root
        else if (rank_of(m) == 2)
            T[i] = own & ~(3ull << 62);  // a root lies within distance 2
        else
            ++cnt;
    }
    if (cnt) atomicAdd(undecided, cnt);  // integer count, order-independent
}

// roots (and nodes left undecided) flagged 1
__global__ __launch_bounds__(kAT) void mis_flag_kernel(int32_t n, const uint64_t *__restrict__ T,
                                                       int32_t *__restrict__ flag) {
    GS(i, n) flag[i] = rank_of(T[i]) >= 1 ? 1 : 0;
}

__global__ __launch_bounds__(kAT) void agg_pass1_kernel(Sell<double> A, const double *__restrict__ diag, double theta,
                                                        const int32_t *__restrict__ root, const int32_t *__restrict__ rid,
                                                        int32_t *__restrict__ agg1) {
    GS(i, A.n) {
        if (root[i]) {
            agg1[i] = rid[i];
            continue;
        }
        const int64_t b0 = A.ptr[i >> 6], b1 = A.ptr[(i >> 6) + 1];
        const double di = diag[i];
        double best = -1.0;
        int32_t bj = -1;
        for (int64_t q = b0 + (i & 63); q < b1; q += 64) {
            int32_t j;
            double s;
            if (strong(A.val, A.col, q, (int32_t)i, di, diag, theta, j, s) && root[j] &&
                (s > best || (s == best && j < bj))) {
                best = s;
                bj = j;
            }
        }
        agg1[i] = bj >= 0 ? rid[bj] : -1;
    }
}

__global__ __launch_bounds__(kAT) void agg_pass2_kernel(Sell<double> A, const double *__restrict__ diag, double theta,
                                                        const int32_t *__restrict__ agg1, int32_t *__restrict__ agg,
                                                        int32_t *__restrict__ lonely) {
    GS(i, A.n) {
        int32_t a = agg1[i];
        if (a < 0) {
            const int64_t b0 = A.ptr[i >> 6], b1 = A.ptr[(i >> 6) + 1];
            const double di = diag[i];
            double best = -1.0;
            int32_t bj = -1;
            for (int64_t q = b0 + (i & 63); q < b1; q += 64) {
                int32_t j;
                double s;
                if (strong(A.val, A.col, q, (int32_t)i, di, diag, theta, j, s) && agg1[j] >= 0 &&
                    (s > best || (s == best && j < bj))) {
                    best = s;
                    bj = j;
                }
            }
            if (bj >= 0) a = agg1[bj];
        }
        agg[i] = a;
        lonely[i] = a < 0 ? 1 : 0;
    }
}

// nodes reached by neither pass become singleton aggregates after the roots
__global__ __launch_bounds__(kAT) void agg_lonely_kernel(int32_t n, const int32_t *__restrict__ lonely,
                                                         const int32_t *__restrict__ lid, const int32_t *__restrict__ nroot,
                                                         int32_t *__restrict__ agg) {
    GS(i, n) if (lonely[i]) agg[i] = *nroot + lid[i];
}

__global__ __launch_bounds__(kAT) void count_kernel(int32_t n, const int32_t *__restrict__ agg,
                                                    int32_t *__restrict__ cnt) {
    GS(i, n) atomicAdd(&cnt[agg[i]], 1);
}
__global__ __launch_bounds__(kAT) void members_fill_kernel(int32_t n, const int32_t *__restrict__ agg,
                                                           const int32_t *__restrict__ ptr, int32_t *__restrict__ cursor,
                                                           int32_t *__restrict__ rows) {
    GS(i, n) {
        const int32_t a = agg[i];
        rows[ptr[a] + atomicAdd(&cursor[a], 1)] = (int32_t)i;
    }
}
// members in ascending row order: the rank of each member is the number of
// smaller members (one wavefront per aggregate; atomic fill order is arbitrary)
__global__ __launch_bounds__(kAT) void members_rank_kernel(int32_t nc, const int32_t *__restrict__ ptr,
                                                           const int32_t *__restrict__ tmp, int32_t *__restrict__ rows) {
    const int lane = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t I = w0; I < nc; I += nw) {
        const int32_t b = ptr[I], e = ptr[I + 1];
        for (int32_t t = b + lane; t < e; t += 64) {
            const int32_t v = tmp[t];
            int32_t rank = 0;
            for (int32_t u = b; u < e; ++u) rank += tmp[u] < v;
            rows[b + rank] = v;
        }
    }
}

// exclusive scan of n ints in one block; out[n] = total
__global__ __launch_bounds__(1024) void scan_int_kernel(int32_t n, const int32_t *__restrict__ in,
                                                        int32_t *__restrict__ out) {
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int32_t chunk = (n + 1023) / 1024;
    const int32_t lo = min(n, t * chunk), hi = min(n, lo + chunk);
    int32_t s = 0;
    for (int32_t k = lo; k < hi; ++k) s += in[k];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int32_t run = 0;
        for (int k = 0; k < 1024; ++k) {
            const int32_t v = part[k];
            part[k] = run;
            run += v;
        }
        out[n] = run;
    }
    __syncthreads();
    int32_t run = part[t];
    for (int32_t k = lo; k < hi; ++k) {
        const int32_t v = in[k];
        out[k] = run;
        run += v;
    }
}


// multi-block exclusive scan of n ints (out[n] = total): block sums, one-block
// scan of the block sums, then per-block scan with offsets
constexpr int kScanItems = 4;
__global__ __launch_bounds__(256) void scan_sums_kernel(int32_t n, const int32_t *__restrict__ in,
                                                        int32_t *__restrict__ sums) {
    __shared__ int32_t w[4];
    const int64_t base = (int64_t)blockIdx.x * 256 * kScanItems;
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)k * 256 + threadIdx.x;
        if (i < n) s += in[i];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) sums[blockIdx.x] = w[0] + w[1] + w[2] + w[3];
}
__global__ __launch_bounds__(256) void scan_apply_kernel(int32_t n, const int32_t *__restrict__ in,
                                                         const int32_t *__restrict__ offs, int32_t *__restrict__ out) {
    __shared__ int32_t wsum[4];
    const int64_t base = (int64_t)blockIdx.x * 256 * kScanItems + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t t = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        t += v[k];
    }
    // inclusive scan of t over the block
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t incl = t;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int32_t off = offs[blockIdx.x];
    for (int k = 0; k < wv; ++k) off += wsum[k];
    int32_t run = off + incl - t;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (base + kScanItems >= n && base < n) out[n] = run;  // the thread holding the last element
}

// ---------------------------------------------------------------------------
// Galerkin coarse operator, one wavefront per coarse row
// ---------------------------------------------------------------------------
// Jcol[q] = aggregate of the column of entry q (same sliced-ELL layout as A)
__global__ __launch_bounds__(kAT) void agg_col_kernel(Sell<double> A, const int32_t *__restrict__ agg,
                                                      int32_t *__restrict__ Jcol) {
    GS(i, A.n) {
        const int64_t b0 = A.ptr[i >> 6], b1 = A.ptr[(i >> 6) + 1];
        for (int64_t q = b0 + (i & 63); q < b1; q += 64) Jcol[q] = agg[A.col[q]];
    }
}
// Row i of A P (P = aggregate indicator): the distinct aggregates of the row's
// columns, in increasing order, each with the sum of its entries (in entry
// order); the nonzero sums go to the row's first apn[i] slots of (apJ, apv).
// The lanes of a wave scan slot k together, so the passes are coalesced.  A
// row with more than kSet distinct aggregates is appended to the spill list
// and collapsed by ap_spill_kernel instead.
constexpr int kSet = 16;
__global__ __launch_bounds__(kAT) void ap_collapse_kernel(Sell<double> A, const int32_t *__restrict__ Jcol,
                                                          int32_t *__restrict__ apJ, double *__restrict__ apv,
                                                          int32_t *__restrict__ apn, int32_t *__restrict__ spill,
                                                          int *__restrict__ nspill) {
    GS(i, A.n) {
        const int64_t b0 = A.ptr[i >> 6] + (i & 63), b1 = A.ptr[(i >> 6) + 1];
        int32_t J[kSet];
        double v[kSet];
        int cnt = 0;
        bool over = false;
#pragma unroll
        for (int t = 0; t < kSet; ++t) {
            J[t] = INT32_MAX;
            v[t] = 0.0;
        }
        for (int64_t q = b0; q < b1 && !over; q += 64) {
            const double a = A.val[q];
            if (a == 0.0) continue;
            const int32_t c = Jcol[q];
            bool found = false;
#pragma unroll
            for (int t = 0; t < kSet; ++t)
                if (J[t] == c) {
                    v[t] += a;
                    found = true;
                }
            if (!found) {
                if (cnt == kSet) {
                    over = true;
                } else {
#pragma unroll
                    for (int t = 0; t < kSet; ++t)
                        if (t == cnt) {
                            J[t] = c;
                            v[t] = a;
                        }
                    ++cnt;
                }
            }
        }
        if (over) {
            spill[atomicAdd(nspill, 1)] = (int32_t)i;  // list order is irrelevant: rows are independent
            continue;
        }
        // ascending aggregate order (selection of the next larger key)
        int64_t out = b0;
        int32_t last = -1;
        int written = 0;
        for (int k = 0; k < cnt; ++k) {
            int32_t jm = INT32_MAX;
            double vm = 0.0;
#pragma unroll
            for (int t = 0; t < kSet; ++t)
                if (J[t] > last && J[t] < jm) {
                    jm = J[t];
                    vm = v[t];
                }
            last = jm;
            if (vm == 0.0) continue;
            apJ[out] = jm;
            apv[out] = vm;
            out += 64;
            ++written;
        }
        apn[i] = written;
    }
}

// The spilled rows of ap_collapse_kernel, one wavefront per row: the row's
// entries as keys (aggregate, slot) sorted in LDS, then one sum per run of
// equal aggregates in slot order (the order of the fast path).  Rows with more
// than CAP entries fall back to repeated minimum extraction by one lane.
template <int CAP>
__global__ __launch_bounds__(64) void ap_spill_kernel(Sell<double> A, const int32_t *__restrict__ Jcol,
                                                      int32_t *__restrict__ apJ, double *__restrict__ apv,
                                                      int32_t *__restrict__ apn, const int32_t *__restrict__ spill,
                                                      const int *__restrict__ nspill) {
    __shared__ uint64_t key[CAP];
    const int lane = threadIdx.x;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int ns = *nspill;
    for (int it = blockIdx.x; it < ns; it += gridDim.x) {
        const int32_t r = spill[it];
        const int64_t b0 = A.ptr[r >> 6] + (r & 63);
        const int w = (int)((A.ptr[(r >> 6) + 1] - A.ptr[r >> 6]) >> 6);
        int m = 0;
        for (int k0 = 0; k0 < w && m <= CAP; k0 += 64) {
            const int k = k0 + lane;
            bool keep = false;
            uint64_t kv = 0;
            if (k < w) {
                const int64_t q = b0 + (int64_t)k * 64;
                if (A.val[q] != 0.0) {
                    keep = true;
                    kv = ((uint64_t)(uint32_t)Jcol[q] << 32) | (uint64_t)(uint32_t)k;
                }
            }
            const uint64_t mask = __ballot(keep);
            const int off = __popcll(mask & below);
            if (keep && m + off < CAP) key[m + off] = kv;
            m += __popcll(mask);
        }
        if (m > CAP) {
            if (lane == 0) {
                int32_t last = -1;
                int written = 0;
                int64_t out = b0;
                for (;;) {
                    int32_t jm = INT32_MAX;
                    for (int k = 0; k < w; ++k) {
                        const int64_t q = b0 + (int64_t)k * 64;
                        const int32_t c = Jcol[q];
                        if (c > last && c < jm && A.val[q] != 0.0) jm = c;
                    }
                    if (jm == INT32_MAX) break;
                    double sum = 0.0;
                    for (int k = 0; k < w; ++k) {
                        const int64_t q = b0 + (int64_t)k * 64;
                        const double a = A.val[q];
                        if (a != 0.0 && Jcol[q] == jm) sum += a;
                    }
                    last = jm;
                    if (sum == 0.0) continue;
                    apJ[out] = jm;
                    apv[out] = sum;
                    out += 64;
                    ++written;
                }
                apn[r] = written;
            }
            __syncthreads();
            continue;
        }
        int mp = 1;
        while (mp < m) mp <<= 1;
        for (int k = m + lane; k < mp; k += 64) key[k] = ~0ull;
        __syncthreads();
        for (int k = 2; k <= mp; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = lane; i < mp; i += 64) {
                    const int p = i ^ j;
                    if (p > i) {
                        const uint64_t a = key[i], b = key[p];
                        const bool up = (i & k) == 0;
                        if ((a > b) == up) {
                            key[i] = b;
                            key[p] = a;
                        }
                    }
                }
                __syncthreads();
            }
        // runs of equal aggregates: lane-contiguous chunks, nonzero sums ranked by a wave scan
        const int C = (m + 63) / 64;
        const int lo = min(m, lane * C), hi = min(m, lo + C);
        int nh = 0;
        for (int t = lo; t < hi; ++t) {
            if (!(t == 0 || (key[t] >> 32) != (key[t - 1] >> 32))) continue;
            const uint32_t Jt = (uint32_t)(key[t] >> 32);
            double s = 0.0;
            for (int u = t; u < m && (uint32_t)(key[u] >> 32) == Jt; ++u) s += A.val[b0 + (int64_t)(uint32_t)key[u] * 64];
            nh += s != 0.0;
        }
        int incl = nh;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        int rank = incl - nh;
        for (int t = lo; t < hi; ++t) {
            if (!(t == 0 || (key[t] >> 32) != (key[t - 1] >> 32))) continue;
            const uint32_t Jt = (uint32_t)(key[t] >> 32);
            double s = 0.0;
            for (int u = t; u < m && (uint32_t)(key[u] >> 32) == Jt; ++u) s += A.val[b0 + (int64_t)(uint32_t)key[u] * 64];
            if (s == 0.0) continue;
            apJ[b0 + (int64_t)rank * 64] = (int32_t)Jt;
            apv[b0 + (int64_t)rank * 64] = s;
            ++rank;
        }
        if (lane == 63) apn[r] = incl;
        __syncthreads();
    }
}

// mode 0: rowlen[I] = number of coarse columns; mode 1: write them (SELL).
// Candidates are the collapsed entries (apn[r] of them) of the aggregate's
// rows r, gathered with one member row per lane.  Rows with more than CAP
// candidates set big[I] and are redone with the larger CAP.
template <int CAP>
__global__ __launch_bounds__(64) void galerkin_kernel(Sell<double> A, const int32_t *__restrict__ Jcol,
                                                      const double *__restrict__ apv, const int32_t *__restrict__ apn,
                                                      const int32_t *__restrict__ mptr, const int32_t *__restrict__ mrows,
                                                      int32_t nc, int mode, int32_t *__restrict__ big,
                                                      int32_t *__restrict__ rowlen, const int64_t *__restrict__ cptr,
                                                      int32_t *__restrict__ ccol, double *__restrict__ cval,
                                                      int *__restrict__ overflow) {
    __shared__ uint64_t key[CAP];
    const int32_t I = blockIdx.x;
    const int lane = threadIdx.x;
    if (I >= nc) return;
    if (CAP > 2048 && !big[I]) return;
    int m = 0;
    bool over = false;
    const int32_t t1 = mptr[I + 1];
    for (int32_t t0 = mptr[I]; t0 < t1; t0 += 64) {
        const int32_t t = t0 + lane;
        int c = 0;
        int64_t b = 0;
        if (t < t1) {
            const int32_t r = mrows[t];
            b = A.ptr[r >> 6] + (r & 63);
            c = apn[r];
        }
        int incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        const int tot = __shfl(incl, 63, 64);
        if (m + tot > CAP) {
            over = true;
            break;
        }
        const int off = m + incl - c;
        for (int k = 0; k < c; ++k) {
            const int64_t q = b + (int64_t)k * 64;
            key[off + k] = ((uint64_t)(uint32_t)Jcol[q] << 32) | (uint64_t)(uint32_t)q;
        }
        m += tot;
    }
    if (over) {
        if (lane == 0) {
            if (CAP <= 2048) big[I] = 1;
            else atomicOr(overflow, 1);
            if (mode == 0 && CAP > 2048) rowlen[I] = 1;
        }
        return;
    }
    if (CAP <= 2048 && mode == 0 && lane == 0) big[I] = 0;
    int mp = 1;
    while (mp < m) mp <<= 1;
    for (int k = m + lane; k < mp; k += 64) key[k] = ~0ull;
    __syncthreads();
    for (int k = 2; k <= mp; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < mp; i += 64) {
                const int p = i ^ j;
                if (p > i) {
                    const uint64_t a = key[i], b = key[p];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        key[i] = b;
                        key[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    const int C = mp / 64 > 0 ? mp / 64 : 1;
    const int lo = min(m, lane * C), hi = min(m, lo + C);
    int nh = 0;
    for (int t = lo; t < hi; ++t) nh += (t == 0 || (key[t] >> 32) != (key[t - 1] >> 32));
    int incl = nh;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    const int total = __shfl(incl, 63, 64);
    if (mode == 0) {
        if (lane == 0) rowlen[I] = total;
        return;
    }
    int rank = incl - nh;
    const int64_t base = cptr[I >> 6] + (I & 63);
    for (int t = lo; t < hi; ++t) {
        if (!(t == 0 || (key[t] >> 32) != (key[t - 1] >> 32))) continue;
        const uint32_t J = (uint32_t)(key[t] >> 32);
        double s = 0.0;
        for (int u = t; u < m && (uint32_t)(key[u] >> 32) == J; ++u) s += apv[(uint32_t)key[u]];
        ccol[base + (int64_t)rank * 64] = (int32_t)J;
        cval[base + (int64_t)rank * 64] = s;
        ++rank;
    }
    const int w = (int)((cptr[(I >> 6) + 1] - cptr[I >> 6]) >> 6);
    for (int k = total + lane; k < w; k += 64) {
        ccol[base + (int64_t)k * 64] = I;
        cval[base + (int64_t)k * 64] = 0.0;
    }
}

// slice widths (max row length of each 64-row slice)
__global__ __launch_bounds__(64) void slice_width_kernel(int32_t n, const int32_t *__restrict__ rowlen,
                                                         int32_t *__restrict__ width,
                                                         unsigned long long *__restrict__ nnz) {
    const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
    int c = i < n ? rowlen[i] : 0;
    int t = c;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        c = max(c, __shfl_down(c, o, 64));
        t += __shfl_down(t, o, 64);
    }
    if (threadIdx.x == 0) {
        width[blockIdx.x] = c;
        atomicAdd(nnz, (unsigned long long)t);  // integer count: order-independent
    }
}
// rows beyond n in the last slice: padding pointing at row 0
__global__ __launch_bounds__(64) void slice_tail_kernel(int32_t n, const int64_t *__restrict__ ptr,
                                                        int32_t *__restrict__ col, double *__restrict__ val) {
    const int32_t sl = n >> 6;
    const int lane = threadIdx.x;
    if ((n & 63) == 0 || lane < (n & 63)) return;
    for (int64_t q = ptr[sl] + lane; q < ptr[sl + 1]; q += 64) {
        col[q] = 0;
        val[q] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// coarsest level: dense inverse
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kAT) void dense_from_sell_kernel(Sell<double> A, double *__restrict__ D) {
    const int32_t n = A.n;
    GS(t, (int64_t)n * n) D[t] = 0.0;
}
__global__ __launch_bounds__(kAT) void dense_scatter_kernel(Sell<double> A, double *__restrict__ D) {
    GS(i, A.n) {
        const int64_t b0 = A.ptr[i >> 6], b1 = A.ptr[(i >> 6) + 1];
        for (int64_t q = b0 + (i & 63); q < b1; q += 64) D[i * A.n + A.col[q]] += A.val[q];
    }
}
// In-place blocked Gauss-Jordan inversion of an SPD matrix (no pivoting
// needed: every pivot block is a Schur complement of an SPD matrix, hence SPD).
// With P the next kGJ pivots, R the other indices and B = M[P,P]^-1 the block
// step is
//   M[P,P] = B,  M[P,R] = B M[P,R],  M[R,P] = -M[R,P] B,
//   M[R,R] = M[R,R] + M[R,P]_new M[P,R]_old,
// done by three kernels: the k x k inverse in LDS (one workgroup), the two
// panels (old M[P,R] saved aside), the rank-k update of M[R,R].
constexpr int kGJ = 64;

// B = M[P,P]^-1 (k <= kGJ), written back in place.  256 threads as a 16 x 16
// grid, each keeping a 4 x 4 tile of the (identity-padded) 64 x 64 block in
// registers; per pivot the owners publish the pivot column and row in LDS
// (double-buffered, one barrier per pivot).
__global__ __launch_bounds__(256) void gj_pivot_kernel(int32_t n, int32_t p0, int32_t k, double *__restrict__ M) {
    __shared__ double colp[2][kGJ], rowp[2][kGJ];
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    double t[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = ty * 4 + a, j = tx * 4 + c;
            // every lane loads (the padding from the block's first entry) so the
            // sixteen loads are in flight together
            const bool in = i < k && j < k;
            const double x = M[(int64_t)(p0 + (in ? i : 0)) * n + p0 + (in ? j : 0)];
            t[a][c] = in ? x : (i == j ? 1.0 : 0.0);
        }
    for (int p = 0; p < k; ++p) {
        const int buf = p & 1;
        // owners of column p and of row p publish them
        {
            const int q = p & 3;
            // the thread's entries in column p (one per tile row) and row p (one per tile column)
            double cv[4], rv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) cv[a] = q == 0 ? t[a][0] : q == 1 ? t[a][1] : q == 2 ? t[a][2] : t[a][3];
#pragma unroll
            for (int c = 0; c < 4; ++c) rv[c] = q == 0 ? t[0][c] : q == 1 ? t[1][c] : q == 2 ? t[2][c] : t[3][c];
            if (tx == (p >> 2)) {
#pragma unroll
                for (int a = 0; a < 4; ++a) colp[buf][ty * 4 + a] = cv[a];
            }
            if (ty == (p >> 2)) {
#pragma unroll
                for (int c = 0; c < 4; ++c) rowp[buf][tx * 4 + c] = rv[c];
            }
        }
        __syncthreads();
        const double pinv = 1.0 / colp[buf][p];
        double cp[4], rw[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) cp[a] = colp[buf][ty * 4 + a];
#pragma unroll
        for (int c = 0; c < 4; ++c) rw[c] = rowp[buf][tx * 4 + c];
        // branch-free: the sweep update everywhere, then row p, column p and
        // the pivot itself by selects
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const bool ip = (ty * 4 + a) == p;
            const double ca = cp[a] * pinv;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const bool jp = (tx * 4 + c) == p;
                const double upd = t[a][c] - ca * rw[c];
                const double rowv = rw[c] * pinv;
                t[a][c] = ip ? (jp ? pinv : rowv) : (jp ? -ca : upd);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = ty * 4 + a, j = tx * 4 + c;
            if (i < k && j < k) M[(int64_t)(p0 + i) * n + p0 + j] = t[a][c];
        }
}

// saves the panels: oc[l][t] = M[p0+l][t], orow[t][l] = M[t][p0+l] (t outside P)
__global__ __launch_bounds__(256) void gj_save_kernel(int32_t n, int32_t p0, int32_t k, const double *__restrict__ M,
                                                      double *__restrict__ oc, double *__restrict__ orow) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)n * k;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = e / k;
        const int l = (int)(e % k);
        if (t >= p0 && t < p0 + k) continue;
        oc[(int64_t)l * n + t] = M[(int64_t)(p0 + l) * n + t];
        orow[t * k + l] = M[t * n + p0 + l];
    }
}

// M[P,t] = B oc[.,t] and M[t,P] = -orow[t,.] B, one (t, l) pair per thread
__global__ __launch_bounds__(256) void gj_panel_kernel(int32_t n, int32_t p0, int32_t k, double *__restrict__ M,
                                                       const double *__restrict__ oc,
                                                       const double *__restrict__ orow) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)n * k;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = e / k;
        const int l = (int)(e % k);
        if (t >= p0 && t < p0 + k) continue;
        double sc = 0.0, sr = 0.0;
        for (int q = 0; q < k; ++q) {
            sc += M[(int64_t)(p0 + l) * n + p0 + q] * oc[(int64_t)q * n + t];
            sr += orow[t * k + q] * M[(int64_t)(p0 + q) * n + p0 + l];
        }
        M[(int64_t)(p0 + l) * n + t] = sc;
        M[t * n + p0 + l] = -sr;
    }
}

// M[i][j] += sum_l M[i][p0+l] oc[l][j] for i, j outside P
__global__ __launch_bounds__(256) void gj_update_kernel(int32_t n, int32_t p0, int32_t k, double *__restrict__ M,
                                                        const double *__restrict__ oc) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)n * n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, j = e % n;
        if ((i >= p0 && i < p0 + k) || (j >= p0 && j < p0 + k)) continue;
        double s = M[e];
        for (int l = 0; l < k; ++l) s += M[i * n + p0 + l] * oc[(int64_t)l * n + j];
        M[e] = s;
    }
}

// ---------------------------------------------------------------------------
// V-cycle kernels
// ---------------------------------------------------------------------------
// x = M^-1 b (first sweep from zero)
template <class X>
__global__ __launch_bounds__(kAT) void vc_scale_kernel(int32_t n, const X *__restrict__ dinv, const X *__restrict__ b,
                                                       X *__restrict__ x, const PcgState *st) {
    if (st && st->done) return;
    GS(i, n) x[i] = dinv[i] * b[i];
}
// r = b - A x
template <class V, class X>
__global__ __launch_bounds__(kAT) void vc_resid_kernel(Sell<V> A, const X *__restrict__ b, const X *__restrict__ x,
                                                       X *__restrict__ r, const PcgState *st) {
    if (st && st->done) return;
    GS(i, A.n) r[i] = b[i] - sell_row_apply<V, X>(A, (int32_t)i, [&](int32_t j) { return x[j]; });
}
// b_c[I] = sum of r over aggregate I: one wavefront per coarse row, members
// strided over the lanes and combined by a fixed shuffle tree
// With xc, also the first smoothing iterate of the coarse level, xc = D_c^-1 bc.
template <class X>
__global__ __launch_bounds__(kAT) void vc_restrict_kernel(int32_t nc, const int32_t *__restrict__ mptr,
                                                          const int32_t *__restrict__ mrows, const X *__restrict__ r,
                                                          X *__restrict__ bc, const X *__restrict__ dinv_c,
                                                          X *__restrict__ xc, const PcgState *st) {
    if (st && st->done) return;
    const int lane = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t I = w0; I < nc; I += nw) {
        X s = 0;
        for (int32_t t = mptr[I] + lane; t < mptr[I + 1]; t += 64) s += r[mrows[t]];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) {
            bc[I] = s;
            if (xc) xc[I] = dinv_c[I] * s;
        }
    }
}
// y = x + P e (injection from the aggregate)
template <class X>
__global__ __launch_bounds__(kAT) void vc_prolong_kernel(int32_t n, const X *__restrict__ x,
                                                         const int32_t *__restrict__ agg, const X *__restrict__ e,
                                                         X *__restrict__ y, const PcgState *st) {
    if (st && st->done) return;
    GS(i, n) y[i] = x[i] + e[agg[i]];
}
// out = y + M^-1 (b - A y); with rz, also the block partials of b . out (the
// CG scalar r.z when this is the last sweep of a V-cycle on level 0)
template <class V, class X>
__global__ __launch_bounds__(kRzThreads) void vc_sweep_kernel(Sell<V> A, const X *__restrict__ dinv, const X *__restrict__ b,
                                                       const X *__restrict__ y, X *__restrict__ out,
                                                       double *__restrict__ rz, const PcgState *st) {
    if (st && st->done) return;
    double v[1] = {0.0};
    GS(i, A.n) {
        const X s = sell_row_apply<V, X>(A, (int32_t)i, [&](int32_t j) { return y[j]; });
        const X o = y[i] + dinv[i] * (b[i] - s);
        out[i] = o;
        v[0] += (double)b[i] * (double)o;
    }
    if (rz) {
        block_reduce<OpSum, 1, kRzThreads>(v);
        if (threadIdx.x == 0) rz[blockIdx.x] = v[0];
    }
}
// prolongation and sweep in one pass (small levels): y = x + P e with
// x = D^-1 b formed on the fly, out = y + D^-1 (b - A y)
template <class V, class X>
__global__ __launch_bounds__(kAT) void vc_post_fused_kernel(Sell<V> A, const X *__restrict__ dinv,
                                                            const X *__restrict__ b, const int32_t *__restrict__ agg,
                                                            const X *__restrict__ e, X *__restrict__ out,
                                                            const PcgState *st) {
    if (st && st->done) return;
    GS(i, A.n) {
        const X s = sell_row_apply<V, X>(A, (int32_t)i, [&](int32_t j) { return dinv[j] * b[j] + e[agg[j]]; });
        const X yi = dinv[i] * b[i] + e[agg[i]];
        out[i] = yi + dinv[i] * (b[i] - s);
    }
}
// Small levels (at most kSmallRows rows): kG lanes per row, lane g taking the
// row's slots g, g + kG, ..., the kG partial sums combined by a fixed
// butterfly, so a row's gathers are spread over several lanes and fewer
// dependent loads sit on one lane.  The lanes of one slot index read
// consecutive rows (coalesced).  MODE 0: out = b - A x.  MODE 1: out = x +
// D^-1 (b - A x).  MODE 2: with y = D^-1 b + P e, out = y + D^-1 (b - A y).
// MODE 3: with y = x + P e, out = y + D^-1 (b - A y).
constexpr int kG = 4;
constexpr int kRowsPerWave = 64 / kG;
template <int MODE, class V, class X>
__global__ __launch_bounds__(kAT) void vc_small_kernel(Sell<V> A, const X *__restrict__ dinv,
                                                       const X *__restrict__ b, const X *__restrict__ x,
                                                       const int32_t *__restrict__ agg, const X *__restrict__ e,
                                                       X *__restrict__ out, const PcgState *st) {
    if (st && st->done) return;
    const int lane = threadIdx.x & 63;
    const int g = lane / kRowsPerWave, rr = lane % kRowsPerWave;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    auto f = [&](int32_t j) -> X {
        if constexpr (MODE <= 1) return x[j];
        else if constexpr (MODE == 2) return dinv[j] * b[j] + e[agg[j]];
        else return x[j] + e[agg[j]];
    };
    for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w * kRowsPerWave < A.n; w += nw) {
        const int32_t i = (int32_t)(w * kRowsPerWave) + rr;
        X s0 = 0, s1 = 0;
        if (i < A.n) {
            const int64_t b1 = A.ptr[(i >> 6) + 1];
            int64_t q = A.ptr[i >> 6] + (i & 63) + (int64_t)g * 64;
            for (; q + kG * 64 < b1; q += 2 * kG * 64) {
                s0 += (X)A.val[q] * f(A.col[q]);
                s1 += (X)A.val[q + kG * 64] * f(A.col[q + kG * 64]);
            }
            if (q < b1) s0 += (X)A.val[q] * f(A.col[q]);
        }
        X sum = s0 + s1;
#pragma unroll
        for (int o = kRowsPerWave; o < 64; o <<= 1) sum += __shfl_xor(sum, o, 64);
        if (g == 0 && i < A.n) {
            if constexpr (MODE == 0) {
                out[i] = b[i] - sum;
            } else {
                X yi;
                if constexpr (MODE == 1) yi = x[i];
                else if constexpr (MODE == 2) yi = dinv[i] * b[i] + e[agg[i]];
                else yi = x[i] + e[agg[i]];
                out[i] = yi + dinv[i] * (b[i] - sum);
            }
        }
    }
}
static inline unsigned grid_small(int32_t n) {
    return (unsigned)std::max<int64_t>(1, ((int64_t)n * kG + kAT - 1) / kAT);
}

// dense coarse solve x = Ainv b: one wavefront per row, lanes along the
// (contiguous) row, fixed-order wave reduction
template <class X>
__global__ __launch_bounds__(kAT) void vc_dense_kernel(int32_t n, const X *__restrict__ Ainv, const X *__restrict__ b,
                                                       X *__restrict__ x, const PcgState *st) {
    if (st && st->done) return;
    const int lane = threadIdx.x & 63;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n;
         i += ((int64_t)gridDim.x * blockDim.x) >> 6) {
        double s = 0.0;
        for (int32_t j = lane; j < n; j += 64) s += (double)Ainv[i * n + j] * (double)b[j];
        s = wave_reduce<OpSum>(s);
        if (lane == 0) x[i] = (X)s;
    }
}
// conversions for the single-precision hierarchy
__global__ __launch_bounds__(kAT) void to_float_kernel(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
    GS(i, n) b[i] = (float)a[i];
}
__global__ __launch_bounds__(kAT) void to_double_kernel(int64_t n, const float *__restrict__ a, double *__restrict__ b) {
    GS(i, n) b[i] = (double)a[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define ALAUNCH(kern, grid, block, ...)                                              \
    do {                                                                             \
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, __VA_ARGS__);        \
        VAG_HIP(hipGetLastError());                                                  \
    } while (0)

void amg_launch_diag(hipStream_t s, Sell<double> A, double *diag, double *dinv) {
    if (A.n > 0) ALAUNCH(amg_diag_kernel, gridv(A.n), kAT, A, diag, dinv);
}
void amg_launch_mis(hipStream_t s, Sell<double> A, const double *diag, double theta, int rounds, uint64_t *T,
                    uint64_t *T1, int *undecided /* [rounds] zeroed */, int32_t *flag, int32_t *hpin,
                    uint8_t *strongq) {
    ALAUNCH(strength_kernel, gridv(A.n), kAT, A, diag, theta, strongq);
    ALAUNCH(mis_init_kernel, gridv(A.n), kAT, A.n, T);
    for (int r = 0; r < rounds; ++r) {
        const int *active = r ? undecided + r - 1 : nullptr;
        ALAUNCH(mis_max_kernel, gridv(A.n), kAT, A, strongq, T, T1, active);
        ALAUNCH(mis_select_kernel, gridv(A.n), kAT, A, strongq, T1, T, undecided + r, active);
        if ((r & 3) == 3 && r + 1 < rounds) {  // stop queueing rounds once nothing is undecided
            VAG_HIP(hipMemcpyAsync(hpin, undecided + r, sizeof(int), hipMemcpyDeviceToHost, s));
            VAG_HIP(hipStreamSynchronize(s));
            if (*hpin == 0) break;
        }
    }
    ALAUNCH(mis_flag_kernel, gridv(A.n), kAT, A.n, T, flag);
}
void amg_launch_scan(hipStream_t s, int32_t n, const int32_t *in, int32_t *out, int32_t *tmp) {
    // tmp: at least 2 * (n / 1024 + 2) ints
    const int32_t nb = (n + 256 * kScanItems - 1) / (256 * kScanItems);
    if (nb <= 1) {
        ALAUNCH(scan_int_kernel, 1, 1024, n, in, out);
        return;
    }
    ALAUNCH(scan_sums_kernel, nb, 256, n, in, tmp);
    ALAUNCH(scan_int_kernel, 1, 1024, nb, tmp, tmp + nb + 1);
    ALAUNCH(scan_apply_kernel, nb, 256, n, in, tmp + nb + 1, out);
}
void amg_launch_aggregate(hipStream_t s, Sell<double> A, const double *diag, double theta, const int32_t *root,
                          const int32_t *rid, int32_t *agg1, int32_t *agg, int32_t *lonely) {
    ALAUNCH(agg_pass1_kernel, gridv(A.n), kAT, A, diag, theta, root, rid, agg1);
    ALAUNCH(agg_pass2_kernel, gridv(A.n), kAT, A, diag, theta, agg1, agg, lonely);
}
void amg_launch_lonely(hipStream_t s, int32_t n, const int32_t *lonely, const int32_t *lid, const int32_t *nroot,
                       int32_t *agg) {
    ALAUNCH(agg_lonely_kernel, gridv(n), kAT, n, lonely, lid, nroot, agg);
}
void amg_launch_members(hipStream_t s, int32_t n, int32_t nc, const int32_t *agg, int32_t *cnt, int32_t *ptr,
                        int32_t *cursor, int32_t *tmp, int32_t *rows, int32_t *scan_tmp) {
    // cnt and cursor zeroed by the caller
    ALAUNCH(count_kernel, gridv(n), kAT, n, agg, cnt);
    amg_launch_scan(s, nc, cnt, ptr, scan_tmp);
    ALAUNCH(members_fill_kernel, gridv(n), kAT, n, agg, ptr, cursor, tmp);
    ALAUNCH(members_rank_kernel, reduce_grid((int64_t)nc * 64, kAT), kAT, nc, ptr, tmp, rows);
}
void amg_launch_collapse(hipStream_t s, Sell<double> A, const int32_t *agg, int32_t *Jcol, int32_t *apJ,
                         double *apv, int32_t *apn, int32_t *spill, int *nspill) {
    ALAUNCH(agg_col_kernel, gridv(A.n), kAT, A, agg, Jcol);
    ALAUNCH(ap_collapse_kernel, gridv(A.n), kAT, A, Jcol, apJ, apv, apn, spill, nspill);
    ALAUNCH(ap_spill_kernel<1024>, 2048, 64, A, Jcol, apJ, apv, apn, spill, nspill);
}
void amg_launch_galerkin(hipStream_t s, Sell<double> A, const int32_t *Jcol, const double *apv, const int32_t *apn,
                         const int32_t *mptr, const int32_t *mrows, int32_t nc, int mode, int32_t *big,
                         int32_t *rowlen, const int64_t *cptr, int32_t *ccol, double *cval, int *overflow) {
    if (nc <= 0) return;
    ALAUNCH(galerkin_kernel<2048>, nc, 64, A, Jcol, apv, apn, mptr, mrows, nc, mode, big, rowlen, cptr, ccol, cval,
            overflow);
    ALAUNCH(galerkin_kernel<8192>, nc, 64, A, Jcol, apv, apn, mptr, mrows, nc, mode, big, rowlen, cptr, ccol, cval,
            overflow);
}
void amg_launch_slices(hipStream_t s, int32_t n, const int32_t *rowlen, int32_t *width, int64_t *ptr,
                       unsigned long long *nnz) {
    const int32_t ns = (n + 63) / 64;
    if (ns > 0) ALAUNCH(slice_width_kernel, ns, 64, n, rowlen, width, nnz);
    launch_slice_scan(s, ns, width, ptr);
}
void amg_launch_slice_tail(hipStream_t s, int32_t n, const int64_t *ptr, int32_t *col, double *val) {
    if (n & 63) ALAUNCH(slice_tail_kernel, 1, 64, n, ptr, col, val);
}
void amg_launch_dense_inverse(hipStream_t s, Sell<double> A, double *D, double *work) {
    const int32_t n = A.n;
    ALAUNCH(dense_from_sell_kernel, gridv((int64_t)n * n), kAT, A, D);
    ALAUNCH(dense_scatter_kernel, gridv(n), kAT, A, D);
    const unsigned gu = (unsigned)std::min<int64_t>(((int64_t)n * n + 255) / 256, 4096);
    const unsigned gp = (unsigned)std::min<int64_t>(((int64_t)n * kGJ + 255) / 256, 4096);
    double *oc = work, *orow = work + (int64_t)kGJ * n;
    for (int32_t p0 = 0; p0 < n; p0 += kGJ) {
        const int32_t k = std::min(kGJ, n - p0);
        ALAUNCH(gj_pivot_kernel, 1, 256, n, p0, k, D);
        ALAUNCH(gj_save_kernel, gp, 256, n, p0, k, D, oc, orow);
        ALAUNCH(gj_panel_kernel, gp, 256, n, p0, k, D, oc, orow);
        ALAUNCH(gj_update_kernel, gu, 256, n, p0, k, D, oc);
    }
}
template <class V, class X>
void amg_launch_pre(hipStream_t s, Sell<V> A, const X *dinv, const X *b, X *x, X *r, const PcgState *st) {
    ALAUNCH(vc_scale_kernel<X>, gridv(A.n), kAT, A.n, dinv, b, x, st);
    amg_launch_resid<V, X>(s, A, b, x, r, st);
}
template <class X>
void amg_launch_restrict(hipStream_t s, int32_t nc, const int32_t *mptr, const int32_t *mrows, const X *r, X *bc,
                         const X *dinv_c, X *xc, const PcgState *st) {
    ALAUNCH(vc_restrict_kernel<X>, gridv((int64_t)nc * 64), kAT, nc, mptr, mrows, r, bc, dinv_c, xc, st);
}
template <class V, class X>
void amg_launch_resid(hipStream_t s, Sell<V> A, const X *b, const X *x, X *r, const PcgState *st) {
    if (A.n <= kSmallRows)
        ALAUNCH((vc_small_kernel<0, V, X>), grid_small(A.n), kAT, A, (const X *)nullptr, b, x, (const int32_t *)nullptr,
                (const X *)nullptr, r, st);
    else
        ALAUNCH((vc_resid_kernel<V, X>), gridv(A.n), kAT, A, b, x, r, st);
}
template <class V, class X>
void amg_launch_post_fused(hipStream_t s, Sell<V> A, const X *dinv, const X *b, const int32_t *agg, const X *e,
                           X *out, const PcgState *st) {
    if (A.n <= kSmallRows)
        ALAUNCH((vc_small_kernel<2, V, X>), grid_small(A.n), kAT, A, dinv, b, (const X *)nullptr, agg, e, out, st);
    else
        ALAUNCH((vc_post_fused_kernel<V, X>), gridv(A.n), kAT, A, dinv, b, agg, e, out, st);
}
template <class V, class X>
void amg_launch_post_x(hipStream_t s, Sell<V> A, const X *dinv, const X *b, const X *x, const int32_t *agg,
                       const X *e, X *out, const PcgState *st) {
    ALAUNCH((vc_small_kernel<3, V, X>), grid_small(A.n), kAT, A, dinv, b, x, agg, e, out, st);
}
template <class V, class X>
void amg_launch_post(hipStream_t s, Sell<V> A, const X *dinv, const X *b, const X *x, const int32_t *agg, const X *e,
                     X *y, X *out, double *rz, const PcgState *st) {
    ALAUNCH(vc_prolong_kernel<X>, gridv(A.n), kAT, A.n, x, agg, e, y, st);
    // with rz the partials must match the Krylov kernels' grid and block size
    if (rz)
        ALAUNCH((vc_sweep_kernel<V, X>), reduce_grid(A.n, kRzThreads), kRzThreads, A, dinv, b, y, out, rz, st);
    else
        ALAUNCH((vc_sweep_kernel<V, X>), gridv(A.n), kAT, A, dinv, b, y, out, nullptr, st);
}
template <class X>
void amg_launch_dense(hipStream_t s, int32_t n, const X *Ainv, const X *b, X *x, const PcgState *st) {
    ALAUNCH(vc_dense_kernel<X>, gridv((int64_t)n * 64), kAT, n, Ainv, b, x, st);
}
template <class V, class X>
void amg_launch_sweep(hipStream_t s, Sell<V> A, const X *dinv, const X *b, const X *x, X *out, const PcgState *st) {
    if (A.n <= kSmallRows)
        ALAUNCH((vc_small_kernel<1, V, X>), grid_small(A.n), kAT, A, dinv, b, x, (const int32_t *)nullptr,
                (const X *)nullptr, out, st);
    else
        ALAUNCH((vc_sweep_kernel<V, X>), gridv(A.n), kAT, A, dinv, b, x, out, nullptr, st);
}
void launch_to_float(hipStream_t s, int64_t n, const double *a, float *b) {
    if (n > 0) ALAUNCH(to_float_kernel, gridv(n), kAT, n, a, b);
}
void launch_to_double(hipStream_t s, int64_t n, const float *a, double *b) {
    if (n > 0) ALAUNCH(to_double_kernel, gridv(n), kAT, n, a, b);
}

#define VC_INST(V, X)                                                                                            \
    template void amg_launch_pre<V, X>(hipStream_t, Sell<V>, const X *, const X *, X *, X *, const PcgState *);    \
    template void amg_launch_resid<V, X>(hipStream_t, Sell<V>, const X *, const X *, X *, const PcgState *);       \
    template void amg_launch_post<V, X>(hipStream_t, Sell<V>, const X *, const X *, const X *, const int32_t *,    \
                                        const X *, X *, X *, double *, const PcgState *);                          \
    template void amg_launch_post_fused<V, X>(hipStream_t, Sell<V>, const X *, const X *, const int32_t *,         \
                                              const X *, X *, const PcgState *);                                   \
    template void amg_launch_post_x<V, X>(hipStream_t, Sell<V>, const X *, const X *, const X *, const int32_t *,  \
                                          const X *, X *, const PcgState *);                                       \
    template void amg_launch_sweep<V, X>(hipStream_t, Sell<V>, const X *, const X *, const X *, X *,               \
                                         const PcgState *);
VC_INST(double, double)
VC_INST(float, double)
VC_INST(float, float)
template void amg_launch_restrict<double>(hipStream_t, int32_t, const int32_t *, const int32_t *, const double *,
                                          double *, const double *, double *, const PcgState *);
template void amg_launch_restrict<float>(hipStream_t, int32_t, const int32_t *, const int32_t *, const float *,
                                         float *, const float *, float *, const PcgState *);
template void amg_launch_dense<double>(hipStream_t, int32_t, const double *, const double *, double *,
                                       const PcgState *);
template void amg_launch_dense<float>(hipStream_t, int32_t, const float *, const float *, float *, const PcgState *);
}  // namespace vag
