// Aggregation AMG for the SPD system of eq eqschur, set up on the device at
// every solve (the matrix values change with the permeabilities).
//
// Coarsening (one level):
//   strength   j is a strong neighbour of i if |a_ij| >= theta sqrt(|a_ii a_jj|)
//   roots      a distance-2 maximal independent set of the strength graph,
//              found by rounds of 2-hop max propagation of (state, priority)
//              keys, the priority a bijective hash of the row index; later
//              rounds exit at once when nothing is left undecided (the host
//              looks every fourth round)
//   aggregates each root starts one; other nodes join their strongest root
//              neighbour, then the strongest already-aggregated neighbour
//   P          piecewise-constant interpolation (one 1 per row)
//   A_c        = P^T A P, one wavefront per coarse row: the rows of A P
//              (each fine row's entries collapsed per aggregate) of the
//              aggregate's members are gathered as (coarse column, gather
//              ordinal) keys with their values in LDS, bitonic-sorted, and
//              each coarse entry sums its candidates in gather order, so the
//              coarse matrix is bitwise reproducible
// Smoother: l1-Jacobi, M = diag(sum_j |a_ij|), convergent for any SPD matrix.
// Cycle: symmetric V-cycle (one pre- and one post-sweep on the finest level,
// `sweeps` of each on the coarser ones), the coarsest level
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
    for (int64_t i = (int64_t)xcd_block() * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// full grid for the grid-stride kernels (no reduction partials)
static inline unsigned gridv(int64_t n) {
    const int64_t b = (n + kAT - 1) / kAT;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 20));
}

// A bijection of [0, 2^30): odd multipliers and right xor-shifts are each
// invertible modulo 2^30, so distinct rows get distinct priorities.
__device__ inline uint32_t perm30(uint32_t x) {
    constexpr uint32_t kM = (1u << 30) - 1;
    x &= kM;
    x = (x * 0x2c1b3c6du) & kM;
    x ^= x >> 15;
    x = (x * 0x297a2d39u) & kM;
    x ^= x >> 13;
    return x;
}
// MIS keys: state in the top two bits (2 root, 1 undecided, 0 out), the
// row's priority below
__device__ inline int rank_of(uint32_t t) { return (int)(t >> 30); }

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

// scol[q] = column of entry q if it is a strong off-diagonal coupling, else
// the row itself (so the MIS passes gather without branches: a row's own key
// never changes a maximum that already includes it)
__global__ __launch_bounds__(kAT) void strength_kernel(Sell<double> A, const double *__restrict__ diag, double theta,
                                                       int32_t *__restrict__ scol) {
    GS(i, A.n) {
        const int64_t b0 = A.ptr[i >> 6], b1 = A.ptr[(i >> 6) + 1];
        const double di = diag[i];
        for (int64_t q = b0 + (i & 63); q < b1; q += 64) {
            int32_t j;
            double s;
            scol[q] = strong(A.val, A.col, q, (int32_t)i, di, diag, theta, j, s) ? j : (int32_t)i;
        }
    }
}

__global__ __launch_bounds__(kAT) void mis_init_kernel(int32_t n, uint32_t *__restrict__ T, uint32_t *__restrict__ T1) {
    GS(i, n) {
        T[i] = (1u << 30) | perm30((uint32_t)i);
        T1[i] = 1u << 30;  // rank 1: computed in the first round
    }
}

// max of key[] over row i and its strong neighbours, four gathers in flight
__device__ inline uint32_t strong_max(const int64_t *__restrict__ ptr, const int32_t *__restrict__ scol, int32_t i,
                                      const uint32_t *__restrict__ key) {
    const int64_t b1 = ptr[(i >> 6) + 1];
    int64_t q = ptr[i >> 6] + (i & 63);
    uint32_t m0 = key[i], m1 = 0, m2 = 0, m3 = 0;
    for (; q + 192 < b1; q += 256) {
        m0 = max(m0, key[scol[q]]);
        m1 = max(m1, key[scol[q + 64]]);
        m2 = max(m2, key[scol[q + 128]]);
        m3 = max(m3, key[scol[q + 192]]);
    }
    for (; q < b1; q += 64) m0 = max(m0, key[scol[q]]);
    return max(max(m0, m1), max(m2, m3));
}

// Per-round counts of undecided rows, spread over kCntSlots counters 128 bytes
// apart: device-wide atomics on one address serialise, and thousands of
// blocks adding to a single counter cost more than the round itself.
__device__ inline bool any_count(const int *__restrict__ c) {
    const int lane = threadIdx.x & 63;
    const int v = lane < kCntSlots ? c[lane * kCntStride] : 0;
    return __ballot(v != 0) != 0;
}

// Tout[i] = max of T over {i} and its strong neighbours, recomputed only
// where the previous round's maximum had rank 1 (an undecided row among
// them).  Rank 0: every row of the set was decided, and decided keys never
// change, so the value is still exact.  Rank 2: a root among them, which stays
// a root, so the maximum still has rank 2; the selection asks of a maximum
// only whether it has rank 2 or, having rank 1, equals an undecided row's own
// key, so its decisions are those of the full recomputation.  The later
// rounds then touch only the rows next to the undecided ones.
__global__ __launch_bounds__(kAT) void mis_max_kernel(int32_t n, const int64_t *__restrict__ ptr,
                                                      const int32_t *__restrict__ scol, const uint32_t *__restrict__ Tin,
                                                      uint32_t *__restrict__ Tout, const int *__restrict__ active) {
    if (active && !any_count(active)) return;
    GS(i, n) {
        if (rank_of(Tout[i]) != 1) continue;
        Tout[i] = strong_max(ptr, scol, (int32_t)i, Tin);
    }
}

// second hop, then the decision of undecided nodes
__global__ __launch_bounds__(kAT) void mis_select_kernel(int32_t n, int hops, const int64_t *__restrict__ ptr,
                                                         const int32_t *__restrict__ scol,
                                                         const uint32_t *__restrict__ T1, uint32_t *__restrict__ T,
                                                         int *__restrict__ undecided, const int *__restrict__ active) {
    __shared__ int wc[kAT / 64];
    if (active && !any_count(active)) return;  // uniform over the block: every wave reads the same counters
    int cnt = 0;
    GS(i, n) {
        const uint32_t own = T[i];
        if (rank_of(own) != 1) continue;
        // two hops: the maximum over the neighbours of the one-hop maxima; one
        // hop: the one-hop maximum itself
        const uint32_t m = hops == 2 ? strong_max(ptr, scol, (int32_t)i, T1) : T1[i];
        if (m == own)
            T[i] = (own & ((1u << 30) - 1)) | (2u << 30);  // root
        else if (rank_of(m) == 2)
            T[i] = own & ((1u << 30) - 1);  // a root lies within distance 2
        else
            ++cnt;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kAT / 64; ++w) t += wc[w];
        if (t) atomicAdd(undecided + (blockIdx.x % kCntSlots) * kCntStride, t);  // integer count, order-independent
    }
}

// roots (and nodes left undecided) flagged 1
__global__ __launch_bounds__(kAT) void mis_flag_kernel(int32_t n, const uint32_t *__restrict__ T,
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
    const int64_t w0 = ((int64_t)xcd_block() * blockDim.x + threadIdx.x) >> 6;
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

// Galerkin coarse row I, one wavefront: the collapsed entries (apn[r] of
// them) of the aggregate's rows r are gathered as (coarse column, value) in
// gather order, one member row per lane; the distinct columns are found with
// an LDS hash set, ranked (each rank counts the smaller columns), and each
// column sums its candidates in gather order (all lanes read candidate k
// together), so the coarse matrix is bitwise reproducible.  mode 0:
// rowlen[I] = number of coarse columns, big[I] = 1 for a row this kernel
// cannot hold; mode 1: write the row (SELL).
constexpr int kGalCand = 1024, kGalHash = 512, kGalDistinct = 256;
__global__ __launch_bounds__(64) void galerkin_hash_kernel(Sell<double> A, const int32_t *__restrict__ Jcol,
                                                           const double *__restrict__ apv,
                                                           const int32_t *__restrict__ apn,
                                                           const int32_t *__restrict__ mptr,
                                                           const int32_t *__restrict__ mrows, int32_t nc, int mode,
                                                           int32_t *__restrict__ big, int32_t *__restrict__ rowlen,
                                                           const int64_t *__restrict__ cptr,
                                                           int32_t *__restrict__ ccol, double *__restrict__ cval) {
    __shared__ int32_t cj[kGalCand];
    __shared__ double cv[kGalCand];
    __shared__ int32_t hs[kGalHash];
    __shared__ int32_t dist[kGalDistinct];
    __shared__ int32_t sorted[kGalDistinct];
    const int32_t I = blockIdx.x;
    const int lane = threadIdx.x;
    if (I >= nc) return;
    if (mode == 1 && big[I]) return;
    for (int k = lane; k < kGalHash; k += 64) hs[k] = -1;
    // gather
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
        if (m + tot > kGalCand) {
            over = true;
            break;
        }
        const int off = m + incl - c;
        for (int k = 0; k < c; ++k) {
            const int64_t q = b + (int64_t)k * 64;
            cj[off + k] = Jcol[q];
            cv[off + k] = apv[q];
        }
        m += tot;
    }
    __syncthreads();
    // distinct columns: an LDS hash set (linear probing); a set that grows
    // past kGalDistinct sends the row to the sorting kernel
    bool full = false;
    if (!over) {
        for (int k = lane; k < m; k += 64) {
            const int32_t J = cj[k];
            uint32_t h = ((uint32_t)J * 2654435761u) & (kGalHash - 1);
            for (int probe = 0; probe < kGalHash; ++probe) {
                const int32_t prev = atomicCAS(&hs[h], -1, J);
                if (prev == -1 || prev == J) break;
                h = (h + 1) & (kGalHash - 1);
            }
        }
    }
    __syncthreads();
    int nd = 0;
    if (!over) {
        // compact the occupied slots
        for (int k0 = 0; k0 < kGalHash; k0 += 64) {
            const int32_t J = hs[k0 + lane];
            const uint64_t mask = __ballot(J >= 0);
            const int below = __popcll(mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
            const int base = nd;
            if (J >= 0 && base + below < kGalDistinct) dist[base + below] = J;
            nd += __popcll(mask);
        }
        full = nd > kGalDistinct;
    }
    if (over || full) {
        if (mode == 0 && lane == 0) big[I] = 1;
        return;
    }
    if (mode == 0 && lane == 0) big[I] = 0;
    __syncthreads();
    // rank sort of the distinct columns
    for (int i = lane; i < nd; i += 64) {
        const int32_t J = dist[i];
        int rank = 0;
        for (int u = 0; u < nd; ++u) rank += dist[u] < J;
        sorted[rank] = J;
    }
    if (mode == 0) {
        if (lane == 0) rowlen[I] = nd;
        return;
    }
    __syncthreads();
    // sums in gather order; lane owns sorted columns lane, lane + 64, ...
    constexpr int kOwn = kGalDistinct / 64;
    int32_t own[kOwn];
    double sum[kOwn];
#pragma unroll
    for (int o = 0; o < kOwn; ++o) {
        own[o] = (lane + 64 * o < nd) ? sorted[lane + 64 * o] : -1;
        sum[o] = 0.0;
    }
    const int nown = (nd + 63) / 64;
    for (int k = 0; k < m; ++k) {
        const int32_t J = cj[k];
        const double v = cv[k];
#pragma unroll
        for (int o = 0; o < kOwn; ++o)
            if (o < nown && own[o] == J) sum[o] += v;
    }
    const int64_t base = cptr[I >> 6] + (I & 63);
#pragma unroll
    for (int o = 0; o < kOwn; ++o) {
        const int k = lane + 64 * o;
        if (k < nd) {
            ccol[base + (int64_t)k * 64] = own[o];
            cval[base + (int64_t)k * 64] = sum[o];
        }
    }
    const int w = (int)((cptr[(I >> 6) + 1] - cptr[I >> 6]) >> 6);
    for (int k = nd + lane; k < w; k += 64) {
        ccol[base + (int64_t)k * 64] = I;
        cval[base + (int64_t)k * 64] = 0.0;
    }
}

// Coarse rows that the hashed kernel below could not take (more than
// kGalCand candidates or kGalDistinct distinct columns; big[I] set): the
// candidates as (coarse column, fine position) keys, bitonic-sorted in LDS,
// each coarse entry summing its candidates in gather order.  mode 0:
// rowlen[I] = number of coarse columns; mode 1: write them (SELL).  More
// than CAP candidates: *overflow.
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
    if (!big[I]) return;
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
            atomicOr(overflow, 1);
            if (mode == 0) rowlen[I] = 1;
        }
        return;
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
                                                         int32_t *__restrict__ width, int32_t *__restrict__ cnt) {
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
        cnt[blockIdx.x] = t;
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
// With P the next kGJ indices, R the others and B = M[P,P]^-1 the block step
// is
//   V = B M[P,R],  W = M[R,P] B,
//   M[R,R] = M[R,R] - M[R,P] V,  M[P,R] = V,  M[R,P] = -W,  M[P,P] = B,
// done by four kernels: the kGJ x kGJ inverse in one workgroup, the two
// panels V and W (64 x 64 tiles in LDS), the update of M[R,R] (64 x 64
// output tiles, the operands staged in LDS), and the write-back of the
// panels.  Only M[P,*] and M[*,P] are read before the write-back, so the
// update needs no copy of the old panels.
constexpr int kGJ = 64;
constexpr int kQ = 4;  // pivots eliminated together inside the diagonal block

// B = M[P,P]^-1 (k <= kGJ), written back in place.  256 threads as a 16 x 16
// grid, each keeping a 4 x 4 tile of the (identity-padded) 64 x 64 block in
// registers.  The elimination takes kQ pivots per step: the owners publish
// the kQ pivot rows and columns in LDS (double-buffered, one barrier per
// step), every thread inverts the kQ x kQ pivot block itself and updates its
// tile by the block rule above, restricted to the diagonal block.
__device__ inline void inv4(double b[kQ][kQ]) {
#pragma unroll
    for (int p = 0; p < kQ; ++p) {
        const double pinv = 1.0 / b[p][p];
        double pr[kQ];  // the pivot row before this step
#pragma unroll
        for (int j = 0; j < kQ; ++j) pr[j] = b[p][j];
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const double ca = b[i][p] * pinv;
#pragma unroll
            for (int j = 0; j < kQ; ++j)
                b[i][j] = (i == p) ? (j == p ? pinv : pr[j] * pinv) : (j == p ? -ca : b[i][j] - ca * pr[j]);
        }
    }
}
__global__ __launch_bounds__(256) void gj_pivot_kernel(int32_t n, int32_t p0, int32_t k, double *__restrict__ M) {
    __shared__ double rowp[2][kQ][kGJ], colp[2][kGJ][kQ];
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
    const int nsteps = (k + kQ - 1) / kQ;
    for (int pb = 0; pb < nsteps; ++pb) {
        const int buf = pb & 1;
        if (ty == pb) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) rowp[buf][a][tx * 4 + c] = t[a][c];
        }
        if (tx == pb) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) colp[buf][ty * 4 + a][c] = t[a][c];
        }
        __syncthreads();
        double B[kQ][kQ], C[4][kQ], R[kQ][4];
#pragma unroll
        for (int a = 0; a < kQ; ++a)
#pragma unroll
            for (int c = 0; c < kQ; ++c) B[a][c] = rowp[buf][a][pb * 4 + c];
        inv4(B);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < kQ; ++c) C[a][c] = colp[buf][ty * 4 + a][c];
#pragma unroll
        for (int a = 0; a < kQ; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) R[a][c] = rowp[buf][a][tx * 4 + c];
        // CB = C B (rows of the tile against the pivot block)
        double CB[4][kQ];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < kQ; ++c) {
                double v = 0.0;
#pragma unroll
                for (int m = 0; m < kQ; ++m) v += C[a][m] * B[m][c];
                CB[a][c] = v;
            }
        const bool ip = ty == pb, jp = tx == pb;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double upd = t[a][c], br = 0.0;
#pragma unroll
                for (int m = 0; m < kQ; ++m) {
                    upd -= CB[a][m] * R[m][c];
                    br += B[a][m] * R[m][c];
                }
                const double bb = a < kQ && c < kQ ? B[a & (kQ - 1)][c & (kQ - 1)] : 0.0;
                t[a][c] = ip ? (jp ? bb : br) : (jp ? -CB[a][c & (kQ - 1)] : upd);
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

// Panels of the step, 64 x 64 tiles: blockIdx.y == 0: V[l][t] = sum_m B[l][m]
// M[p0+m][t] (64 x n, row-major); blockIdx.y == 1: W[t][l] = sum_m M[t][p0+m]
// B[m][l] (n x 64, row-major).  Tiles of P itself are skipped.
__global__ __launch_bounds__(256) void gj_panel_kernel(int32_t n, int32_t p0, int32_t k,
                                                       const double *__restrict__ M, double *__restrict__ V,
                                                       double *__restrict__ W) {
    __shared__ double Bs[kGJ][kGJ + 1], Ps[kGJ][kGJ + 1];
    const int32_t t0 = blockIdx.x * kGJ;
    if (t0 == p0) return;
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    const bool left = blockIdx.y == 1;
    // Bs = B (zero-padded), Ps = the panel tile: M[P, T] (V) or M[T, P] (W)
    // a fixed trip count, unrolled, so that all the tile loads are in flight together
#pragma unroll
    for (int it = 0; it < kGJ * kGJ / 256; ++it) {
        const int e = threadIdx.x + it * 256;
        const int r = e >> 6, c = e & 63;
        // clamped addresses and selects rather than conditional loads, so that the
        // loads of all iterations are issued before the first wait
        const bool ib = r < k && c < k;
        const double bv = M[(int64_t)(p0 + (ib ? r : 0)) * n + p0 + (ib ? c : 0)];
        Bs[r][c] = ib ? bv : 0.0;
        const bool ip = left ? (t0 + r < n && c < k) : (r < k && t0 + c < n);
        const int64_t row = left ? (ip ? t0 + r : p0) : p0 + (ip ? r : 0);
        const int64_t col = left ? p0 + (ip ? c : 0) : (ip ? t0 + c : p0);
        const double pv = M[row * n + col];
        Ps[r][c] = ip ? pv : 0.0;
    }
    __syncthreads();
    double acc[4][4] = {};
    if (!left) {
        // V tile: rows l (4 ty + a), columns t (4 tx + c)
        for (int m = 0; m < k; ++m) {
            double bv[4], pv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) bv[a] = Bs[ty * 4 + a][m];
#pragma unroll
            for (int c = 0; c < 4; ++c) pv[c] = Ps[m][tx * 4 + c];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[a][c] += bv[a] * pv[c];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int l = ty * 4 + a, t = t0 + tx * 4 + c;
                if (l < k && t < n) V[(int64_t)l * n + t] = acc[a][c];
            }
    } else {
        // W tile: rows t (4 ty + a), columns l (4 tx + c)
        for (int m = 0; m < k; ++m) {
            double pv[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) pv[a] = Ps[ty * 4 + a][m];
#pragma unroll
            for (int c = 0; c < 4; ++c) bv[c] = Bs[m][tx * 4 + c];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[a][c] += pv[a] * bv[c];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int t = t0 + ty * 4 + a, l = tx * 4 + c;
                if (t < n && l < k) W[(int64_t)t * kGJ + l] = acc[a][c];
            }
    }
}

// M[i][j] -= sum_l M[i][p0+l] V[l][j] for i, j outside P, one 64 x 64 output
// tile per workgroup
__global__ __launch_bounds__(256) void gj_update_kernel(int32_t n, int32_t p0, int32_t k, double *__restrict__ M,
                                                        const double *__restrict__ V) {
    __shared__ double Ls[kGJ][kGJ + 1], Vs[kGJ][kGJ + 1];
    const int32_t i0 = blockIdx.y * kGJ, j0 = blockIdx.x * kGJ;
    if (i0 == p0 || j0 == p0) return;
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
    for (int it = 0; it < kGJ * kGJ / 256; ++it) {
        const int e = threadIdx.x + it * 256;
        const int r = e >> 6, c = e & 63;
        const bool il = i0 + r < n && c < k, iv = r < k && j0 + c < n;
        const double lv = M[(int64_t)(il ? i0 + r : p0) * n + p0 + (il ? c : 0)];
        const double vv = V[(int64_t)(iv ? r : 0) * n + (iv ? j0 + c : 0)];
        Ls[r][c] = il ? lv : 0.0;
        Vs[r][c] = iv ? vv : 0.0;
    }
    __syncthreads();
    double acc[4][4] = {};
    for (int l = 0; l < k; ++l) {
        double lv[4], vv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) lv[a] = Ls[ty * 4 + a][l];
#pragma unroll
        for (int c = 0; c < 4; ++c) vv[c] = Vs[l][tx * 4 + c];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[a][c] += lv[a] * vv[c];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = i0 + ty * 4 + a, j = j0 + tx * 4 + c;
            if (i < n && j < n) M[(int64_t)i * n + j] -= acc[a][c];
        }
}

// M[P,t] = V[.,t] and M[t,P] = -W[t,.] for t outside P
__global__ __launch_bounds__(256) void gj_writeback_kernel(int32_t n, int32_t p0, int32_t k, double *__restrict__ M,
                                                           const double *__restrict__ V, const double *__restrict__ W) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)n * k;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(e / n);
        const int64_t t = e % n;
        if (t >= p0 && t < p0 + k) continue;
        M[(int64_t)(p0 + l) * n + t] = V[(int64_t)l * n + t];
        M[t * n + p0 + l] = -W[t * kGJ + l];
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
// b_c[I] = sum of r over aggregate I: kRL lanes per coarse row (four coarse
// rows per wavefront), members strided over the lanes and combined by a fixed
// shuffle tree.  With xc, also the first smoothing iterate of the coarse
// level, xc = D_c^-1 bc.
constexpr int kRL = 16;
template <class X>
__global__ __launch_bounds__(kAT) void vc_restrict_kernel(int32_t nc, const int32_t *__restrict__ mptr,
                                                          const int32_t *__restrict__ mrows, const X *__restrict__ r,
                                                          X *__restrict__ bc, const X *__restrict__ dinv_c,
                                                          X *__restrict__ xc, const PcgState *st) {
    if (st && st->done) return;
    const int sub = threadIdx.x & (kRL - 1);
    const int64_t g0 = ((int64_t)xcd_block() * blockDim.x + threadIdx.x) / kRL;
    const int64_t ng = ((int64_t)gridDim.x * blockDim.x) / kRL;
    // every lane of a wavefront runs the same number of passes (the shuffles need them all)
    for (int64_t gb = g0 - (g0 & (64 / kRL - 1)); gb < nc; gb += ng) {
        const int64_t I = gb + (g0 & (64 / kRL - 1));
        X s = 0;
        if (I < nc)
            for (int32_t t = mptr[I] + sub; t < mptr[I + 1]; t += kRL) s += r[mrows[t]];
#pragma unroll
        for (int o = kRL / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (sub == 0 && I < nc) {
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
// With zq also the partials of qv . out (flexible CG: the new preconditioned
// residual against the last A p).
template <class V, class X>
__global__ __launch_bounds__(kRzThreads) void vc_sweep_kernel(Sell<V> A, const X *__restrict__ dinv, const X *__restrict__ b,
                                                       const X *__restrict__ y, X *__restrict__ out,
                                                       double *__restrict__ rz, double *__restrict__ zq,
                                                       const X *__restrict__ qv, const PcgState *st) {
    if (st && st->done) return;
    double v[2] = {0.0, 0.0};
    GS(i, A.n) {
        const X s = sell_row_apply<V, X>(A, (int32_t)i, [&](int32_t j) { return y[j]; });
        const X o = y[i] + dinv[i] * (b[i] - s);
        out[i] = o;
        v[0] += (double)b[i] * (double)o;
        if (zq) v[1] += (double)qv[i] * (double)o;
    }
    if (rz) {
        block_reduce<OpSum, 2, kRzThreads>(v);
        if (threadIdx.x == 0) {
            rz[blockIdx.x] = v[0];
            if (zq) zq[blockIdx.x] = v[1];
        }
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
    for (int64_t w = ((int64_t)xcd_block() * blockDim.x + threadIdx.x) >> 6; w * kRowsPerWave < A.n; w += nw) {
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
            if (A.dg) sum += (X)A.dg[i] * f(i);
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

// ---------------------------------------------------------------------------
// K-cycle: on a coarse level m the coarse correction is two steps of a
// flexible CG on A_m e = b, each preconditioned by the V-cycle from level m
// (Krylov acceleration of the coarse-grid correction, which unsmoothed
// aggregation needs to keep its convergence independent of the level count).
// With c = B(b), v = A c, rho = c.v, alpha1 = c.b / rho, rt = b - alpha1 v,
// d = B(rt), w = A d, gamma = d.v, beta = d.w - gamma^2 / rho,
// alpha2 = d.rt / beta:   e = (alpha1 - gamma alpha2 / rho) c + alpha2 d.
// Scalars are formed by each consuming kernel from per-block partials, in a
// fixed order.  parts: [c.v | c.b | d.w | d.v | d.rt] x G.
// ---------------------------------------------------------------------------
template <class X>
__device__ inline void kc_scalars(const double *parts, int G, double &rho, double &a1, double &g, double &a2) {
    rho = sum_parts<OpSum, kAT>(parts, G);
    const double cb = sum_parts<OpSum, kAT>(parts + G, G);
    a1 = rho > 0.0 ? cb / rho : 0.0;
    g = 0.0;
    a2 = 0.0;
}
// v = A c; partials c.v and c.b
template <class V, class X>
__global__ __launch_bounds__(kAT) void kc_av_kernel(Sell<V> A, const X *__restrict__ c, const X *__restrict__ b,
                                                    X *__restrict__ v, double *__restrict__ parts,
                                                    const PcgState *st) {
    if (st && st->done) return;
    double p[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n; i += (int64_t)gridDim.x * blockDim.x) {
        const X vi = sell_row_apply<V, X>(A, (int32_t)i, [&](int32_t j) { return c[j]; });
        v[i] = vi;
        p[0] += (double)c[i] * (double)vi;
        p[1] += (double)c[i] * (double)b[i];
    }
    block_reduce<OpSum, 2, kAT>(p);
    if (threadIdx.x == 0) {
        parts[blockIdx.x] = p[0];
        parts[gridDim.x + blockIdx.x] = p[1];
    }
}
// rt = b - alpha1 v, and the next V-cycle's first iterate xa = D^-1 rt
template <class X>
__global__ __launch_bounds__(kAT) void kc_rt_kernel(int32_t n, const X *__restrict__ b, const X *__restrict__ v,
                                                    const X *__restrict__ dinv, const double *__restrict__ parts,
                                                    X *__restrict__ rt, X *__restrict__ xa, const PcgState *st) {
    if (st && st->done) return;
    double rho, a1, g, a2;
    kc_scalars<X>(parts, gridDim.x, rho, a1, g, a2);
    const X a = (X)a1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const X r = b[i] - a * v[i];
        rt[i] = r;
        xa[i] = dinv[i] * r;
    }
}
// w = A d; partials d.w, d.v, d.rt
template <class V, class X>
__global__ __launch_bounds__(kAT) void kc_aw_kernel(Sell<V> A, const X *__restrict__ d, const X *__restrict__ v,
                                                    const X *__restrict__ rt, X *__restrict__ w,
                                                    double *__restrict__ parts, const PcgState *st) {
    if (st && st->done) return;
    double p[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n; i += (int64_t)gridDim.x * blockDim.x) {
        const X wi = sell_row_apply<V, X>(A, (int32_t)i, [&](int32_t j) { return d[j]; });
        w[i] = wi;
        p[0] += (double)d[i] * (double)wi;
        p[1] += (double)d[i] * (double)v[i];
        p[2] += (double)d[i] * (double)rt[i];
    }
    block_reduce<OpSum, 3, kAT>(p);
    if (threadIdx.x == 0) {
        const int G = gridDim.x;
        parts[2 * G + blockIdx.x] = p[0];
        parts[3 * G + blockIdx.x] = p[1];
        parts[4 * G + blockIdx.x] = p[2];
    }
}
// e = (alpha1 - gamma alpha2 / rho) c + alpha2 d
template <class X>
__global__ __launch_bounds__(kAT) void kc_combine_kernel(int32_t n, const X *__restrict__ c, const X *__restrict__ d,
                                                         const double *__restrict__ parts, X *__restrict__ e,
                                                         const PcgState *st) {
    if (st && st->done) return;
    const int G = gridDim.x;
    double rho, a1, g, a2;
    kc_scalars<X>(parts, G, rho, a1, g, a2);
    if (rho > 0.0) {
        const double dw = sum_parts<OpSum, kAT>(parts + 2 * G, G);
        g = sum_parts<OpSum, kAT>(parts + 3 * G, G);
        const double drt = sum_parts<OpSum, kAT>(parts + 4 * G, G);
        const double beta = dw - g * g / rho;
        a2 = beta > 0.0 ? drt / beta : 0.0;
    }
    const X ac = (X)(rho > 0.0 ? a1 - g * a2 / rho : 0.0), ad = (X)a2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        e[i] = ac * c[i] + ad * d[i];
}

// dense coarse solve x = Ainv b: one wavefront per row, lanes along the
// (contiguous) row, fixed-order wave reduction
template <class X>
__global__ __launch_bounds__(kAT) void vc_dense_kernel(int32_t n, const X *__restrict__ Ainv, const X *__restrict__ b,
                                                       X *__restrict__ x, const PcgState *st) {
    if (st && st->done) return;
    const int lane = threadIdx.x & 63;
    for (int64_t i = ((int64_t)xcd_block() * blockDim.x + threadIdx.x) >> 6; i < n;
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
// FP32 copy of a level's matrix that keeps every row sum: the off-diagonal
// entries are rounded to FP32 and the diagonal, kept apart in FP64, absorbs
// their rounding (dg_i = sum_j a_ij - sum_{j != i} fl32(a_ij)).  The rounding
// error is then a Laplacian-like matrix with zero row sums: it leaves the
// constant vector alone and perturbs each coupling by a relative 2^-24, so
// the near-null (smooth) modes that the coarse levels must resolve are kept.
__global__ __launch_bounds__(kAT) void to_float_rowsum_kernel(Sell<double> A, float *__restrict__ v32,
                                                              double *__restrict__ dg) {
    GS(i, A.n) {
        const int64_t b0 = A.ptr[i >> 6], b1 = A.ptr[(i >> 6) + 1];
        double s = 0.0, so = 0.0;
        for (int64_t q = b0 + (i & 63); q < b1; q += 64) {
            const double a = A.val[q];
            s += a;
            if (A.col[q] == i) {
                v32[q] = 0.0f;
            } else {
                const float f = (float)a;
                v32[q] = f;
                so += (double)f;
            }
        }
        dg[i] = s - so;
    }
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
void amg_launch_mis(hipStream_t s, Sell<double> A, const double *diag, double theta, int rounds, int hops,
                    uint32_t *T, uint32_t *T1, int *undecided, int32_t *flag, int *hcnt, int32_t *scol) {
    ALAUNCH(strength_kernel, gridv(A.n), kAT, A, diag, theta, scol);
    ALAUNCH(mis_init_kernel, gridv(A.n), kAT, A.n, T, T1);
    for (int r = 0; r < rounds; ++r) {
        int *cur = undecided + (int64_t)r * kCntSlots * kCntStride;
        const int *active = r ? cur - kCntSlots * kCntStride : nullptr;
        ALAUNCH(mis_max_kernel, gridv(A.n), kAT, A.n, A.ptr, scol, T, T1, active);
        ALAUNCH(mis_select_kernel, gridv(A.n), kAT, A.n, hops, A.ptr, scol, T1, T, cur, active);
        if ((r & 3) == 3 && r + 1 < rounds) {  // stop queueing rounds once nothing is undecided
            VAG_HIP(hipMemcpyAsync(hcnt, cur, kCntSlots * kCntStride * sizeof(int), hipMemcpyDeviceToHost, s));
            VAG_HIP(hipStreamSynchronize(s));
            bool any = false;
            for (int k = 0; k < kCntSlots; ++k) any = any || hcnt[k * kCntStride] != 0;
            if (!any) break;
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
    ALAUNCH(galerkin_hash_kernel, nc, 64, A, Jcol, apv, apn, mptr, mrows, nc, mode, big, rowlen, cptr, ccol, cval);
    ALAUNCH(galerkin_kernel<8192>, nc, 64, A, Jcol, apv, apn, mptr, mrows, nc, mode, big, rowlen, cptr, ccol, cval,
            overflow);
}
void amg_launch_slices(hipStream_t s, int32_t n, const int32_t *rowlen, int32_t *width, int32_t *cnt, int64_t *ptr,
                       unsigned long long *nnz) {
    const int32_t ns = (n + 63) / 64;
    if (ns > 0) ALAUNCH(slice_width_kernel, ns, 64, n, rowlen, width, cnt);
    launch_slice_scan(s, ns, width, kSliceRows, ptr, cnt, nnz);
}
void amg_launch_slice_tail(hipStream_t s, int32_t n, const int64_t *ptr, int32_t *col, double *val) {
    if (n & 63) ALAUNCH(slice_tail_kernel, 1, 64, n, ptr, col, val);
}
void amg_launch_dense_inverse(hipStream_t s, Sell<double> A, double *D, double *work) {
    const int32_t n = A.n;
    ALAUNCH(dense_from_sell_kernel, gridv((int64_t)n * n), kAT, A, D);
    ALAUNCH(dense_scatter_kernel, gridv(n), kAT, A, D);
    const unsigned nt = (unsigned)((n + kGJ - 1) / kGJ);
    const unsigned gw = (unsigned)std::min<int64_t>(((int64_t)n * kGJ + 255) / 256, 4096);
    double *V = work, *W = work + (int64_t)kGJ * n;
    for (int32_t p0 = 0; p0 < n; p0 += kGJ) {
        const int32_t k = std::min(kGJ, n - p0);
        ALAUNCH(gj_pivot_kernel, 1, 256, n, p0, k, D);
        if (nt > 1) {
            hipLaunchKernelGGL(gj_panel_kernel, dim3(nt, 2), dim3(256), 0, s, n, p0, k, D, V, W);
            VAG_HIP(hipGetLastError());
            hipLaunchKernelGGL(gj_update_kernel, dim3(nt, nt), dim3(256), 0, s, n, p0, k, D, V);
            VAG_HIP(hipGetLastError());
            ALAUNCH(gj_writeback_kernel, gw, 256, n, p0, k, D, V, W);
        }
    }
}
int kc_grid(int32_t n) { return (int)reduce_grid(n, kAT); }
template <class V, class X>
void amg_launch_kc_av(hipStream_t s, Sell<V> A, const X *c, const X *b, X *v, double *parts, const PcgState *st) {
    ALAUNCH((kc_av_kernel<V, X>), kc_grid(A.n), kAT, A, c, b, v, parts, st);
}
template <class X>
void amg_launch_kc_rt(hipStream_t s, int32_t n, const X *b, const X *v, const X *dinv, const double *parts, X *rt,
                      X *xa, const PcgState *st) {
    ALAUNCH(kc_rt_kernel<X>, kc_grid(n), kAT, n, b, v, dinv, parts, rt, xa, st);
}
template <class V, class X>
void amg_launch_kc_aw(hipStream_t s, Sell<V> A, const X *d, const X *v, const X *rt, X *w, double *parts,
                      const PcgState *st) {
    ALAUNCH((kc_aw_kernel<V, X>), kc_grid(A.n), kAT, A, d, v, rt, w, parts, st);
}
template <class X>
void amg_launch_kc_combine(hipStream_t s, int32_t n, const X *c, const X *d, const double *parts, X *e,
                           const PcgState *st) {
    ALAUNCH(kc_combine_kernel<X>, kc_grid(n), kAT, n, c, d, parts, e, st);
}
template void amg_launch_kc_av<double, double>(hipStream_t, Sell<double>, const double *, const double *, double *,
                                               double *, const PcgState *);
template void amg_launch_kc_av<float, double>(hipStream_t, Sell<float>, const double *, const double *, double *,
                                              double *, const PcgState *);
template void amg_launch_kc_aw<double, double>(hipStream_t, Sell<double>, const double *, const double *,
                                               const double *, double *, double *, const PcgState *);
template void amg_launch_kc_aw<float, double>(hipStream_t, Sell<float>, const double *, const double *,
                                              const double *, double *, double *, const PcgState *);
template void amg_launch_kc_rt<double>(hipStream_t, int32_t, const double *, const double *, const double *,
                                       const double *, double *, double *, const PcgState *);
template void amg_launch_kc_combine<double>(hipStream_t, int32_t, const double *, const double *, const double *,
                                            double *, const PcgState *);
template <class V, class X>
void amg_launch_pre(hipStream_t s, Sell<V> A, const X *dinv, const X *b, X *x, X *r, const PcgState *st) {
    ALAUNCH(vc_scale_kernel<X>, gridv(A.n), kAT, A.n, dinv, b, x, st);
    amg_launch_resid<V, X>(s, A, b, x, r, st);
}
template <class X>
void amg_launch_restrict(hipStream_t s, int32_t nc, const int32_t *mptr, const int32_t *mrows, const X *r, X *bc,
                         const X *dinv_c, X *xc, const PcgState *st) {
    ALAUNCH(vc_restrict_kernel<X>, gridv((int64_t)nc * kRL), kAT, nc, mptr, mrows, r, bc, dinv_c, xc, st);
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
                     X *y, X *out, double *rz, const PcgState *st, double *zq, const X *qv) {
    ALAUNCH(vc_prolong_kernel<X>, gridv(A.n), kAT, A.n, x, agg, e, y, st);
    // with rz the partials must match the Krylov kernels' grid and block size
    if (rz)
        ALAUNCH((vc_sweep_kernel<V, X>), reduce_grid(A.n, kRzThreads), kRzThreads, A, dinv, b, y, out, rz, zq, qv, st);
    else
        ALAUNCH((vc_sweep_kernel<V, X>), gridv(A.n), kAT, A, dinv, b, y, out, nullptr, nullptr, nullptr, st);
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
        ALAUNCH((vc_sweep_kernel<V, X>), gridv(A.n), kAT, A, dinv, b, x, out, nullptr, nullptr, nullptr, st);
}
void launch_to_float(hipStream_t s, int64_t n, const double *a, float *b) {
    if (n > 0) ALAUNCH(to_float_kernel, gridv(n), kAT, n, a, b);
}
void launch_to_float_rowsum(hipStream_t s, Sell<double> A, float *v32, double *dg) {
    if (A.n > 0) ALAUNCH(to_float_rowsum_kernel, gridv(A.n), kAT, A, v32, dg);
}
void launch_to_double(hipStream_t s, int64_t n, const float *a, double *b) {
    if (n > 0) ALAUNCH(to_double_kernel, gridv(n), kAT, n, a, b);
}

#define VC_INST(V, X)                                                                                            \
    template void amg_launch_pre<V, X>(hipStream_t, Sell<V>, const X *, const X *, X *, X *, const PcgState *);    \
    template void amg_launch_resid<V, X>(hipStream_t, Sell<V>, const X *, const X *, X *, const PcgState *);       \
    template void amg_launch_post<V, X>(hipStream_t, Sell<V>, const X *, const X *, const X *, const int32_t *,    \
                                        const X *, X *, X *, double *, const PcgState *, double *, const X *);     \
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
