// After the Darcy solve: cell recovery (eq eqschurcell), VAG fluxes
// (eqs VAGFluxMatrix, VAGFluxFracture), porous volumes (§3.2.1), CFL time step
// (eq eq_CFL) and the explicit upwind steps (eq darcyfluxH, §3.2.2).
//
// Control-volume vector layout: [cells | fracture faces | nodes].
//
// The fluxes are fixed during transport, so the explicit step is linear:
// c^{n+1} = T c^n with, per control volume i and dt/phi_i = w_i,
//   T_ii = 1 - w_i * (sum of outgoing fluxes), T_ij = w_i * (incoming flux from j).
// Each pair (K,nu) contributes one off-diagonal, in the row of the downstream
// control volume.  T is built once per transport call in slices of 64 rows
// (one wavefront), the rows of a slice sorted longest first; level k of a
// slice holds entry k of its rows that have more than k entries, packed
// densely (jagged diagonals), so no padding is stored or fetched, and every
// step is one sweep over it in which each level is a coalesced run of loads.
// Dirichlet nodes keep T_ii = 1, no off-diagonal, so they stay at c_bar.
#include <mutex>

#include "reduce.h"

namespace vag {

constexpr int kT = 256;
static inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

__global__ __launch_bounds__(kT) void node_pressure_kernel(int32_t nn, const int32_t *__restrict__ node_unk,
                                                           const double *__restrict__ x,
                                                           const double *__restrict__ p_bar,
                                                           double *__restrict__ u_node) {
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nn) return;
    const int32_t k = node_unk[s];
    u_node[s] = k >= 0 ? x[k] : p_bar[s];
}

__global__ __launch_bounds__(128) void cell_flux_kernel(
    int32_t nc, const int32_t *__restrict__ hex8, const uint8_t *__restrict__ fmask,
    const int32_t *__restrict__ cell_frac, const int32_t *__restrict__ frac_cell, const double *__restrict__ aK,
    const double *__restrict__ rK, const double *__restrict__ AKK, const double *__restrict__ fside,
    const double *__restrict__ u_node, const double *__restrict__ u_frac, double *__restrict__ u_cell,
    double *__restrict__ F_cell, double *__restrict__ F_cell_frac) {
    const int32_t K = blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= nc) return;
    const unsigned mask = fmask[K];
    double u[8], r[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        u[a] = u_node[hex8[8 * (int64_t)K + a]];
        r[a] = rK[(int64_t)a * nc + K];
    }
    double t = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) t += r[a] * u[a];
#pragma unroll
    for (int f = 0; f < 6; ++f)
        if ((mask >> f) & 1u) {
            const int32_t sg = cell_frac[6 * (int64_t)K + f];
            const int side = frac_cell[2 * (int64_t)sg] == K ? 0 : 1;
            t += fside[(2 * (int64_t)sg + side) * 6 + 5] * u_frac[sg];
        }
    const double uK = t / AKK[K];  // eq eqschurcell with zero cell right-hand side
    u_cell[K] = uK;
    double F[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) s += aK[(int64_t)sym8(a, c) * nc + K] * (uK - u[c]);
        F[a] = s;
    }
#pragma unroll
    for (int f = 0; f < 6; ++f)
        if ((mask >> f) & 1u) {
            const int32_t sg = cell_frac[6 * (int64_t)K + f];
            const int side = frac_cell[2 * (int64_t)sg] == K ? 0 : 1;
            const double *o = fside + (2 * (int64_t)sg + side) * 6;
            const double us = u_frac[sg];
            double Fs = o[0] * (uK - us);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                Fs += o[1 + i] * (uK - u[hexf(f, i)]);
                F[hexf(f, i)] += o[1 + i] * (uK - us);
            }
            F_cell_frac[2 * (int64_t)sg + side] = Fs;
        }
#pragma unroll
    for (int a = 0; a < 8; ++a) F_cell[8 * (int64_t)K + a] = F[a];
}

__global__ __launch_bounds__(kT) void frac_flux_kernel(int32_t nf, const int32_t *__restrict__ frac_nodes,
                                                       const double *__restrict__ A5,
                                                       const double *__restrict__ u_node,
                                                       const double *__restrict__ u_frac,
                                                       double *__restrict__ F_frac) {
    const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    double u[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] = u_node[frac_nodes[4 * (int64_t)f + i]];
    const double us = u_frac[f];
    const double *M = A5 + 25 * (int64_t)f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) s += M[5 * (1 + i) + 1 + j] * (us - u[j]);
        F_frac[4 * (int64_t)f + i] = s;
    }
}

// Porous volumes with alpha_{K,s} = 1/16 and alpha_{sigma,s} = 1/8: matrix
// nodes take 1/16 of each adjacent cell, fracture nodes 1/8 of each adjacent
// fracture face, Dirichlet nodes nothing.  With pmax, a cell (fracture face)
// gives a node its share only if its permeability reaches pmax[node] (§3.2.1,
// nodes between rock types).
__global__ __launch_bounds__(kT) void porous_kernel(
    int32_t nc, int32_t nf, int32_t nn, const int32_t *__restrict__ hex8, const int32_t *__restrict__ frac_nodes,
    const uint8_t *__restrict__ dirichlet, const uint8_t *__restrict__ frac_node,
    const int32_t *__restrict__ ncp, const int32_t *__restrict__ ncl, const int32_t *__restrict__ nfp,
    const int32_t *__restrict__ nfl, const double *__restrict__ vol, const double *__restrict__ poro,
    const double *__restrict__ area, const double *__restrict__ fwidth, const double *__restrict__ fporo,
    const double *__restrict__ perm, const double *__restrict__ fperm, const double *__restrict__ pmax,
    double *__restrict__ phi_cell, double *__restrict__ phi_frac, double *__restrict__ phi_node) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nc) {
        const int32_t K = (int32_t)i;
        const double mK = pmax ? perm_measure(perm, K) : 0.0;
        double sa = 0.0;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int32_t s = hex8[8 * (int64_t)K + a];
            if (!dirichlet[s] && !frac_node[s] && (!pmax || mK >= pmax[s])) sa += 1.0 / 16.0;
        }
        phi_cell[K] = (1.0 - sa) * (vol[K] * poro[K]);
    } else if (i < (int64_t)nc + nf) {
        const int32_t f = (int32_t)(i - nc);
        double sa = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int32_t s = frac_nodes[4 * (int64_t)f + k];
            if (!dirichlet[s] && (!pmax || fperm[f] >= pmax[s])) sa += 1.0 / 8.0;
        }
        phi_frac[f] = (1.0 - sa) * (fwidth[f] * area[f] * fporo[f]);
    } else if (i < (int64_t)nc + nf + nn) {
        const int32_t s = (int32_t)(i - nc - nf);
        double p = 0.0;
        if (!dirichlet[s]) {
            if (frac_node[s]) {
                for (int32_t q = nfp[s]; q < nfp[s + 1]; ++q) {
                    const int32_t f = nfl[q] >> 2;
                    if (!pmax || fperm[f] >= pmax[s]) p += (1.0 / 8.0) * (fwidth[f] * area[f] * fporo[f]);
                }
            } else {
                for (int32_t q = ncp[s]; q < ncp[s + 1]; ++q) {
                    const int32_t K = ncl[q] >> 3;
                    if (!pmax || perm_measure(perm, K) >= pmax[s]) p += (1.0 / 16.0) * (vol[K] * poro[K]);
                }
            }
        }
        phi_node[s] = p;
    }
}

__global__ __launch_bounds__(kT) void node_pmax_kernel(int32_t nn, const uint8_t *__restrict__ frac_node,
                                                       const int32_t *__restrict__ ncp, const int32_t *__restrict__ ncl,
                                                       const int32_t *__restrict__ nfp, const int32_t *__restrict__ nfl,
                                                       const double *__restrict__ perm,
                                                       const double *__restrict__ fperm, double *__restrict__ pmax) {
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nn) return;
    double m = -1.0;
    if (frac_node[s])
        for (int32_t q = nfp[s]; q < nfp[s + 1]; ++q) m = fmax(m, fperm[nfl[q] >> 2]);
    else
        for (int32_t q = ncp[s]; q < ncp[s + 1]; ++q) m = fmax(m, perm_measure(perm, ncl[q] >> 3));
    pmax[s] = m;
}

// Sum of outgoing fluxes of a control volume (denominators of eq eq_CFL).
__device__ inline double cell_out(int32_t K, unsigned mask, const int32_t *cell_frac, const int32_t *frac_cell,
                                  const double *F_cell, const double *F_cell_frac) {
    double o = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) o += fmax(F_cell[8 * (int64_t)K + a], 0.0);
    if (mask) {
#pragma unroll
        for (int f = 0; f < 6; ++f)
            if ((mask >> f) & 1u) {
                const int32_t sg = cell_frac[6 * (int64_t)K + f];
                const int side = frac_cell[2 * (int64_t)sg] == K ? 0 : 1;
                o += fmax(F_cell_frac[2 * (int64_t)sg + side], 0.0);
            }
    }
    return o;
}
__device__ inline double frac_out(int32_t f, const int32_t *frac_cell, const double *F_frac,
                                  const double *F_cell_frac) {
    double o = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) o += fmax(F_frac[4 * (int64_t)f + i], 0.0);
    for (int side = 0; side < 2; ++side)
        if (frac_cell[2 * (int64_t)f + side] >= 0) o += fmax(-F_cell_frac[2 * (int64_t)f + side], 0.0);
    return o;
}
__device__ inline double node_out(int32_t s, const int32_t *ncp, const int32_t *ncl, const int32_t *nfp,
                                  const int32_t *nfl, const double *F_cell, const double *F_frac) {
    double o = 0.0;
    for (int32_t q = ncp[s]; q < ncp[s + 1]; ++q) o += fmax(-F_cell[ncl[q]], 0.0);
    for (int32_t q = nfp[s]; q < nfp[s + 1]; ++q) o += fmax(-F_frac[nfl[q]], 0.0);
    return o;
}

// The CFL kernels run 1024-thread blocks: the grid of a deterministic
// reduction is capped at kReduceBlocks, and with 256 threads a block the
// chip held two waves per SIMD, each walking ~100 control volumes through
// dependent gathers.  A minimum is exact in any grouping, so dt does not
// depend on the launch shape.
constexpr int kCflT = 1024;

__global__ __launch_bounds__(kCflT) void cfl_kernel(
    int32_t nc, int32_t nf, int32_t nn, const int32_t *__restrict__ hex8, const uint8_t *__restrict__ fmask,
    const int32_t *__restrict__ cell_frac, const int32_t *__restrict__ frac_cell,
    const uint8_t *__restrict__ dirichlet, const int32_t *__restrict__ ncp, const int32_t *__restrict__ ncl,
    const int32_t *__restrict__ nfp, const int32_t *__restrict__ nfl, const double *__restrict__ F_cell,
    const double *__restrict__ F_cell_frac, const double *__restrict__ F_frac, const double *__restrict__ wout,
    const double *__restrict__ phi_cell, const double *__restrict__ phi_frac, const double *__restrict__ phi_node,
    double *__restrict__ parts) {
    const double inf = __builtin_inf();
    double v[3] = {inf, inf, inf};
    const int64_t total = (int64_t)nc + nf + nn;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < nc) {
            const int32_t K = (int32_t)i;
            const double o = cell_out(K, fmask[K], cell_frac, frac_cell, F_cell, F_cell_frac);
            if (o > 0.0) v[0] = fmin(v[0], phi_cell[K] / o);
        } else if (i < (int64_t)nc + nf) {
            const int32_t f = (int32_t)(i - nc);
            const double o = frac_out(f, frac_cell, F_frac, F_cell_frac) + (wout ? wout[f] : 0.0);
            if (o > 0.0) v[1] = fmin(v[1], phi_frac[f] / o);
        } else {
            const int32_t s = (int32_t)(i - nc - nf);
            if (!dirichlet[s]) {
                const double o = node_out(s, ncp, ncl, nfp, nfl, F_cell, F_frac);
                if (o > 0.0) v[2] = fmin(v[2], phi_node[s] / o);
            }
        }
    }
    block_partials<OpMin, 3, kCflT>(v, parts, gridDim.x);
}

__global__ __launch_bounds__(kT) void cfl_finish_kernel(const double *__restrict__ parts, int G, double cfl,
                                                        double *__restrict__ dt_out) {
    const double a = sum_parts<OpMin, kT>(parts, G);
    const double b = sum_parts<OpMin, kT>(parts + G, G);
    const double c = sum_parts<OpMin, kT>(parts + 2 * (size_t)G, G);
    if (threadIdx.x == 0) {
        dt_out[0] = a;
        dt_out[1] = b;
        dt_out[2] = c;
        dt_out[3] = cfl * fmin(a, fmin(b, c));
    }
}

// ---------------------------------------------------------------------------
// upwind operator T in sliced ELL
// ---------------------------------------------------------------------------
__device__ inline int upwind_row_count(int64_t i, int32_t nc, int32_t nf, const uint8_t *fmask,
                                       const int32_t *cell_frac, const int32_t *frac_cell, const uint8_t *dirichlet,
                                       const int32_t *ncp, const int32_t *ncl, const int32_t *nfp,
                                       const int32_t *nfl, const double *F_cell, const double *F_cell_frac,
                                       const double *F_frac, const double *wsrc) {
    int c = 0;
    if (i < nc) {
        const int32_t K = (int32_t)i;
#pragma unroll
        for (int a = 0; a < 8; ++a) c += F_cell[8 * (int64_t)K + a] < 0.0;
        const unsigned mask = fmask[K];
        if (mask)
            for (int f = 0; f < 6; ++f)
                if ((mask >> f) & 1u) {
                    const int32_t sg = cell_frac[6 * (int64_t)K + f];
                    const int side = frac_cell[2 * (int64_t)sg] == K ? 0 : 1;
                    c += F_cell_frac[2 * (int64_t)sg + side] < 0.0;
                }
    } else if (i < (int64_t)nc + nf) {
        const int32_t f = (int32_t)(i - nc);
#pragma unroll
        for (int k = 0; k < 4; ++k) c += F_frac[4 * (int64_t)f + k] < 0.0;
        for (int side = 0; side < 2; ++side)
            if (frac_cell[2 * (int64_t)f + side] >= 0) c += F_cell_frac[2 * (int64_t)f + side] > 0.0;
        if (wsrc) c += wsrc[f] > 0.0;  // injection: an entry on the constant control volume
    } else {
        const int32_t s = (int32_t)(i - nc - nf);
        if (!dirichlet[s]) {
            for (int32_t q = ncp[s]; q < ncp[s + 1]; ++q) c += F_cell[ncl[q]] > 0.0;
            for (int32_t q = nfp[s]; q < nfp[s + 1]; ++q) c += F_frac[nfl[q]] > 0.0;
        }
    }
    return c;
}

// Sorts the rows of a slice (one wavefront, lane = row in the slice, c = its
// entry count) longest first and writes meta, the slice's width and count.
__device__ inline void slice_sort_rows(int c, int lane, int32_t *__restrict__ slice_width,
                                       uint16_t *__restrict__ meta, int32_t *__restrict__ slice_nnz) {
    // sort the slice's rows by entry count, longest first (ties: lower lane
    // first), with a bitonic network over the wavefront: slot l then holds
    // the l-th longest row, so the lanes that run out of entries are the last
    // ones and whole cache lines of padding are never read
    int key = (c << 8) | (63 - lane);  // larger key = longer row, then lower lane
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int other = __shfl_xor(key, j, 64);
            const bool up = ((lane & k) == 0);          // descending in this k-block
            const bool lower = ((lane & j) == 0);
            const int hi = max(key, other), lo = min(key, other);
            key = (lower == up) ? hi : lo;
        }
    }
    const int cnt = key >> 8, src = 63 - (key & 255);
    meta[(int64_t)blockIdx.x * kSliceRows + lane] = (uint16_t)((src << 8) | cnt);
    int sum = c;
    int w = cnt;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        w = max(w, __shfl_down(w, o, 64));
        sum += __shfl_down(sum, o, 64);
    }
    if (lane == 0) {
        slice_width[blockIdx.x] = w;
        slice_nnz[blockIdx.x] = sum;
    }
}

__global__ __launch_bounds__(kSliceRows) void upwind_count_kernel(
    int32_t nc, int32_t nf, int32_t nn, const uint8_t *__restrict__ fmask, const int32_t *__restrict__ cell_frac,
    const int32_t *__restrict__ frac_cell, const uint8_t *__restrict__ dirichlet, const int32_t *__restrict__ ncp,
    const int32_t *__restrict__ ncl, const int32_t *__restrict__ nfp, const int32_t *__restrict__ nfl,
    const double *__restrict__ F_cell, const double *__restrict__ F_cell_frac, const double *__restrict__ F_frac,
    const double *__restrict__ wsrc, int32_t *__restrict__ slice_width, uint16_t *__restrict__ meta,
    int32_t *__restrict__ slice_nnz) {
    // one block = one wavefront = one slice
    const int lane = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kSliceRows + lane;
    const int64_t total = (int64_t)nc + nf + nn;
    int c = 0;
    if (i < total)
        c = upwind_row_count(i, nc, nf, fmask, cell_frac, frac_cell, dirichlet, ncp, ncl, nfp, nfl, F_cell,
                             F_cell_frac, F_frac, wsrc);
    slice_sort_rows(c, lane, slice_width, meta, slice_nnz);
}

// exclusive scan of per_width * w over the slices, one block; with cnt, also
// *total = sum of cnt (the entries without padding)
__global__ __launch_bounds__(1024) void slice_scan_kernel(int32_t nslice, const int32_t *__restrict__ w,
                                                          int per_width, int64_t *__restrict__ ptr,
                                                          const int32_t *__restrict__ cnt,
                                                          unsigned long long *__restrict__ total) {
    __shared__ int64_t wsum[16], csum[16];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int32_t chunk = (nslice + 1023) / 1024;
    const int32_t lo = min(nslice, t * chunk), hi = min(nslice, lo + chunk);
    int64_t s = 0, c = 0;
    for (int32_t k = lo; k < hi; ++k) {
        s += (int64_t)w[k] * per_width;
        if (cnt) c += cnt[k];
    }
    // inclusive scan over the block: within each wavefront, then over the 16 wavefront totals
    int64_t v = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if (lane == 63) wsum[wid] = v;
    if (lane == 0) csum[wid] = c;
    __syncthreads();
    int64_t before = 0;
    for (int k = 0; k < wid; ++k) before += wsum[k];
    if (t == 1023) ptr[nslice] = before + v;
    if (t == 0 && total) {
        unsigned long long tc = 0;
        for (int k = 0; k < 16; ++k) tc += (unsigned long long)csum[k];
        *total = tc;
    }
    int64_t run = before + v - s;
    for (int32_t k = lo; k < hi; ++k) {
        ptr[k] = run;
        run += (int64_t)w[k] * per_width;
    }
}

// Slot threadIdx.x of the slice (one block of 64 threads) holds the row named
// by its meta entry, returned; entry k of slot t goes to level_off[k] + t
// (level k holds the slots with more than k entries, which the longest-first
// order puts first).  cnts and level_off are the block's shared arrays.
__device__ inline int slice_levels(const uint16_t *__restrict__ meta, uint8_t *cnts, int32_t *level_off) {
    const int lane = threadIdx.x;
    const uint16_t mt = meta[(int64_t)blockIdx.x * kSliceRows + lane];
    cnts[lane] = (uint8_t)(mt & 255);
    __syncthreads();
    const int width = cnts[0];
    for (int k = lane; k < width; k += kSliceRows) {
        int c = 0;
        for (int u = 0; u < kSliceRows; ++u) c += cnts[u] > k;
        level_off[k + 1] = c;
    }
    __syncthreads();
    if (lane == 0) {
        level_off[0] = 0;
        for (int k = 1; k <= width; ++k) level_off[k] += level_off[k - 1];
    }
    __syncthreads();
    return mt >> 8;
}

__global__ __launch_bounds__(kSliceRows) void upwind_fill_kernel(
    int32_t nc, int32_t nf, int32_t nn, const int32_t *__restrict__ hex8, const uint8_t *__restrict__ fmask,
    const int32_t *__restrict__ cell_frac, const int32_t *__restrict__ frac_cell,
    const int32_t *__restrict__ frac_nodes, const uint8_t *__restrict__ dirichlet, const int32_t *__restrict__ ncp,
    const int32_t *__restrict__ ncl, const int32_t *__restrict__ nfp, const int32_t *__restrict__ nfl,
    const double *__restrict__ F_cell, const double *__restrict__ F_cell_frac, const double *__restrict__ F_frac,
    const double *__restrict__ wsrc, const double *__restrict__ wout, const double *__restrict__ phi_cell,
    const double *__restrict__ phi_frac, const double *__restrict__ phi_node,
    const double *__restrict__ dtp, const int64_t *__restrict__ slice_ptr, const uint16_t *__restrict__ meta,
    int32_t *__restrict__ tcol, double *__restrict__ tval, double *__restrict__ tdiag) {
    __shared__ uint8_t cnts[kSliceRows];
    __shared__ int32_t level_off[257];
    const int lane = threadIdx.x;
    const int src = slice_levels(meta, cnts, level_off);
    const int64_t i = (int64_t)blockIdx.x * kSliceRows + src;
    const int64_t total = (int64_t)nc + nf + nn;
    if (i >= total) return;
    const int64_t base = slice_ptr[blockIdx.x] + lane;
    const double dt = dtp[3];
    int k = 0;
    double d = 1.0;
    auto emit = [&](int64_t c, double v) {
        tcol[base + level_off[k]] = (int32_t)c;
        tval[base + level_off[k]] = v;
        ++k;
    };
    const int32_t off_f = nc, off_n = nc + nf;
    if (i < nc) {
        const int32_t K = (int32_t)i;
        const double w = dt / phi_cell[K];
        double out = 0.0;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const double F = F_cell[8 * (int64_t)K + a];
            if (F > 0.0) out += F;
            else if (F < 0.0) emit(off_n + hex8[8 * (int64_t)K + a], -w * F);
        }
        const unsigned mask = fmask[K];
        if (mask)
            for (int f = 0; f < 6; ++f)
                if ((mask >> f) & 1u) {
                    const int32_t sg = cell_frac[6 * (int64_t)K + f];
                    const int side = frac_cell[2 * (int64_t)sg] == K ? 0 : 1;
                    const double F = F_cell_frac[2 * (int64_t)sg + side];
                    if (F > 0.0) out += F;
                    else if (F < 0.0) emit(off_f + sg, -w * F);
                }
        d = 1.0 - w * out;
    } else if (i < (int64_t)nc + nf) {
        const int32_t f = (int32_t)(i - nc);
        const double w = dt / phi_frac[f];
        double out = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double F = F_frac[4 * (int64_t)f + q];
            if (F > 0.0) out += F;
            else if (F < 0.0) emit(off_n + frac_nodes[4 * (int64_t)f + q], -w * F);
        }
        for (int side = 0; side < 2; ++side) {
            const int32_t K = frac_cell[2 * (int64_t)f + side];
            if (K < 0) continue;
            const double F = F_cell_frac[2 * (int64_t)f + side];
            if (F < 0.0) out -= F;
            else if (F > 0.0) emit(K, w * F);
        }
        // a well: production leaves at c_sigma, injection enters from the
        // constant control volume (index total, concentration 1)
        if (wout) out += wout[f];
        if (wsrc && wsrc[f] > 0.0) emit(total, w * wsrc[f]);
        d = 1.0 - w * out;
    } else {
        const int32_t s = (int32_t)(i - nc - nf);
        if (!dirichlet[s]) {
            const double w = dt / phi_node[s];
            double in_neg = 0.0;
            for (int32_t q = ncp[s]; q < ncp[s + 1]; ++q) {
                const double F = F_cell[ncl[q]];
                if (F < 0.0) in_neg += F;
                else if (F > 0.0) emit(ncl[q] >> 3, w * F);
            }
            for (int32_t q = nfp[s]; q < nfp[s + 1]; ++q) {
                const double F = F_frac[nfl[q]];
                if (F < 0.0) in_neg += F;
                else if (F > 0.0) emit(off_f + (nfl[q] >> 2), w * F);
            }
            d = 1.0 + w * in_neg;
        }
    }
    tdiag[i] = d;
}

// c_out = c + theta (T c - c); theta = 1 is the plain step.  Slot t of a
// slice holds row (slice, meta >> 8) with meta & 255 entries.
// Column compression of the upwind operator, one wavefront per slice: when the
// columns of a slice's entries lie within 65536 of their minimum, the slice
// stores 16-bit offsets from that minimum (tbase[slice] = the minimum) and
// the sweep reads 2 bytes per column instead of 4; otherwise tbase = -1 and
// the 32-bit columns are read.  Cells and nodes of a slice are neighbours in
// the mesh, so nearly every slice qualifies.
__global__ __launch_bounds__(kSliceRows) void upwind_pack_kernel(int32_t nrow, const int64_t *__restrict__ slice_ptr,
                                                                 const uint16_t *__restrict__ meta,
                                                                 const int32_t *__restrict__ tcol,
                                                                 uint16_t *__restrict__ tcol16,
                                                                 int32_t *__restrict__ tbase) {
    const int32_t sl = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t b0 = slice_ptr[sl], b1 = slice_ptr[sl + 1];
    int32_t lo = INT32_MAX, hi = -1;
    for (int64_t q = b0 + lane; q < b1; q += kSliceRows) {
        const int32_t c = tcol[q];
        lo = min(lo, c);
        hi = max(hi, c);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o, 64));
        hi = max(hi, __shfl_xor(hi, o, 64));
    }
    const bool compact = hi < 0 || (int64_t)hi - lo <= 65535;
    if (compact)
        for (int64_t q = b0 + lane; q < b1; q += kSliceRows) tcol16[q] = (uint16_t)(tcol[q] - lo);
    if (lane == 0) tbase[sl] = compact ? (hi < 0 ? 0 : lo) : -1;
}

// One explicit step, c_out = T c_in (theta < 1: the shortened last step of a
// final-time run, c_in + theta (T c_in - c_in)).  Lane l of slice sl handles
// the row named by meta[sl*64 + l], which has m & 255 entries; level k starts
// after the entries of the lower levels, whose sizes (the lanes with more than
// k' entries) a ballot over the wavefront gives, so the packed layout needs
// no stored level offsets.  Lanes are sorted longest first: lane 0 holds the
// slice's widest row.
// The row of one lane: level k of the slice starts at the sum of the sizes of
// the levels below it (a ballot gives each size: the lanes with more than k
// entries).  A lane without entry k loads a clamped address inside the slice
// (lines the wavefront fetches anyway) and adds nothing, so the loop has no
// branches and keeps the loads of four levels in flight.  A slice without
// entries (last < level0) has width 0 and loads nothing.
template <bool C16>
__device__ __forceinline__ double upwind_row(const UpwindOp &T, const double *__restrict__ c_in, int cnt,
                                             int width, int64_t level0, int64_t last, int lane, int32_t cb,
                                             double a0) {
    double a1 = 0.0, a2 = 0.0, a3 = 0.0;
    auto col = [&](int64_t q) -> int32_t { return C16 ? cb + (int32_t)T.tcol16[q] : T.tcol[q]; };
    int64_t lv = level0;  // start of level k
    int k = 0;
    for (; k + 3 < width; k += 4) {
        const int n0 = __popcll(__ballot(cnt > k)), n1 = __popcll(__ballot(cnt > k + 1));
        const int n2 = __popcll(__ballot(cnt > k + 2)), n3 = __popcll(__ballot(cnt > k + 3));
        const int64_t p0 = lv + lane, p1 = p0 + n0, p2 = p1 + n1, p3 = p2 + n2;
        const int64_t q0 = p0 < last ? p0 : last, q1 = p1 < last ? p1 : last;
        const int64_t q2 = p2 < last ? p2 : last, q3 = p3 < last ? p3 : last;
        // columns, values, then the gathers: twelve loads in flight
        const int32_t c0 = col(q0), c1 = col(q1), c2 = col(q2), c3 = col(q3);
        const double v0 = T.tval[q0], v1 = T.tval[q1], v2 = T.tval[q2], v3 = T.tval[q3];
        const double x0 = c_in[c0], x1 = c_in[c1], x2 = c_in[c2], x3 = c_in[c3];
        a1 += cnt > k ? v0 * x0 : 0.0;
        a2 += cnt > k + 1 ? v1 * x1 : 0.0;
        a3 += cnt > k + 2 ? v2 * x2 : 0.0;
        a0 += cnt > k + 3 ? v3 * x3 : 0.0;
        lv += n0 + n1 + n2 + n3;
    }
    for (; k < width; ++k) {
        const int n0 = __popcll(__ballot(cnt > k));
        const int64_t p0 = lv + lane, q0 = p0 < last ? p0 : last;
        const double v0 = T.tval[q0] * c_in[col(q0)];
        a1 += cnt > k ? v0 : 0.0;
        lv += n0;
    }
    return (a0 + a1) + (a2 + a3);
}

// The step for block b of a launch over T (b mod 8 names the XCD: the
// hardware deals the blocks out in turn, so a batched launch starts each
// operator's blocks at a multiple of 8).  Item q of XCD x is its run of A
// slices and its run of B slices merged in proportion: item q is an A slice
// iff floor((q+1) a / w) > floor(q a / w), and floor(q a / w) A slices come
// before it.  Every other step sweeps each XCD's run backwards, so that it
// starts on the slices the previous step read last, which the last-level
// cache still holds.
__device__ inline void transport_step_block(const UpwindOp &T, const double *__restrict__ c_in,
                                            double *__restrict__ c_out, double theta, int backward, int32_t b) {
    const int x = b & 7;
    const int32_t q0 = 4 * (b >> 3) + (int32_t)(threadIdx.x >> 6);
    const int32_t a = T.xlo[x + 1] - T.xlo[x], w = a + T.ylo[x + 1] - T.ylo[x];
    const int lane = threadIdx.x & (kSliceRows - 1);
    if (q0 >= w) return;  // whole wavefronts
    const int32_t q = backward ? w - 1 - q0 : q0;
    const int32_t na = (int32_t)((int64_t)q * a / w);
    const int32_t sl = (int32_t)((int64_t)(q + 1) * a / w) > na ? T.xlo[x] + na : T.ylo[x] + (q - na);
    const int32_t t = sl * kSliceRows + lane;
    const uint16_t m = T.meta[t];
    const int32_t i = sl * kSliceRows + (m >> 8);
    const bool row = i < T.nrow;
    const int cnt = row ? (m & 255) : 0;
    const int width = __shfl(cnt, 0, kSliceRows);
    const int64_t level0 = T.slice_ptr[sl], last = T.slice_ptr[sl + 1] - 1;
    const int32_t cb = T.tbase[sl];
    const double ci = row ? c_in[i] : 0.0;
    const double d = row ? T.tdiag[i] * ci : 0.0;
    const double acc = cb >= 0 ? upwind_row<true>(T, c_in, cnt, width, level0, last, lane, cb, d)
                               : upwind_row<false>(T, c_in, cnt, width, level0, last, lane, cb, d);
    if (row) c_out[i] = (theta == 1.0) ? acc : ci + theta * (acc - ci);
}

__global__ __launch_bounds__(256) void transport_step_kernel(UpwindOp T, const double *__restrict__ c_in,
                                                             double *__restrict__ c_out, double theta, int backward) {
    transport_step_block(T, c_in, c_out, theta, backward, (int32_t)blockIdx.x);
}

// One step of several operators in one launch: operator j takes blocks
// [B.blk[j], B.blk[j + 1]), each block the same work as in its own launch.
__global__ __launch_bounds__(256) void transport_batch_kernel(TransportBatch B) {
    const int32_t b = (int32_t)blockIdx.x;
    int j = 0;
    while (j + 1 < B.n && b >= B.blk[j + 1]) ++j;
    const TransportJob &J = B.job[j];
    transport_step_block(J.T, J.c_in, J.c_out, J.theta, J.backward, b - B.blk[j]);
}

// Cost of the slices before slice s: the bytes the sweep moves for them
// (12 per entry, 32 per row).  Thread x < 9 splits segment A = [0, sa),
// thread 9 + x segment B = [sa, nslice): the first slice whose cost from the
// segment's start reaches x/8 of the segment's.  The two segments are swept
// interleaved only where their mean row lengths differ by more than 3/2
// (tetrahedra: 2 against 12 entries per row); where they are alike
// (hexahedra: 4 and 4), one contiguous run per XCD over all slices moves
// fewer bytes (at 192^3, 1158 against 1221 MB per step: interleaving puts
// two fronts into each XCD's L2, and the gathers of a z-layer's neighbours
// then miss more often), so segment A is then the whole range and B empty.
__global__ __launch_bounds__(64) void xcd_split_kernel(int32_t nslice, int32_t sa,
                                                       const int64_t *__restrict__ slice_ptr,
                                                       int32_t *__restrict__ xlo) {
    const int t = threadIdx.x, x = t % 9;
    if (t >= 18) return;
    const double ma = sa > 0 ? (double)slice_ptr[sa] / sa : 0.0;
    const double mb = nslice > sa ? (double)(slice_ptr[nslice] - slice_ptr[sa]) / (nslice - sa) : 0.0;
    const bool apart = fmax(ma, mb) > 1.5 * fmin(ma, mb);
    if (!apart) sa = nslice;
    const int32_t b0 = t < 9 ? 0 : sa, b1 = t < 9 ? sa : nslice;
    auto cost = [&](int32_t sl) { return 12 * slice_ptr[sl] + 32 * (int64_t)kSliceRows * sl; };
    const int64_t base = cost(b0), want = (cost(b1) - base) * x / 8;
    int32_t lo = b0, hi = b1;
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (cost(mid) - base < want) lo = mid + 1; else hi = mid;
    }
    xlo[t] = x == 8 ? b1 : lo;
}

// One explicit step without the upwind operator (the entry point for callers
// that cannot allocate): every control volume gathers the upwind fluxes
// H = c_up F of eq darcyfluxH from the resident Darcy fluxes, one thread per
// control volume.  Cells read their 8 node fluxes and fracture faces; a
// fracture face its 4 node fluxes, its (at most 2) cells and its well; a node
// its cells and faces through the node -> (cell, slot) and node -> (face, slot)
// lists.  Outflow leaves at the control volume's own concentration, inflow
// enters at the upstream one's; a well injects c_inj Q^+ (wsrc) and produces
// Q^- (wout) at the face's concentration.  Dirichlet nodes keep their value
// (the state holds c_bar there).  The result is the step of
// transport_step_kernel up to the order of the additions:
//   c_out = c_in - theta * dt / phi * (sum of the control volume's H).
__global__ __launch_bounds__(kT) void transport_gather_kernel(
    int32_t nc, int32_t nf, int32_t nn, const int32_t *__restrict__ hex8, const uint8_t *__restrict__ fmask,
    const int32_t *__restrict__ cell_frac, const int32_t *__restrict__ frac_cell,
    const int32_t *__restrict__ frac_nodes, const uint8_t *__restrict__ dirichlet, const int32_t *__restrict__ ncp,
    const int32_t *__restrict__ ncl, const int32_t *__restrict__ nfp, const int32_t *__restrict__ nfl,
    const double *__restrict__ F_cell, const double *__restrict__ F_cell_frac, const double *__restrict__ F_frac,
    const double *__restrict__ wsrc, const double *__restrict__ wout, const double *__restrict__ phi_cell,
    const double *__restrict__ phi_frac, const double *__restrict__ phi_node, const double *__restrict__ dtp,
    double theta, const double *__restrict__ c_in, double *__restrict__ c_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t off_f = nc, off_n = (int64_t)nc + nf;
    if (i >= off_n + nn) return;
    const double tdt = theta * dtp[3];
    const double ci = c_in[i];
    double sum = 0.0;  // sum of the outgoing H of control volume i
    double phi;
    if (i < nc) {
        const int32_t K = (int32_t)i;
        phi = phi_cell[K];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const double F = F_cell[8 * (int64_t)K + a];
            sum += F > 0.0 ? ci * F : c_in[off_n + hex8[8 * (int64_t)K + a]] * F;
        }
        const unsigned mask = fmask[K];
        if (mask)
            for (int f = 0; f < 6; ++f)
                if ((mask >> f) & 1u) {
                    const int32_t sg = cell_frac[6 * (int64_t)K + f];
                    const int side = frac_cell[2 * (int64_t)sg] == K ? 0 : 1;
                    const double F = F_cell_frac[2 * (int64_t)sg + side];
                    sum += F > 0.0 ? ci * F : c_in[off_f + sg] * F;
                }
    } else if (i < off_n) {
        const int32_t f = (int32_t)(i - off_f);
        phi = phi_frac[f];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double F = F_frac[4 * (int64_t)f + q];
            sum += F > 0.0 ? ci * F : c_in[off_n + frac_nodes[4 * (int64_t)f + q]] * F;
        }
        for (int side = 0; side < 2; ++side) {
            const int32_t K = frac_cell[2 * (int64_t)f + side];
            if (K < 0) continue;
            const double F = F_cell_frac[2 * (int64_t)f + side];  // from K into the face
            sum -= F > 0.0 ? c_in[K] * F : ci * F;
        }
        if (wout) sum += ci * wout[f];
        if (wsrc) sum -= wsrc[f];
    } else {
        const int32_t s = (int32_t)(i - off_n);
        if (dirichlet[s]) {
            c_out[i] = ci;
            return;
        }
        phi = phi_node[s];
        for (int32_t q = ncp[s]; q < ncp[s + 1]; ++q) {
            const double F = F_cell[ncl[q]];  // from cell ncl[q] / 8 into the node
            sum -= F > 0.0 ? c_in[ncl[q] >> 3] * F : ci * F;
        }
        for (int32_t q = nfp[s]; q < nfp[s + 1]; ++q) {
            const double F = F_frac[nfl[q]];  // from face nfl[q] / 4 into the node
            sum -= F > 0.0 ? c_in[off_f + (nfl[q] >> 2)] * F : ci * F;
        }
    }
    c_out[i] = ci - (tdt / phi) * sum;
}

// Scratch of the allocation-free transport entry point: the CFL partial minima
// (3 per reduction block) and the four values of dt_out.  One copy per device,
// held until the process ends; host code reaches it only through the address
// that hipGetSymbolAddress returns for the current device.
constexpr size_t kNoallocScratchDoubles = 3 * (size_t)kReduceBlocks + 8;
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

double *noalloc_scratch(size_t *doubles) {
    int dev = 0;
    VAG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Error(VAG_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        VAG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error(VAG_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *doubles = kNoallocScratchDoubles;
    return g_scratch_ptr[dev];
}

__global__ void set_dirichlet_kernel(int32_t nn, int32_t offset, const uint8_t *__restrict__ dirichlet,
                                     const double *__restrict__ c_bar, double *__restrict__ c) {
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nn && dirichlet[s]) c[offset + s] = c_bar[s];
}

// ---------------------------------------------------------------------------
// general cells: the same steps on the incidence lists of the control volumes
// ---------------------------------------------------------------------------
// Flux F_e leaves the first control volume of edge e when positive; at the
// far end (edge & 1) it counts with the opposite sign.
__device__ inline double inc_flux(const GenInc &I, const double *F, int64_t q) {
    const int32_t e = I.edge[q];
    const double f = F[e >> 1];
    return (e & 1) ? -f : f;
}

__global__ __launch_bounds__(kCflT) void gen_cfl_kernel(GenInc I, const double *__restrict__ F,
                                                     const double *__restrict__ wout,
                                                     const double *__restrict__ phi_cell,
                                                     const double *__restrict__ phi_frac,
                                                     const double *__restrict__ phi_node, double *__restrict__ parts) {
    const double inf = __builtin_inf();
    double v[3] = {inf, inf, inf};
    const int64_t off_f = I.nc, off_n = (int64_t)I.nc + I.nf, total = off_n + I.nn;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int kind = i < off_f ? 0 : (i < off_n ? 1 : 2);
        if (kind == 2 && I.dirichlet[i - off_n]) continue;
        double o = 0.0;
        for (int64_t q = I.ptr[i]; q < I.ptr[i + 1]; ++q) o += fmax(inc_flux(I, F, q), 0.0);
        if (kind == 1 && wout) o += wout[i - off_f];
        if (o > 0.0) {
            const double phi = kind == 0 ? phi_cell[i] : (kind == 1 ? phi_frac[i - off_f] : phi_node[i - off_n]);
            v[kind] = fmin(v[kind], phi / o);
        }
    }
    block_partials<OpMin, 3, kCflT>(v, parts, gridDim.x);
}

// entries of row i: one per inflow (negative outgoing flux), plus a well's
// injection on a fracture face; none for a Dirichlet node
__device__ inline int gen_row_count(const GenInc &I, const double *F, const double *wsrc, int64_t i) {
    const int64_t off_f = I.nc, off_n = (int64_t)I.nc + I.nf;
    if (i >= off_n && I.dirichlet[i - off_n]) return 0;
    int c = 0;
    for (int64_t q = I.ptr[i]; q < I.ptr[i + 1]; ++q) c += inc_flux(I, F, q) < 0.0;
    if (wsrc && i >= off_f && i < off_n) c += wsrc[i - off_f] > 0.0;
    return c;
}

__global__ __launch_bounds__(kSliceRows) void gen_upwind_count_kernel(GenInc I, const double *__restrict__ F,
                                                                      const double *__restrict__ wsrc,
                                                                      int32_t *__restrict__ slice_width,
                                                                      uint16_t *__restrict__ meta,
                                                                      int32_t *__restrict__ slice_nnz) {
    const int lane = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kSliceRows + lane;
    const int64_t total = (int64_t)I.nc + I.nf + I.nn;
    const int c = i < total ? gen_row_count(I, F, wsrc, i) : 0;
    slice_sort_rows(c, lane, slice_width, meta, slice_nnz);
}

// Row i of the upwind operator: T_ij = w_i (inflow from j), T_ii = 1 - w_i
// (outflow), w_i = dt / phi_i; a well's production counts as outflow of its
// face and its injection as an entry on the constant control volume.
__global__ __launch_bounds__(kSliceRows) void gen_upwind_fill_kernel(
    GenInc I, const double *__restrict__ F, const double *__restrict__ wsrc, const double *__restrict__ wout,
    const double *__restrict__ phi_cell, const double *__restrict__ phi_frac, const double *__restrict__ phi_node,
    const double *__restrict__ dtp, const int64_t *__restrict__ slice_ptr, const uint16_t *__restrict__ meta,
    int32_t *__restrict__ tcol, double *__restrict__ tval, double *__restrict__ tdiag) {
    __shared__ uint8_t cnts[kSliceRows];
    __shared__ int32_t level_off[257];
    const int lane = threadIdx.x;
    const int src = slice_levels(meta, cnts, level_off);
    const int64_t i = (int64_t)blockIdx.x * kSliceRows + src;
    const int64_t off_f = I.nc, off_n = (int64_t)I.nc + I.nf, total = off_n + I.nn;
    if (i >= total) return;
    const int64_t base = slice_ptr[blockIdx.x] + lane;
    double d = 1.0;
    if (!(i >= off_n && I.dirichlet[i - off_n])) {
        const double phi = i < off_f ? phi_cell[i] : (i < off_n ? phi_frac[i - off_f] : phi_node[i - off_n]);
        const double w = dtp[3] / phi;
        double out = 0.0;
        int k = 0;
        for (int64_t q = I.ptr[i]; q < I.ptr[i + 1]; ++q) {
            const double f = inc_flux(I, F, q);
            if (f > 0.0) {
                out += f;
            } else if (f < 0.0) {
                tcol[base + level_off[k]] = I.other[q];
                tval[base + level_off[k]] = -w * f;
                ++k;
            }
        }
        if (i >= off_f && i < off_n) {
            if (wout) out += wout[i - off_f];
            if (wsrc && wsrc[i - off_f] > 0.0) {
                tcol[base + level_off[k]] = (int32_t)total;
                tval[base + level_off[k]] = w * wsrc[i - off_f];
                ++k;
            }
        }
        d = 1.0 - w * out;
    }
    tdiag[i] = d;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_node_pressure(hipStream_t s, int32_t nn, const int32_t *node_unk, const double *x, const double *p_bar,
                          double *u_node) {
    hipLaunchKernelGGL(node_pressure_kernel, dim3(nb(nn, kT)), dim3(kT), 0, s, nn, node_unk, x, p_bar, u_node);
    VAG_HIP(hipGetLastError());
}
void launch_cell_flux(hipStream_t s, int32_t nc, const int32_t *hex8, const uint8_t *fmask,
                      const int32_t *cell_frac, const int32_t *frac_cell, const double *aK, const double *rK,
                      const double *AKK, const double *fside, const double *u_node, const double *u_frac,
                      double *u_cell, double *F_cell, double *F_cell_frac) {
    hipLaunchKernelGGL(cell_flux_kernel, dim3(nb(nc, 128)), dim3(128), 0, s, nc, hex8, fmask, cell_frac, frac_cell,
                       aK, rK, AKK, fside, u_node, u_frac, u_cell, F_cell, F_cell_frac);
    VAG_HIP(hipGetLastError());
}
void launch_frac_flux(hipStream_t s, int32_t nf, const int32_t *frac_nodes, const double *A5, const double *u_node,
                      const double *u_frac, double *F_frac) {
    if (nf <= 0) return;
    hipLaunchKernelGGL(frac_flux_kernel, dim3(nb(nf, kT)), dim3(kT), 0, s, nf, frac_nodes, A5, u_node, u_frac,
                       F_frac);
    VAG_HIP(hipGetLastError());
}
void launch_porous(hipStream_t s, int32_t nc, int32_t nf, int32_t nn, const int32_t *hex8,
                   const int32_t *frac_nodes, const uint8_t *dirichlet, const uint8_t *frac_node,
                   const int32_t *node_cell_ptr, const int32_t *node_cell, const int32_t *node_frac_ptr,
                   const int32_t *node_frac, const double *vol, const double *poro, const double *area,
                   const double *fwidth, const double *fporo, const double *perm, const double *fperm,
                   const double *pmax, double *phi_cell, double *phi_frac, double *phi_node) {
    const int64_t total = (int64_t)nc + nf + nn;
    hipLaunchKernelGGL(porous_kernel, dim3(nb(total, kT)), dim3(kT), 0, s, nc, nf, nn, hex8, frac_nodes, dirichlet,
                       frac_node, node_cell_ptr, node_cell, node_frac_ptr, node_frac, vol, poro, area, fwidth,
                       fporo, perm, fperm, pmax, phi_cell, phi_frac, phi_node);
    VAG_HIP(hipGetLastError());
}
void launch_node_pmax(hipStream_t s, int32_t nn, const uint8_t *frac_node, const int32_t *node_cell_ptr,
                      const int32_t *node_cell, const int32_t *node_frac_ptr, const int32_t *node_frac,
                      const double *perm, const double *fperm, double *pmax) {
    if (nn <= 0) return;
    hipLaunchKernelGGL(node_pmax_kernel, dim3(nb(nn, kT)), dim3(kT), 0, s, nn, frac_node, node_cell_ptr, node_cell,
                       node_frac_ptr, node_frac, perm, fperm, pmax);
    VAG_HIP(hipGetLastError());
}
void launch_cfl(hipStream_t s, int32_t nc, int32_t nf, int32_t nn, const int32_t *hex8, const uint8_t *fmask,
                const int32_t *cell_frac, const int32_t *frac_cell, const uint8_t *dirichlet,
                const int32_t *node_cell_ptr, const int32_t *node_cell, const int32_t *node_frac_ptr,
                const int32_t *node_frac, const double *F_cell, const double *F_cell_frac, const double *F_frac,
                const double *wout, const double *phi_cell, const double *phi_frac, const double *phi_node,
                double cfl, double *parts, double *dt_out) {
    const int64_t total = (int64_t)nc + nf + nn;
    const unsigned G = reduce_grid(total, kCflT);
    hipLaunchKernelGGL(cfl_kernel, dim3(G), dim3(kCflT), 0, s, nc, nf, nn, hex8, fmask, cell_frac, frac_cell,
                       dirichlet, node_cell_ptr, node_cell, node_frac_ptr, node_frac, F_cell, F_cell_frac, F_frac,
                       wout, phi_cell, phi_frac, phi_node, parts);
    hipLaunchKernelGGL(cfl_finish_kernel, dim3(1), dim3(kT), 0, s, parts, (int)G, cfl, dt_out);
    VAG_HIP(hipGetLastError());
}
void launch_upwind_count(hipStream_t s, int32_t nc, int32_t nf, int32_t nn, const uint8_t *fmask,
                         const int32_t *cell_frac, const int32_t *frac_cell, const uint8_t *dirichlet,
                         const int32_t *node_cell_ptr, const int32_t *node_cell, const int32_t *node_frac_ptr,
                         const int32_t *node_frac, const double *F_cell, const double *F_cell_frac,
                         const double *F_frac, const double *wsrc, int32_t *slice_width, uint16_t *meta,
                         int32_t *slice_nnz) {
    const int64_t total = (int64_t)nc + nf + nn;
    hipLaunchKernelGGL(upwind_count_kernel, dim3(nb(total, kSliceRows)), dim3(kSliceRows), 0, s, nc, nf, nn, fmask,
                       cell_frac, frac_cell, dirichlet, node_cell_ptr, node_cell, node_frac_ptr, node_frac, F_cell,
                       F_cell_frac, F_frac, wsrc, slice_width, meta, slice_nnz);
    VAG_HIP(hipGetLastError());
}
void launch_slice_scan(hipStream_t s, int32_t nslice, const int32_t *slice_width, int per_width, int64_t *slice_ptr,
                       const int32_t *slice_nnz, unsigned long long *total) {
    hipLaunchKernelGGL(slice_scan_kernel, dim3(1), dim3(1024), 0, s, nslice, slice_width, per_width, slice_ptr,
                       slice_nnz, total);
    VAG_HIP(hipGetLastError());
}
void launch_upwind_fill(hipStream_t s, int32_t nc, int32_t nf, int32_t nn, const int32_t *hex8,
                        const uint8_t *fmask, const int32_t *cell_frac, const int32_t *frac_cell,
                        const int32_t *frac_nodes, const uint8_t *dirichlet, const int32_t *node_cell_ptr,
                        const int32_t *node_cell, const int32_t *node_frac_ptr, const int32_t *node_frac,
                        const double *F_cell, const double *F_cell_frac, const double *F_frac, const double *wsrc,
                        const double *wout, const double *phi_cell, const double *phi_frac, const double *phi_node,
                        const double *dt, const int64_t *slice_ptr, const uint16_t *meta, int32_t *tcol,
                        double *tval, double *tdiag) {
    const int64_t total = (int64_t)nc + nf + nn;
    hipLaunchKernelGGL(upwind_fill_kernel, dim3(nb(total, kSliceRows)), dim3(kSliceRows), 0, s, nc, nf, nn, hex8,
                       fmask, cell_frac, frac_cell, frac_nodes, dirichlet, node_cell_ptr, node_cell, node_frac_ptr,
                       node_frac, F_cell, F_cell_frac, F_frac, wsrc, wout, phi_cell, phi_frac, phi_node, dt,
                       slice_ptr, meta, tcol, tval, tdiag);
    VAG_HIP(hipGetLastError());
}
void launch_upwind_pack(hipStream_t s, const UpwindOp &T, uint16_t *tcol16, int32_t *tbase) {
    const int64_t nslice = (T.nrow + kSliceRows - 1) / kSliceRows;
    if (nslice <= 0) return;
    hipLaunchKernelGGL(upwind_pack_kernel, dim3((unsigned)nslice), dim3(kSliceRows), 0, s, T.nrow, T.slice_ptr, T.meta,
                       T.tcol, tcol16, tbase);
    VAG_HIP(hipGetLastError());
}
void launch_xcd_split(hipStream_t s, int32_t nslice, int32_t sa, const int64_t *slice_ptr, int32_t *xlo) {
    hipLaunchKernelGGL(xcd_split_kernel, dim3(1), dim3(64), 0, s, nslice, sa, slice_ptr, xlo);
    VAG_HIP(hipGetLastError());
}
int32_t transport_step_blocks(const UpwindOp &T) {
    int32_t per_xcd = 0;  // blocks per XCD: the longest merged run, 4 slices per block
    for (int x = 0; x < 8; ++x)
        per_xcd = std::max(per_xcd, (T.xlo[x + 1] - T.xlo[x] + T.ylo[x + 1] - T.ylo[x] + 3) / 4);
    return 8 * per_xcd;
}
void launch_transport_step(hipStream_t s, const UpwindOp &T, const double *c_in, double *c_out, double theta,
                           bool backward) {
    const int32_t nb = transport_step_blocks(T);
    if (nb <= 0) return;
    hipLaunchKernelGGL(transport_step_kernel, dim3((unsigned)nb), dim3(256), 0, s, T, c_in, c_out, theta,
                       backward ? 1 : 0);
    VAG_HIP(hipGetLastError());
}
void launch_transport_batch(hipStream_t s, TransportBatch &B) {
    if (B.n < 1 || B.n > kBatchJobs) throw Error(VAG_ERR_ARG, "transport batch size out of range");
    B.blk[0] = 0;
    for (int j = 0; j < B.n; ++j) B.blk[j + 1] = B.blk[j] + transport_step_blocks(B.job[j].T);
    if (B.blk[B.n] <= 0) return;
    hipLaunchKernelGGL(transport_batch_kernel, dim3((unsigned)B.blk[B.n]), dim3(256), 0, s, B);
    VAG_HIP(hipGetLastError());
}
void launch_transport_gather(hipStream_t s, int32_t nc, int32_t nf, int32_t nn, const int32_t *hex8,
                             const uint8_t *fmask, const int32_t *cell_frac, const int32_t *frac_cell,
                             const int32_t *frac_nodes, const uint8_t *dirichlet, const int32_t *node_cell_ptr,
                             const int32_t *node_cell, const int32_t *node_frac_ptr, const int32_t *node_frac,
                             const double *F_cell, const double *F_cell_frac, const double *F_frac,
                             const double *wsrc, const double *wout, const double *phi_cell, const double *phi_frac,
                             const double *phi_node, const double *dt, double theta, const double *c_in,
                             double *c_out) {
    const int64_t total = (int64_t)nc + nf + nn;
    if (total <= 0) return;
    hipLaunchKernelGGL(transport_gather_kernel, dim3(nb(total, kT)), dim3(kT), 0, s, nc, nf, nn, hex8, fmask,
                       cell_frac, frac_cell, frac_nodes, dirichlet, node_cell_ptr, node_cell, node_frac_ptr, node_frac,
                       F_cell, F_cell_frac, F_frac, wsrc, wout, phi_cell, phi_frac, phi_node, dt, theta, c_in, c_out);
    VAG_HIP(hipGetLastError());
}
void launch_set_dirichlet(hipStream_t s, int32_t nn, int32_t offset, const uint8_t *dirichlet, const double *c_bar,
                          double *c) {
    hipLaunchKernelGGL(set_dirichlet_kernel, dim3(nb(nn, 256)), dim3(256), 0, s, nn, offset, dirichlet, c_bar, c);
    VAG_HIP(hipGetLastError());
}

void launch_gen_cfl(hipStream_t s, const GenInc &I, const double *F, const double *wout, const double *phi_cell,
                    const double *phi_frac, const double *phi_node, double cfl, double *parts, double *dt_out) {
    const int64_t total = (int64_t)I.nc + I.nf + I.nn;
    const unsigned G = reduce_grid(total, kCflT);
    hipLaunchKernelGGL(gen_cfl_kernel, dim3(G), dim3(kCflT), 0, s, I, F, wout, phi_cell, phi_frac, phi_node, parts);
    hipLaunchKernelGGL(cfl_finish_kernel, dim3(1), dim3(kT), 0, s, parts, (int)G, cfl, dt_out);
    VAG_HIP(hipGetLastError());
}
void launch_gen_upwind_count(hipStream_t s, const GenInc &I, const double *F, const double *wsrc,
                             int32_t *slice_width, uint16_t *meta, int32_t *slice_nnz) {
    const int64_t total = (int64_t)I.nc + I.nf + I.nn;
    hipLaunchKernelGGL(gen_upwind_count_kernel, dim3(nb(total, kSliceRows)), dim3(kSliceRows), 0, s, I, F, wsrc,
                       slice_width, meta, slice_nnz);
    VAG_HIP(hipGetLastError());
}
void launch_gen_upwind_fill(hipStream_t s, const GenInc &I, const double *F, const double *wsrc, const double *wout,
                            const double *phi_cell, const double *phi_frac, const double *phi_node, const double *dt,
                            const int64_t *slice_ptr, const uint16_t *meta, int32_t *tcol, double *tval,
                            double *tdiag) {
    const int64_t total = (int64_t)I.nc + I.nf + I.nn;
    hipLaunchKernelGGL(gen_upwind_fill_kernel, dim3(nb(total, kSliceRows)), dim3(kSliceRows), 0, s, I, F, wsrc,
                       wout, phi_cell, phi_frac, phi_node, dt, slice_ptr, meta, tcol, tval, tdiag);
    VAG_HIP(hipGetLastError());
}

}  // namespace vag
