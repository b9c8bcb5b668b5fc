// The sparsity pattern of the cell-eliminated system (eq eqschur) of a
// hexahedral mesh, built on the device.  After the cell elimination the
// unknowns of a cell (its free nodes and fracture faces) are pairwise
// coupled, so the row of a free node is the union of the unknowns of its
// cells, plus the free nodes of every eliminated fracture-face group that
// holds the node (the group's Schur complement couples them); the row of a
// kept fracture face is the union over its one or two cells.
//
// Three passes, one thread per row (natural numbering: free nodes by node
// index, then kept faces by face index):
//  1. an upper bound of the row's length (the candidates before duplicates
//     go), scanned into offsets of a scratch array;
//  2. the candidates inserted one by one into the row's sorted list,
//     duplicates skipped: the row and its exact length.  The list lives in
//     registers (kRegCols entries, each insertion a fixed sequence of
//     compare-and-select steps); a longer row is built again in the scratch
//     array by a second kernel, with the same insertions in global memory;
//  3. after the host has renumbered the rows from their lengths, each row
//     mapped to the system numbering and sorted into the CSR layout.
// The node -> cell lists that pass 1 and 2 (and the assembly) read are built
// here as well.
#include "amg.h"
#include "vag_internal.h"

namespace vag {

namespace {
constexpr int kPT = 256;

// the row of thread i: a free node (i < nn) or a kept fracture face; -1 if none
__device__ inline int32_t pattern_row(const PatArgs &g, int64_t i) {
    if (i < g.nn) return g.node_unk[i];
    const int32_t u = g.frac_unk[i - g.nn];
    return u < g.nunk ? u : -1;
}

// calls f(K) for each cell around the row's node (or beside its face)
template <class F>
__device__ inline void pattern_cells(const PatArgs &g, int64_t i, F &&f) {
    if (i < g.nn) {
        for (int32_t q = g.node_cell_ptr[i]; q < g.node_cell_ptr[i + 1]; ++q) f(g.node_cell[q] >> 3);
    } else {
        const int64_t sg = i - g.nn;
        for (int side = 0; side < 2; ++side) {
            const int32_t K = g.frac_cell[2 * sg + side];
            if (K >= 0) f(K);
        }
    }
}
}  // namespace

__global__ __launch_bounds__(kPT) void pattern_bound_kernel(PatArgs g, int32_t *__restrict__ ub) {
    const int64_t i = (int64_t)blockIdx.x * kPT + threadIdx.x;
    if (i >= (int64_t)g.nn + g.nf) return;
    const int32_t row = pattern_row(g, i);
    if (row < 0) return;
    int32_t c = 0;
    pattern_cells(g, i, [&](int32_t K) { c += 8 + __popc(g.fmask[K]); });
    if (i < g.nn)
        for (int32_t q = g.node_grp_ptr[row]; q < g.node_grp_ptr[row + 1]; ++q) {
            const int32_t G = g.node_grp[q];
            c += g.grp_nptr[G + 1] - g.grp_nptr[G];
        }
    ub[row] = c;
}

namespace {
constexpr int kRegCols = 32;

// a sorted list of distinct columns held in registers; m counts the distinct
// columns added, also past kRegCols (then the list has lost its largest ones
// and the row goes to the global-memory kernel)
struct RegList {
    int32_t a[kRegCols];
    int32_t m = 0;
    __device__ RegList() {
#pragma unroll
        for (int k = 0; k < kRegCols; ++k) a[k] = INT32_MAX;
    }
    // c inserted where it keeps the order (every entry above it moves up one)
    __device__ void insert(int32_t c) {
#pragma unroll
        for (int k = kRegCols - 1; k > 0; --k) a[k] = a[k - 1] > c ? a[k - 1] : (a[k] > c ? c : a[k]);
        a[0] = a[0] > c ? c : a[0];
        ++m;
    }
    __device__ void add(int32_t c) {
        bool here = false;
#pragma unroll
        for (int k = 0; k < kRegCols; ++k) here |= a[k] == c;
        if (!here) insert(c);
    }
};

// calls add(c) for every candidate column of the row (natural numbering)
template <class Add>
__device__ inline void pattern_candidates(const PatArgs &g, int64_t i, int32_t row, Add &&add) {
    pattern_cells(g, i, [&](int32_t K) {
        const int32_t *cn = g.hex8 + 8 * (int64_t)K;
        for (int a = 0; a < 8; ++a) add(g.node_unk[cn[a]]);
        const uint8_t fm = g.fmask[K];
        for (int lf = 0; lf < 6; ++lf)
            if (fm >> lf & 1) add(g.frac_unk[g.cell_frac[6 * (int64_t)K + lf]]);
    });
    if (i < g.nn)
        for (int32_t q = g.node_grp_ptr[row]; q < g.node_grp_ptr[row + 1]; ++q) {
            const int32_t G = g.node_grp[q];
            for (int32_t k = g.grp_nptr[G]; k < g.grp_nptr[G + 1]; ++k) add(g.grp_node[k]);
        }
}
}  // namespace

// the row in registers; len = -1 where it holds more than kRegCols columns.
// Dirichlet nodes (-1) and eliminated faces (>= nunk) are no columns.
__global__ __launch_bounds__(kPT) void pattern_rows_kernel(PatArgs g, const int64_t *__restrict__ off,
                                                           int32_t *__restrict__ raw, int32_t *__restrict__ len) {
    const int64_t i = (int64_t)blockIdx.x * kPT + threadIdx.x;
    if (i >= (int64_t)g.nn + g.nf) return;
    const int32_t row = pattern_row(g, i);
    if (row < 0) return;
    RegList L;
    pattern_candidates(g, i, row, [&](int32_t c) {
        if (c >= 0 && c < g.nunk) L.add(c);
    });
    if (L.m > kRegCols) {
        len[row] = -1;
        return;
    }
    int32_t *out = raw + off[row];
#pragma unroll
    for (int k = 0; k < kRegCols; ++k)
        if (k < L.m) out[k] = L.a[k];
    len[row] = L.m;
}

// the rows the register kernel left (len -1), with the list in the scratch
// array: each candidate moves the larger entries up by one unless present
__global__ __launch_bounds__(kPT) void pattern_long_rows_kernel(PatArgs g, const int64_t *__restrict__ off,
                                                                int32_t *raw, int32_t *__restrict__ len) {
    const int64_t i = (int64_t)blockIdx.x * kPT + threadIdx.x;
    if (i >= (int64_t)g.nn + g.nf) return;
    const int32_t row = pattern_row(g, i);
    if (row < 0 || len[row] >= 0) return;
    int32_t *out = raw + off[row];
    int32_t m = 0;
    pattern_candidates(g, i, row, [&](int32_t c) {
        if (c < 0 || c >= g.nunk) return;
        int32_t j = m;
        while (j > 0 && out[j - 1] > c) --j;
        if (j > 0 && out[j - 1] == c) return;
        for (int32_t k = m; k > j; --k) out[k] = out[k - 1];
        out[j] = c;
        ++m;
    });
    len[row] = m;
}

// new row r is natural row sys_old[r], its length row_ptr[r + 1] - row_ptr[r];
// its columns mapped by sys_new and sorted (in registers up to kRegCols
// columns, else by insertion in place in the output row)
__global__ __launch_bounds__(kPT) void pattern_sort_kernel(int32_t n, const int32_t *__restrict__ row_ptr,
                                                           const int32_t *__restrict__ sys_old,
                                                           const int64_t *__restrict__ off,
                                                           const int32_t *__restrict__ raw,
                                                           const int32_t *__restrict__ sys_new, int32_t *col) {
    const int32_t r = blockIdx.x * kPT + threadIdx.x;
    if (r >= n) return;
    const int32_t *src = raw + off[sys_old[r]];
    const int32_t len = row_ptr[r + 1] - row_ptr[r];
    int32_t *dst = col + row_ptr[r];
    if (len <= kRegCols) {
        RegList L;
        for (int32_t k = 0; k < len; ++k) L.insert(sys_new[src[k]]);
#pragma unroll
        for (int k = 0; k < kRegCols; ++k)
            if (k < len) dst[k] = L.a[k];
        return;
    }
    for (int32_t k = 0; k < len; ++k) {
        const int32_t v = sys_new[src[k]];
        int32_t j = k;
        for (; j > 0; --j) {
            const int32_t u = dst[j - 1];
            if (u <= v) break;
            dst[j] = u;
        }
        dst[j] = v;
    }
}

// exclusive scan of n ints into n + 1 int64 offsets: sums of blocks of
// kScanPer items, one block scans those, each block then scans its own items
constexpr int kScanPer = 4 * kPT;
__global__ __launch_bounds__(kPT) void scan64_sums_kernel(int32_t n, const int32_t *__restrict__ in,
                                                          int64_t *__restrict__ sums) {
    __shared__ int64_t w[kPT / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanPer;
    int64_t t = 0;
    for (int k = 0; k < 4; ++k) {
        const int64_t i = base + (int64_t)k * kPT + threadIdx.x;
        if (i < n) t += in[i];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_down(t, o, 64);
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t b = 0;
        for (int k = 0; k < kPT / 64; ++k) b += w[k];
        sums[blockIdx.x] = b;
    }
}
__global__ __launch_bounds__(1024) void scan64_top_kernel(int32_t nb, int64_t *sums) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int32_t chunk = (nb + 1023) / 1024;
    const int32_t lo = min(nb, t * chunk), hi = min(nb, lo + chunk);
    int64_t acc = 0;
    for (int32_t k = lo; k < hi; ++k) acc += sums[k];
    part[t] = acc;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int k = 0; k < 1024; ++k) {
            const int64_t v = part[k];
            part[k] = run;
            run += v;
        }
        sums[nb] = run;
    }
    __syncthreads();
    int64_t run = part[t];
    for (int32_t k = lo; k < hi; ++k) {
        const int64_t v = sums[k];
        sums[k] = run;
        run += v;
    }
}
__global__ __launch_bounds__(kPT) void scan64_apply_kernel(int32_t n, int32_t nb, const int32_t *__restrict__ in,
                                                           const int64_t *__restrict__ sums,
                                                           int64_t *__restrict__ out) {
    __shared__ int64_t w[kPT / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanPer + (int64_t)threadIdx.x * 4;
    int64_t v[4], t = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        t += v[k];
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t incl = t;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) w[wv] = incl;
    __syncthreads();
    int64_t run = sums[blockIdx.x] + incl - t;
    for (int k = 0; k < wv; ++k) run += w[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[nb];
}

// node -> (cell, slot) lists: counts, their scan, the entries K * 8 + a put
// in place by atomic cursors, then every list sorted (ascending, as a pass
// over the cells in order would give)
__global__ __launch_bounds__(kPT) void zero_int_kernel(int32_t n, int32_t *__restrict__ v) {
    const int32_t i = blockIdx.x * kPT + threadIdx.x;
    if (i < n) v[i] = 0;
}
__global__ __launch_bounds__(kPT) void node_cell_count_kernel(int64_t n8, const int32_t *__restrict__ hex8,
                                                              int32_t *cnt) {
    const int64_t i = (int64_t)blockIdx.x * kPT + threadIdx.x;
    if (i < n8) atomicAdd(&cnt[hex8[i]], 1);
}
__global__ __launch_bounds__(kPT) void node_cell_fill_kernel(int64_t n8, const int32_t *__restrict__ hex8,
                                                             const int32_t *__restrict__ ptr, int32_t *cur,
                                                             int32_t *__restrict__ cells) {
    const int64_t i = (int64_t)blockIdx.x * kPT + threadIdx.x;
    if (i >= n8) return;
    const int32_t s = hex8[i];
    cells[ptr[s] + atomicAdd(&cur[s], 1)] = (int32_t)i;
}
__global__ __launch_bounds__(kPT) void node_cell_sort_kernel(int32_t nn, const int32_t *__restrict__ ptr,
                                                             int32_t *cells) {
    const int32_t s = blockIdx.x * kPT + threadIdx.x;
    if (s >= nn) return;
    int32_t *b = cells + ptr[s];
    const int32_t len = ptr[s + 1] - ptr[s];
    for (int32_t k = 1; k < len; ++k) {
        const int32_t v = b[k];
        int32_t j = k;
        for (; j > 0; --j) {
            const int32_t u = b[j - 1];
            if (u <= v) break;
            b[j] = u;
        }
        b[j] = v;
    }
}

void launch_node_cell(hipStream_t s, int32_t nn, int64_t nc, const int32_t *hex8, int32_t *ptr, int32_t *cells,
                      int32_t *work) {
    const int64_t n8 = 8 * nc;
    const unsigned gn = (unsigned)((nn + kPT - 1) / kPT), g8 = (unsigned)((n8 + kPT - 1) / kPT);
    int32_t *cnt = work, *tmp = work + nn;
    hipLaunchKernelGGL(zero_int_kernel, dim3(gn), dim3(kPT), 0, s, nn, cnt);
    hipLaunchKernelGGL(node_cell_count_kernel, dim3(g8), dim3(kPT), 0, s, n8, hex8, cnt);
    VAG_HIP(hipGetLastError());
    amg_launch_scan(s, nn, cnt, ptr, tmp);
    hipLaunchKernelGGL(zero_int_kernel, dim3(gn), dim3(kPT), 0, s, nn, cnt);
    hipLaunchKernelGGL(node_cell_fill_kernel, dim3(g8), dim3(kPT), 0, s, n8, hex8, ptr, cnt, cells);
    hipLaunchKernelGGL(node_cell_sort_kernel, dim3(gn), dim3(kPT), 0, s, nn, ptr, cells);
    VAG_HIP(hipGetLastError());
}

void launch_pattern_bound(hipStream_t s, const PatArgs &g, int32_t *ub) {
    const int64_t n = (int64_t)g.nn + g.nf;
    if (n <= 0) return;
    hipLaunchKernelGGL(pattern_bound_kernel, dim3((unsigned)((n + kPT - 1) / kPT)), dim3(kPT), 0, s, g, ub);
    VAG_HIP(hipGetLastError());
}

void launch_pattern_rows(hipStream_t s, const PatArgs &g, const int64_t *off, int32_t *raw, int32_t *len) {
    const int64_t n = (int64_t)g.nn + g.nf;
    if (n <= 0) return;
    const dim3 grid((unsigned)((n + kPT - 1) / kPT));
    hipLaunchKernelGGL(pattern_rows_kernel, grid, dim3(kPT), 0, s, g, off, raw, len);
    hipLaunchKernelGGL(pattern_long_rows_kernel, grid, dim3(kPT), 0, s, g, off, raw, len);
    VAG_HIP(hipGetLastError());
}

void launch_scan64(hipStream_t s, int32_t n, const int32_t *in, int64_t *out, int64_t *sums) {
    if (n <= 0) return;
    const int32_t nb = (int32_t)(((int64_t)n + kScanPer - 1) / kScanPer);
    hipLaunchKernelGGL(scan64_sums_kernel, dim3(nb), dim3(kPT), 0, s, n, in, sums);
    hipLaunchKernelGGL(scan64_top_kernel, dim3(1), dim3(1024), 0, s, nb, sums);
    hipLaunchKernelGGL(scan64_apply_kernel, dim3(nb), dim3(kPT), 0, s, n, nb, in, sums, out);
    VAG_HIP(hipGetLastError());
}

void launch_pattern_sort(hipStream_t s, int32_t n, const int32_t *row_ptr, const int32_t *sys_old,
                         const int64_t *off, const int32_t *raw, const int32_t *sys_new, int32_t *col) {
    if (n <= 0) return;
    hipLaunchKernelGGL(pattern_sort_kernel, dim3((unsigned)((n + kPT - 1) / kPT)), dim3(kPT), 0, s, n, row_ptr,
                       sys_old, off, raw, sys_new, col);
    VAG_HIP(hipGetLastError());
}

}  // namespace vag
