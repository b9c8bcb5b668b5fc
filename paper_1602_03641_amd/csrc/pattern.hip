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
//  2. the candidates inserted one by one into the row's sorted list in the
//     scratch array, duplicates skipped: the row and its exact length;
//  3. after the host has renumbered the rows from their lengths, each row
//     mapped to the system numbering and sorted into the CSR layout.
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

__global__ __launch_bounds__(kPT) void pattern_rows_kernel(PatArgs g, const int64_t *__restrict__ off,
                                                           int32_t *raw, int32_t *__restrict__ len) {
    const int64_t i = (int64_t)blockIdx.x * kPT + threadIdx.x;
    if (i >= (int64_t)g.nn + g.nf) return;
    const int32_t row = pattern_row(g, i);
    if (row < 0) return;
    int32_t *out = raw + off[row];
    int32_t m = 0;
    // insert c into the sorted list out[0, m) unless it is there already;
    // Dirichlet nodes (-1) and eliminated faces (>= nunk) are no columns
    auto add = [&](int32_t c) {
        if (c < 0 || c >= g.nunk) return;
        int32_t j = m;
        while (j > 0 && out[j - 1] > c) --j;
        if (j > 0 && out[j - 1] == c) return;
        for (int32_t k = m; k > j; --k) out[k] = out[k - 1];
        out[j] = c;
        ++m;
    };
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
    len[row] = m;
}

// new row r is natural row sys_old[r], its length row_ptr[r + 1] - row_ptr[r];
// the natural row is sorted in the natural numbering, and the renumbering
// keeps rows in place up to a window, so few insertions move far
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

void launch_pattern_bound(hipStream_t s, const PatArgs &g, int32_t *ub) {
    const int64_t n = (int64_t)g.nn + g.nf;
    if (n <= 0) return;
    hipLaunchKernelGGL(pattern_bound_kernel, dim3((unsigned)((n + kPT - 1) / kPT)), dim3(kPT), 0, s, g, ub);
    VAG_HIP(hipGetLastError());
}

void launch_pattern_rows(hipStream_t s, const PatArgs &g, const int64_t *off, int32_t *raw, int32_t *len) {
    const int64_t n = (int64_t)g.nn + g.nf;
    if (n <= 0) return;
    hipLaunchKernelGGL(pattern_rows_kernel, dim3((unsigned)((n + kPT - 1) / kPT)), dim3(kPT), 0, s, g, off, raw,
                       len);
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
