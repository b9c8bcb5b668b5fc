// Assembly of the cell-eliminated VAG system (§3.1 and §4.2 of the paper).
//
// vag_local_kernel   one thread per cell: the local VAG matrix a_{K,nu}^{nu'}
//                    (eq VAGFluxMatrix) from the 24 sub-tetrahedra, its row sums
//                    r_nu and A_KK = sum r_nu.
// vag_frac_kernel    one thread per fracture face: the 5x5 P1 stiffness of
//                    d_f Lambda_f / mu on the face's 4 triangles (eq VAGFluxFracture).
// asm_node_rows_kernel one thread per free-node row: the row gathers, from
//                    every cell around its node, row s of the cell Schur block
//                    M_K = a - r r^T / A_KK (eq eqschur) and the couplings to
//                    the fracture faces of those cells; Dirichlet columns go to
//                    b.  Each row is written by one thread only, so no atomics
//                    are needed and the summation order is fixed.
// asm_face_rows_kernel / asm_elim_rows_kernel  the same gather for the rows
//                    of kept fracture faces and for the dense blocks of the
//                    eliminated fracture-face groups.
//
// Storage of the local data (structure of arrays, coalesced by cell index):
//   aK[36][nc]  packed upper triangle of the node block a_{s,s'}
//   rK[8][nc]   row sums r_s (including couplings to fracture faces)
//   AKK[nc], vol[nc]
//   fside[nf*2][6] per (fracture face, side): a_{sigma,sigma}, a_{sigma,s} for
//               the face's 4 nodes in the cell's local face order, r_sigma
//   A5[nf][25]  fracture 5x5 over (sigma, input nodes 0..3)
#include <climits>

#include "vag_internal.h"

namespace vag {

namespace {

struct V3 {
    double x, y, z;
};
__device__ inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline V3 cross(V3 a, V3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
// L = [xx yy zz xy xz yz]
__device__ inline V3 tmul(const double *L, V3 v) {
    return {L[0] * v.x + L[3] * v.y + L[4] * v.z, L[3] * v.x + L[1] * v.y + L[5] * v.z,
            L[4] * v.x + L[5] * v.y + L[2] * v.z};
}

}  // namespace

__global__ __launch_bounds__(128) void vag_local_kernel(
    int32_t nc, const double *__restrict__ xyz, const int32_t *__restrict__ hex8,
    const double *__restrict__ perm, double inv_mu, const uint8_t *__restrict__ fmask,
    const int32_t *__restrict__ cell_frac, const int32_t *__restrict__ frac_cell, double *__restrict__ aK,
    double *__restrict__ rK, double *__restrict__ AKKo, double *__restrict__ volo,
    double *__restrict__ fside, int *__restrict__ bad_cell) {
    const int32_t K = blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= nc) return;
    V3 X[8];
    V3 xK = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const int32_t s = hex8[8 * (int64_t)K + a];
        X[a] = {xyz[3 * (int64_t)s], xyz[3 * (int64_t)s + 1], xyz[3 * (int64_t)s + 2]};
        xK.x += 0.125 * X[a].x;
        xK.y += 0.125 * X[a].y;
        xK.z += 0.125 * X[a].z;
    }
    double L[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) L[i] = perm[6 * (int64_t)K + i] * inv_mu;
    const unsigned mask = fmask[K];

    double acc[36];
#pragma unroll
    for (int i = 0; i < 36; ++i) acc[i] = 0.0;
    double rx[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) rx[i] = 0.0;
    double akk = 0.0, vol = 0.0;
    bool bad = false;

#pragma unroll
    for (int f = 0; f < 6; ++f) {
        V3 xs = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            xs.x += 0.25 * X[hexf(f, i)].x;
            xs.y += 0.25 * X[hexf(f, i)].y;
            xs.z += 0.25 * X[hexf(f, i)].z;
        }
        // 5x5 stiffness over (face centre, face nodes 0..3) from the 4 sub-tets
        double S[15];
#pragma unroll
        for (int i = 0; i < 15; ++i) S[i] = 0.0;
        const V3 a = sub(xs, xK);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i1 = e, i2 = (e + 1) & 3;
            const V3 b = sub(X[hexf(f, i1)], xK);
            const V3 c = sub(X[hexf(f, i2)], xK);
            // J = [a b c]; rows of J^{-1} are (b x c, c x a, a x b) / det:
            // the gradients of the barycentric coordinates of x_sigma, s_1, s_2
            const V3 uc = cross(b, c), u1 = cross(c, a), u2 = cross(a, b);
            const double det = dot(a, uc);
            bad |= !(det > 0.0);
            vol += det * (1.0 / 6.0);
            // |T| g_i . L g_j = (u_i . L u_j) / (6 det)
            const double w = 1.0 / (6.0 * det);
            const V3 Lc = tmul(L, uc), L1 = tmul(L, u1), L2 = tmul(L, u2);
            S[sym5(0, 0)] += w * dot(uc, Lc);
            S[sym5(0, 1 + i1)] += w * dot(uc, L1);
            S[sym5(0, 1 + i2)] += w * dot(uc, L2);
            S[sym5(1 + i1, 1 + i1)] += w * dot(u1, L1);
            S[sym5(1 + i1, 1 + i2)] += w * dot(u1, L2);
            S[sym5(1 + i2, 1 + i2)] += w * dot(u2, L2);
        }
        if (!((mask >> f) & 1u)) {
            // non-fracture face: the centre value is the mean of the 4 nodes
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = i; j < 4; ++j)
                    acc[sym8(hexf(f, i), hexf(f, j))] +=
                        S[sym5(1 + i, 1 + j)] + 0.25 * (S[sym5(0, 1 + i)] + S[sym5(0, 1 + j)]) +
                        0.0625 * S[sym5(0, 0)];
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = i; j < 4; ++j) acc[sym8(hexf(f, i), hexf(f, j))] += S[sym5(1 + i, 1 + j)];
            const int32_t sg = cell_frac[6 * (int64_t)K + f];
            const int side = (frac_cell[2 * (int64_t)sg] == K) ? 0 : 1;
            double *o = fside + (2 * (int64_t)sg + side) * 6;
            double rs = S[sym5(0, 0)];
            o[0] = S[sym5(0, 0)];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                o[1 + i] = S[sym5(0, 1 + i)];
                rs += S[sym5(0, 1 + i)];
                rx[hexf(f, i)] += S[sym5(0, 1 + i)];
            }
            o[5] = rs;
            akk += rs;
        }
    }
    // node-block diagonal entries appear once per pair (i <= j) per face; the
    // off-diagonal (i < j) entries were added once, matching a symmetric store.
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        double r = rx[s];
#pragma unroll
        for (int t = 0; t < 8; ++t) r += acc[sym8(s, t)];
        rK[(int64_t)s * nc + K] = r;
        akk += r;
    }
#pragma unroll
    for (int i = 0; i < 36; ++i) aK[(int64_t)i * nc + K] = acc[i];
    AKKo[K] = akk;
    volo[K] = vol;
    if (bad) atomicMin(bad_cell, K);
}

__global__ __launch_bounds__(256) void vag_frac_kernel(int32_t nf, const double *__restrict__ xyz,
                                                       const int32_t *__restrict__ frac_nodes,
                                                       const double *__restrict__ width,
                                                       const double *__restrict__ perm, double inv_mu,
                                                       double *__restrict__ A5, double *__restrict__ area) {
    const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    V3 X[4];
    V3 xs = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int32_t s = frac_nodes[4 * (int64_t)f + i];
        X[i] = {xyz[3 * (int64_t)s], xyz[3 * (int64_t)s + 1], xyz[3 * (int64_t)s + 2]};
        xs.x += 0.25 * X[i].x;
        xs.y += 0.25 * X[i].y;
        xs.z += 0.25 * X[i].z;
    }
    const double kappa = width[f] * perm[f] * inv_mu;
    double M[25];
#pragma unroll
    for (int i = 0; i < 25; ++i) M[i] = 0.0;
    double A = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        // triangle (x_sigma, s_e, s_e+1); edge vectors opposite each vertex,
        // traversed cyclically: K_ij = kappa (e_i . e_j) / (4 |T|)
        const int id[3] = {0, 1 + e, 1 + ((e + 1) & 3)};
        const V3 p0 = xs, p1 = X[e], p2 = X[(e + 1) & 3];
        const V3 e0 = sub(p2, p1), e1 = sub(p0, p2), e2 = sub(p1, p0);
        const V3 n = cross(e2, sub(p2, p0));
        const double twoA = sqrt(dot(n, n));
        A += 0.5 * twoA;
        const double w = kappa / (2.0 * twoA);
        const V3 E[3] = {e0, e1, e2};
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) M[id[i] * 5 + id[j]] += w * dot(E[i], E[j]);
    }
#pragma unroll
    for (int i = 0; i < 25; ++i) A5[25 * (int64_t)f + i] = M[i];
    area[f] = A;
}

// ---------------------------------------------------------------------------
// Assembly of the cell-eliminated system, row by row: the thread of a row
// gathers the entries of M_K = a - r r^T / A_KK from the cells of its node
// (or face) and the fracture blocks of its faces, in a fixed order, and adds
// them at the positions found by binary search in the row's sorted columns.
// Each row is written by one thread only: no atomics, no colouring, and the
// summation order does not depend on timing.
// ---------------------------------------------------------------------------

// vertex index of cell node a on local face f, or -1
__device__ inline int face_vertex(int f, int a) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (hexf(f, i) == a) return i;
    return -1;
}

// position of column c in row r (real entries, sorted), -1 if absent
__device__ inline int64_t sell_find(const AsmArgs &g, int32_t r, int32_t c) {
    const int64_t base = g.sell_ptr[r >> 6] + (r & 63);
    int lo = 0, hi = g.row_len[r];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (g.sell_col[base + 64 * (int64_t)mid] < c) lo = mid + 1; else hi = mid;
    }
    if (lo < g.row_len[r] && g.sell_col[base + 64 * (int64_t)lo] == c) return base + 64 * (int64_t)lo;
    return -1;
}

// Adds v to (r, column unknown c) of the system; c < 0: Dirichlet column of
// node `node`, to the right-hand side; c >= nsys: an eliminated face, held
// by its group block instead (nothing to do).
__device__ inline void add_sys(const AsmArgs &g, int32_t r, int32_t c, int32_t node, double v, double &rhs) {
    if (c < 0) {
        rhs -= v * g.p_bar[node];
    } else if (c < g.nsys) {
        const int64_t q = sell_find(g, r, c);
        if (q >= 0) g.A[q] += v; else atomicMin(g.bad, INT_MIN);
    }
}

// The coefficients the scheme takes (§2: Lambda_m symmetric positive
// definite; d_f and Lambda_f positive): a cell's packed tensor passes when
// its leading principal minors are positive and every entry is finite, a
// fracture face when its width and permeability are positive and finite.
// bad[0] receives the least failing cell, bad[1] the least failing face.
__global__ __launch_bounds__(256) void check_coef_kernel(int32_t nc, const double *__restrict__ perm, int32_t nf,
                                                         const double *__restrict__ fwidth,
                                                         const double *__restrict__ fperm, int *bad) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < nc) {
        const double *L = perm + 6 * i;
        const double xx = L[0], yy = L[1], zz = L[2], xy = L[3], xz = L[4], yz = L[5];
        const double m2 = xx * yy - xy * xy;
        const double m3 = xx * (yy * zz - yz * yz) - xy * (xy * zz - yz * xz) + xz * (xy * yz - yy * xz);
        bool fin = true;
        for (int k = 0; k < 6; ++k) fin &= isfinite(L[k]);
        if (!(fin && xx > 0.0 && m2 > 0.0 && m3 > 0.0)) atomicMin(&bad[0], (int)i);
    } else if (i < (int64_t)nc + nf) {
        const int32_t f = (int32_t)(i - nc);
        const double w = fwidth[f], k = fperm[f];
        if (!(isfinite(w) && isfinite(k) && w > 0.0 && k > 0.0)) atomicMin(&bad[1], f);
    }
}

// Slots of the M_K columns in the node rows, found once per handle (the
// per-solve assembly then adds at known slots).  A row of up to kPosRegs
// columns is read into registers once and a column's slot is the count of
// smaller columns there; longer rows take a binary search in the stored row.
constexpr int kPosRegs = 32;
__global__ __launch_bounds__(128) void node_pos_kernel(AsmArgs g, uint16_t *__restrict__ node_pos) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= g.nfree) return;
    const int32_t s = g.unk_node[r];
    const int64_t base = g.sell_ptr[r >> 6] + (r & 63);
    const int32_t len = g.row_len[r];
    const bool regs = len <= kPosRegs;
    int32_t a[kPosRegs];
#pragma unroll
    for (int k = 0; k < kPosRegs; ++k) a[k] = regs && k < len ? g.sell_col[base + 64 * (int64_t)k] : INT32_MAX;
    for (int32_t q = g.node_cell_ptr[s]; q < g.node_cell_ptr[s + 1]; ++q) {
        const int32_t K = g.node_cell[q] >> 3;
        // the cell's 8 unknowns first (loads in flight together), its 8 slots
        // stored at the end as one 16-byte write
        int32_t uc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) uc[c] = g.node_unk[g.hex8[8 * (int64_t)K + c]];
        uint32_t pw[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int32_t u = uc[c];
            uint16_t k = 0xffff;
            if (u >= 0) {
                int64_t slot = -1;
                if (regs) {
                    int32_t below = 0;
                    bool found = false;
#pragma unroll
                    for (int j = 0; j < kPosRegs; ++j) {
                        below += a[j] < u;
                        found |= a[j] == u;
                    }
                    if (found) slot = below;
                } else {
                    const int64_t p = sell_find(g, r, u);
                    if (p >= 0) slot = (p - base) / 64;
                }
                if (slot < 0 || slot >= 0xffff) atomicMin(g.bad, INT_MIN);
                else k = (uint16_t)slot;
            }
            pw[c >> 1] |= (uint32_t)k << (16 * (c & 1));
        }
        *reinterpret_cast<uint4 *>(node_pos + 8 * (int64_t)q) = make_uint4(pw[0], pw[1], pw[2], pw[3]);
    }
}

// One thread per node row.  The row's first kAccSlots slots accumulate in
// LDS (the thread's own column of acc) and are stored once at the end: a
// read-modify-write of the row in global memory would make every addition
// wait for the previous one, since the compiler cannot tell the slots apart.
// Slots beyond kAccSlots (rows next to eliminated fracture groups) are added
// in global memory, which the caller has zeroed.
constexpr int kAccSlots = 32;
__global__ __launch_bounds__(128) void asm_node_rows_kernel(AsmArgs g) {
    __shared__ double acc[kAccSlots][128];
    const int tid = threadIdx.x;
    const int32_t r = blockIdx.x * blockDim.x + tid;
    if (r >= g.nfree) return;
    const int32_t s = g.unk_node[r];
    const int64_t base = g.sell_ptr[r >> 6] + (r & 63);
    const int w = min(g.row_len[r], kAccSlots);
    for (int k = 0; k < w; ++k) acc[k][tid] = 0.0;
    double rhs = 0.0;
    auto put = [&](int k, double v) {
        if (k < kAccSlots) acc[k][tid] += v;
        else g.A[base + 64 * (int64_t)k] += v;
    };
    // column unknown c (node `node` or a face; c < 0: Dirichlet node; c >= nsys:
    // an eliminated face, held by its group block)
    auto put_col = [&](int32_t c, int32_t node, double v) {
        if (c < 0) {
            rhs -= v * g.p_bar[node];
        } else if (c < g.nsys) {
            const int64_t p = sell_find(g, r, c);
            if (p >= 0) put((int)((p - base) >> 6), v);
            else atomicMin(g.bad, INT_MIN);
        }
    };
    // cells of the node: row a of M_K
    for (int32_t q = g.node_cell_ptr[s]; q < g.node_cell_ptr[s + 1]; ++q) {
        const int32_t K = g.node_cell[q] >> 3;
        const int a = g.node_cell[q] & 7;
        const double inv = 1.0 / g.AKK[K];
        const double ra = g.rK[(int64_t)a * g.nc + K];
        // the cell's loads first, all in flight together: an addition to a
        // slot beyond kAccSlots stores to the row in global memory, which the
        // compiler would not move a later load past
        double v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = g.aK[(int64_t)sym8(a, c) * g.nc + K] - ra * g.rK[(int64_t)c * g.nc + K] * inv;
        const uint4 pos = *reinterpret_cast<const uint4 *>(g.node_pos + 8 * (int64_t)q);  // 8 slots, 16 bytes
        const uint32_t pw[4] = {pos.x, pos.y, pos.z, pos.w};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint16_t k = (uint16_t)(pw[c >> 1] >> (16 * (c & 1)));
            if (k != 0xffff) put(k, v[c]);
            else rhs -= v[c] * g.p_bar[g.hex8[8 * (int64_t)K + c]];  // Dirichlet column
        }
        const unsigned mask = g.fmask[K];
        for (int f = 0; f < 6; ++f) {
            if (!((mask >> f) & 1u)) continue;
            const int32_t sig = g.cell_frac[6 * (int64_t)K + f];
            const int sd = g.frac_cell[2 * (int64_t)sig] == K ? 0 : 1;
            const double *o = g.fside + (2 * (int64_t)sig + sd) * 6;
            const int i = face_vertex(f, a);
            const double v = (i >= 0 ? o[1 + i] : 0.0) - ra * o[5] * inv;
            put_col(g.frac_unk[sig], -1, v);
        }
    }
    // fracture blocks of the faces the node is a vertex of: row 1+i of the 5x5 block
    for (int32_t q = g.node_frac_ptr[s]; q < g.node_frac_ptr[s + 1]; ++q) {
        const int32_t sig = g.node_frac[q] >> 2;
        const int i = g.node_frac[q] & 3;
        const double *M = g.A5 + 25 * (int64_t)sig + 5 * (1 + i);
        put_col(g.frac_unk[sig], -1, M[0]);
        for (int k = 0; k < 4; ++k) {
            const int32_t node = g.frac_nodes[4 * (int64_t)sig + k];
            put_col(g.node_unk[node], node, M[1 + k]);
        }
    }
    for (int k = 0; k < w; ++k) g.A[base + 64 * (int64_t)k] = acc[k][tid];
    g.b[r] += rhs;
}

// Row of fracture face sig (kept: system row r; eliminated: row of its group
// block).  blk = null for a kept face.
__device__ inline void asm_face_row(const AsmArgs &g, int32_t sig, int32_t r, double *blk, int32_t G, double &rhs) {
    int gsize = 0, W = 0;
    const int32_t *B = nullptr;
    int m = 0;
    if (blk) {
        gsize = g.grp_ptr[G + 1] - g.grp_ptr[G];
        m = g.grp_nptr[G + 1] - g.grp_nptr[G];
        W = gsize + m;
        B = g.grp_node + g.grp_nptr[G];
    }
    // adds v to column unknown c (node `node` or face sig2)
    auto put = [&](int32_t c, int32_t node, int32_t sig2, double v) {
        if (!blk) {
            add_sys(g, r, c, node, v, rhs);
        } else if (c < 0) {
            rhs -= v * g.p_bar[node];
        } else if (c >= g.nsys) {
            blk[g.face_loc[sig2]] += v;
        } else {
            int lo = 0, hi = m;  // free node: its index in the group's sorted node list
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (B[mid] < c) lo = mid + 1; else hi = mid;
            }
            if (lo < m && B[lo] == c) blk[gsize + lo] += v; else atomicMin(g.bad, INT_MIN);
        }
    };
    (void)W;
    for (int side = 0; side < 2; ++side) {
        const int32_t K = g.frac_cell[2 * (int64_t)sig + side];
        if (K < 0) continue;
        int f = 0;
        while (f < 6 && g.cell_frac[6 * (int64_t)K + f] != sig) ++f;
        const unsigned mask = g.fmask[K];
        const double inv = 1.0 / g.AKK[K];
        const double *o = g.fside + (2 * (int64_t)sig + side) * 6;
        const double rs = o[5];
        for (int c = 0; c < 8; ++c) {
            const int32_t node = g.hex8[8 * (int64_t)K + c];
            const int i = face_vertex(f, c);
            const double v = (i >= 0 ? o[1 + i] : 0.0) - rs * g.rK[(int64_t)c * g.nc + K] * inv;
            put(g.node_unk[node], node, -1, v);
        }
        for (int f2 = 0; f2 < 6; ++f2) {
            if (!((mask >> f2) & 1u)) continue;
            const int32_t sig2 = g.cell_frac[6 * (int64_t)K + f2];
            const int sd2 = g.frac_cell[2 * (int64_t)sig2] == K ? 0 : 1;
            const double v = (f2 == f ? o[0] : 0.0) - rs * g.fside[(2 * (int64_t)sig2 + sd2) * 6 + 5] * inv;
            put(g.frac_unk[sig2], -1, sig2, v);
        }
    }
    // fracture block: row 0 of the 5x5 block
    const double *M = g.A5 + 25 * (int64_t)sig;
    put(g.frac_unk[sig], -1, sig, M[0]);
    for (int k = 0; k < 4; ++k) {
        const int32_t node = g.frac_nodes[4 * (int64_t)sig + k];
        put(g.node_unk[node], node, -1, M[1 + k]);
    }
}

__global__ __launch_bounds__(128) void asm_face_rows_kernel(AsmArgs g, int32_t nkept) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nkept) return;
    const int32_t r = g.nfree + t;
    double rhs = 0.0;
    asm_face_row(g, g.unk_face[t], r, nullptr, -1, rhs);
    g.b[r] += rhs;
}

// rows of eliminated faces into the dense group blocks [A_GG | A_GB], b_G
__global__ __launch_bounds__(128) void asm_elim_rows_kernel(AsmArgs g, int32_t nelim) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nelim) return;
    const int32_t sig = g.grp_face[t];
    const int32_t G = g.face_grp[sig];
    const int gsize = g.grp_ptr[G + 1] - g.grp_ptr[G];
    const int W = gsize + g.grp_nptr[G + 1] - g.grp_nptr[G];
    double *blk = g.Gb + g.grp_off[G] + (int64_t)g.face_loc[sig] * W;
    double rhs = 0.0;
    asm_face_row(g, sig, -1, blk, G, rhs);
    g.b[g.frac_unk[sig]] += rhs;
}

// Fills the sliced-ELL columns from the CSR pattern (one thread per slice
// lane), the real row lengths and the diagonal positions.
__global__ __launch_bounds__(256) void sell_fill_kernel(int32_t n, int64_t nslice, const int32_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col,
                                                        const int64_t *__restrict__ sell_ptr,
                                                        int32_t *__restrict__ sell_col, int32_t *__restrict__ row_len,
                                                        int32_t *__restrict__ diag_pos) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nslice * 64) return;
    const int64_t sl = t >> 6;
    const int32_t r = (int32_t)t;
    const int32_t w = (int32_t)((sell_ptr[sl + 1] - sell_ptr[sl]) / 64);
    const int32_t len = r < n ? row_ptr[r + 1] - row_ptr[r] : 0;
    const int32_t pad = r < n ? r : 0;  // padding: own row, value 0
    int64_t pos = sell_ptr[sl] + (t & 63);
    for (int32_t k = 0; k < w; ++k, pos += 64) {
        const int32_t c = k < len ? col[row_ptr[r] + k] : pad;
        sell_col[pos] = c;
        if (k < len && c == r) diag_pos[r] = (int32_t)pos;
    }
    if (r < n) row_len[r] = len;
}

// 16-bit column offsets (one wavefront per slice).  Level k of a slice (entry
// k of each of its 64 rows, one group of 64 stored entries) gets its own base,
// the least column among the level's real entries: in a slice of rows of one
// pattern a level holds the neighbours in one direction, whose columns lie
// close together even where the slice as a whole spans more than 65536
// columns (the z-stride of a 192^3 node numbering is 37249).  When every
// level's real columns lie within 65536 of its base, col16 = col - base and
// cbase[group] = base; otherwise all of the slice's groups get cbase = -1 and
// the row loops read the 32-bit columns.  Padding entries (past a row's
// length, value 0) and rows past n take offset 0: the level's base, a valid
// column.
__global__ __launch_bounds__(64) void sell_pack_kernel(int32_t n, const int64_t *__restrict__ ptr,
                                                       const int32_t *__restrict__ col,
                                                       const int32_t *__restrict__ row_len,
                                                       uint16_t *__restrict__ col16, int32_t *__restrict__ cbase) {
    const int64_t sl = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t r = sl * 64 + lane;
    const int len = r < n ? row_len[r] : 0;
    const int64_t b0 = ptr[sl], width = (ptr[sl + 1] - b0) / 64;
    auto level = [&](int64_t k, int32_t &lo, int32_t &hi) {
        const bool real = k < len;
        const int32_t c = real ? col[b0 + 64 * k + lane] : 0;
        lo = real ? c : INT32_MAX;
        hi = real ? c : -1;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lo = min(lo, __shfl_xor(lo, o, 64));
            hi = max(hi, __shfl_xor(hi, o, 64));
        }
        return c;
    };
    bool compact = true;
    for (int64_t k = 0; k < width; ++k) {
        int32_t lo, hi;
        level(k, lo, hi);
        compact = compact && hi >= 0 && (int64_t)hi - lo <= 65535;
    }
    for (int64_t k = 0; k < width; ++k) {
        int32_t lo, hi;
        const int32_t c = level(k, lo, hi);
        if (compact) col16[b0 + 64 * k + lane] = k < len ? (uint16_t)(c - lo) : (uint16_t)0;
        if (lane == 0) cbase[(b0 >> 6) + k] = compact ? lo : -1;
    }
}

// system positions of the node pairs of each eliminated group
__global__ __launch_bounds__(64) void grp_pos_kernel(AsmArgs g, const int64_t *__restrict__ grp_poff,
                                                     int32_t *__restrict__ grp_pos) {
    const int32_t G = blockIdx.x;
    const int m = g.grp_nptr[G + 1] - g.grp_nptr[G];
    const int32_t *B = g.grp_node + g.grp_nptr[G];
    for (int e = threadIdx.x; e < m * m; e += 64) {
        const int64_t q = sell_find(g, B[e / m], B[e % m]);
        if (q < 0) atomicMin(g.bad, INT_MIN);
        grp_pos[grp_poff[G] + e] = q < 0 ? 0 : (int32_t)q;
    }
}

// Exact elimination of fracture-face groups of one colour, one wavefront per
// group.  The group block [A_GG | A_GB] (g x (g+m), row-major) and its
// right-hand side b_G are factored in LDS: A_GG = L L^T, Y = L^-1 A_GB,
// y = L^-1 b_G; then A_BB -= Y^T Y and b_B -= Y^T y are subtracted from the
// node rows.  L, Y and y are written back for the recovery of u_G.
// Groups of one colour share no free node, so the updates do not collide;
// every sum runs in a fixed order (deterministic).
__global__ __launch_bounds__(64) void vag_group_elim_kernel(
    int32_t first, int32_t ngroup, const int32_t *__restrict__ grp_ptr, const int32_t *__restrict__ grp_face,
    const int32_t *__restrict__ grp_nptr, const int32_t *__restrict__ grp_node, const int64_t *__restrict__ grp_off,
    const int64_t *__restrict__ grp_poff, const int32_t *__restrict__ grp_pos, const int32_t *__restrict__ frac_unk,
    double *__restrict__ Gb, double *__restrict__ A, double *__restrict__ b, int *__restrict__ bad) {
    extern __shared__ double lds[];
    const int32_t G = first + blockIdx.x;
    if (blockIdx.x >= ngroup) return;
    const int tid = threadIdx.x;
    const int g = grp_ptr[G + 1] - grp_ptr[G];
    const int m = grp_nptr[G + 1] - grp_nptr[G];
    const int W = g + m + 1;                       // LDS row: [A_GG | A_GB | b_G]
    double *blk = Gb + grp_off[G];
    const int32_t *faces = grp_face + grp_ptr[G];
    const int32_t *B = grp_node + grp_nptr[G];
    for (int e = tid; e < g * W; e += 64) {
        const int i = e / W, c = e - i * W;
        lds[e] = c < g + m ? blk[(int64_t)i * (g + m) + c] : b[frac_unk[faces[i]]];
    }
    __syncthreads();
    // right-looking Cholesky of A_GG
    for (int k = 0; k < g; ++k) {
        const double piv = lds[k * W + k];
        if (!(piv > 0.0)) {
            if (tid == 0) atomicMin(bad, -1 - G);
            return;  // uniform across the block: piv is read from LDS by every lane
        }
        const double d = sqrt(piv);
        __syncthreads();
        if (tid == 0) lds[k * W + k] = d;
        for (int i = k + 1 + tid; i < g; i += 64) lds[i * W + k] /= d;
        __syncthreads();
        const int rem = g - k - 1;
        for (int e = tid; e < rem * rem; e += 64) {
            const int i = k + 1 + e / rem, j = k + 1 + e % rem;
            if (j <= i) lds[i * W + j] -= lds[i * W + k] * lds[j * W + k];
        }
        __syncthreads();
    }
    // forward substitution, one column of [A_GB | b_G] per lane
    for (int c = g + tid; c < W; c += 64) {
        for (int i = 0; i < g; ++i) {
            double v = lds[i * W + c];
            for (int k = 0; k < i; ++k) v -= lds[i * W + k] * lds[k * W + c];
            lds[i * W + c] = v / lds[i * W + i];
        }
    }
    __syncthreads();
    for (int e = tid; e < g * W; e += 64) {
        const int i = e / W, c = e - i * W;
        if (c < g + m) blk[(int64_t)i * (g + m) + c] = lds[e];
        else b[frac_unk[faces[i]]] = lds[e];
    }
    // Schur complement on the node rows
    const int32_t *pos = grp_pos + grp_poff[G];
    for (int e = tid; e < m * m; e += 64) {
        const int p = e / m, q = e - p * m;
        double sum = 0.0;
        for (int k = 0; k < g; ++k) sum += lds[k * W + g + p] * lds[k * W + g + q];
        A[pos[e]] -= sum;
    }
    for (int p = tid; p < m; p += 64) {
        double sum = 0.0;
        for (int k = 0; k < g; ++k) sum += lds[k * W + g + p] * lds[k * W + g + m];
        b[B[p]] -= sum;
    }
}

// Recovery of the eliminated faces: u_G = L^-T (y - Y u_B), one wavefront per group.
__global__ __launch_bounds__(64) void vag_group_back_kernel(
    int32_t ngroup, const int32_t *__restrict__ grp_ptr, const int32_t *__restrict__ grp_face,
    const int32_t *__restrict__ grp_nptr, const int32_t *__restrict__ grp_node, const int64_t *__restrict__ grp_off,
    const int32_t *__restrict__ frac_unk, const double *__restrict__ Gb, const double *__restrict__ b,
    double *__restrict__ x) {
    __shared__ double z[kGroupMaxFaces];
    const int32_t G = blockIdx.x;
    if (G >= ngroup) return;
    const int tid = threadIdx.x;
    const int g = grp_ptr[G + 1] - grp_ptr[G];
    const int m = grp_nptr[G + 1] - grp_nptr[G];
    const double *blk = Gb + grp_off[G];
    const int32_t *faces = grp_face + grp_ptr[G];
    const int32_t *B = grp_node + grp_nptr[G];
    if (tid < g) {
        double v = b[frac_unk[faces[tid]]];
        for (int p = 0; p < m; ++p) v -= blk[(int64_t)tid * (g + m) + g + p] * x[B[p]];
        z[tid] = v;
    }
    __syncthreads();
    if (tid == 0) {
        for (int i = g - 1; i >= 0; --i) {
            double v = z[i];
            for (int k = i + 1; k < g; ++k) v -= blk[(int64_t)k * (g + m) + i] * z[k];
            z[i] = v / blk[(int64_t)i * (g + m) + i];
        }
    }
    __syncthreads();
    if (tid < g) x[frac_unk[faces[tid]]] = z[tid];
}

__global__ void vag_diag_inv_kernel(int32_t n, const int32_t *__restrict__ diag_pos,
                                    const double *__restrict__ A, double *__restrict__ dinv) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dinv[i] = 1.0 / A[diag_pos[i]];
}

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

void launch_local(hipStream_t s, int32_t nc, const double *xyz, const int32_t *hex8, const double *perm,
                  double mu, const uint8_t *fmask, const int32_t *cell_frac, const int32_t *frac_cell,
                  double *aK, double *rK, double *AKK, double *vol, double *fside, int *bad_cell) {
    if (nc <= 0) return;
    hipLaunchKernelGGL(vag_local_kernel, dim3(nblk(nc, 128)), dim3(128), 0, s, nc, xyz, hex8, perm,
                       1.0 / mu, fmask, cell_frac, frac_cell, aK, rK, AKK, vol, fside, bad_cell);
    VAG_HIP(hipGetLastError());
}

void launch_frac_local(hipStream_t s, int32_t nf, const double *xyz, const int32_t *frac_nodes,
                       const double *width, const double *perm, double mu, double *A5, double *area) {
    if (nf <= 0) return;
    hipLaunchKernelGGL(vag_frac_kernel, dim3(nblk(nf, 256)), dim3(256), 0, s, nf, xyz, frac_nodes, width,
                       perm, 1.0 / mu, A5, area);
    VAG_HIP(hipGetLastError());
}

void launch_check_coef(hipStream_t s, int32_t nc, const double *perm, int32_t nf, const double *fwidth,
                       const double *fperm, int *bad) {
    const int64_t n = (int64_t)nc + nf;
    if (n <= 0) return;
    hipLaunchKernelGGL(check_coef_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nc, perm, nf, fwidth,
                       fperm, bad);
    VAG_HIP(hipGetLastError());
}

void launch_node_pos(hipStream_t s, const AsmArgs &g, uint16_t *node_pos) {
    if (g.nfree > 0) hipLaunchKernelGGL(node_pos_kernel, dim3(nblk(g.nfree, 128)), dim3(128), 0, s, g, node_pos);
    VAG_HIP(hipGetLastError());
}

void launch_assemble(hipStream_t s, const AsmArgs &g, int32_t nkept, int32_t nelim) {
    if (g.nfree > 0) hipLaunchKernelGGL(asm_node_rows_kernel, dim3(nblk(g.nfree, 128)), dim3(128), 0, s, g);
    VAG_HIP(hipGetLastError());
    if (nkept > 0) hipLaunchKernelGGL(asm_face_rows_kernel, dim3(nblk(nkept, 128)), dim3(128), 0, s, g, nkept);
    VAG_HIP(hipGetLastError());
    if (nelim > 0) hipLaunchKernelGGL(asm_elim_rows_kernel, dim3(nblk(nelim, 128)), dim3(128), 0, s, g, nelim);
    VAG_HIP(hipGetLastError());
}

void launch_sell_fill(hipStream_t s, int32_t n, int64_t nslice, const int32_t *row_ptr, const int32_t *col,
                      const int64_t *sell_ptr, int32_t *sell_col, int32_t *row_len, int32_t *diag_pos) {
    if (nslice <= 0) return;
    hipLaunchKernelGGL(sell_fill_kernel, dim3(nblk(nslice * 64, 256)), dim3(256), 0, s, n, nslice, row_ptr, col,
                       sell_ptr, sell_col, row_len, diag_pos);
    VAG_HIP(hipGetLastError());
}

void launch_sell_pack(hipStream_t s, int32_t n, const int64_t *ptr, const int32_t *col, const int32_t *row_len,
                      uint16_t *col16, int32_t *cbase) {
    const int64_t nslice = ((int64_t)n + 63) / 64;
    if (nslice <= 0) return;
    hipLaunchKernelGGL(sell_pack_kernel, dim3((unsigned)nslice), dim3(64), 0, s, n, ptr, col, row_len, col16, cbase);
    VAG_HIP(hipGetLastError());
}

void launch_grp_pos(hipStream_t s, const AsmArgs &g, int32_t ngroup, const int64_t *grp_poff, int32_t *grp_pos) {
    if (ngroup <= 0) return;
    hipLaunchKernelGGL(grp_pos_kernel, dim3(ngroup), dim3(64), 0, s, g, grp_poff, grp_pos);
    VAG_HIP(hipGetLastError());
}

void launch_group_elim(hipStream_t s, int32_t first, int32_t ngroup, int max_g, int max_m, const int32_t *grp_ptr,
                       const int32_t *grp_face, const int32_t *grp_nptr, const int32_t *grp_node,
                       const int64_t *grp_off, const int64_t *grp_poff, const int32_t *grp_pos,
                       const int32_t *frac_unk, double *Gb, double *A, double *b, int *bad) {
    if (ngroup <= 0) return;
    if (max_g > kGroupMaxFaces || max_m > kGroupMaxNodes) throw Error(VAG_ERR_ARG, "internal: group too large");
    const size_t lds = (size_t)max_g * (max_g + max_m + 1) * sizeof(double);
    hipLaunchKernelGGL(vag_group_elim_kernel, dim3(ngroup), dim3(64), lds, s, first, ngroup, grp_ptr, grp_face,
                       grp_nptr, grp_node, grp_off, grp_poff, grp_pos, frac_unk, Gb, A, b, bad);
    VAG_HIP(hipGetLastError());
}

void launch_group_back(hipStream_t s, int32_t ngroup, const int32_t *grp_ptr, const int32_t *grp_face,
                       const int32_t *grp_nptr, const int32_t *grp_node, const int64_t *grp_off,
                       const int32_t *frac_unk, const double *Gb, const double *b, double *x) {
    if (ngroup <= 0) return;
    hipLaunchKernelGGL(vag_group_back_kernel, dim3(ngroup), dim3(64), 0, s, ngroup, grp_ptr, grp_face, grp_nptr,
                       grp_node, grp_off, frac_unk, Gb, b, x);
    VAG_HIP(hipGetLastError());
}

void launch_diag_inv(hipStream_t s, int32_t n, const int32_t *diag_pos, const double *A, double *dinv) {
    if (n <= 0) return;
    hipLaunchKernelGGL(vag_diag_inv_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, n, diag_pos, A, dinv);
    VAG_HIP(hipGetLastError());
}

}  // namespace vag
