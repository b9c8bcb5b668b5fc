// Assembly of the cell-eliminated VAG system (§3.1 and §4.2 of the paper).
//
// vag_local_kernel   one thread per cell: the local VAG matrix a_{K,nu}^{nu'}
//                    (eq VAGFluxMatrix) from the 24 sub-tetrahedra, its row sums
//                    r_nu and A_KK = sum r_nu.
// vag_frac_kernel    one thread per fracture face: the 5x5 P1 stiffness of
//                    d_f Lambda_f / mu on the face's 4 triangles (eq VAGFluxFracture).
// vag_scatter_kernel one thread per cell of one colour: the cell Schur block
//                    M_K = a - r r^T / A_KK (eq eqschur) and, for fracture
//                    faces the cell owns (lower cell index), the fracture block,
//                    added into the CSR values; Dirichlet columns go to b.
//                    Cells of a colour share no node, so no atomics are needed
//                    and the summation order is fixed.
//
// Storage of the local data (structure of arrays, coalesced by cell index):
//   aK[36][nc]  packed upper triangle of the node block a_{s,s'}
//   rK[8][nc]   row sums r_s (including couplings to fracture faces)
//   AKK[nc], vol[nc]
//   fside[nf*2][6] per (fracture face, side): a_{sigma,sigma}, a_{sigma,s} for
//               the face's 4 nodes in the cell's local face order, r_sigma
//   A5[nf][25]  fracture 5x5 over (sigma, input nodes 0..3)
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

// Adds v at the position given by a slot code; a Dirichlet column goes to b.
__device__ inline void put(int32_t slot, double v, int32_t row, double pb, double *__restrict__ A,
                           double *__restrict__ b) {
    if (slot >= 0)
        A[slot] += v;
    else if (slot == -2)
        b[row] -= v * pb;
}

// Scatters M_K = a - r r^T / A_KK of the cells of one colour.  Rows of an
// eliminated fracture face go to the dense group blocks Gb instead of A.
__global__ __launch_bounds__(128) void vag_scatter_kernel(
    int32_t ncell, const int32_t *__restrict__ cells, int32_t nc, int32_t nsys,
    const int32_t *__restrict__ hex8, const uint8_t *__restrict__ fmask,
    const int32_t *__restrict__ cell_frac, const int32_t *__restrict__ frac_cell,
    const int32_t *__restrict__ frac_slot, const int32_t *__restrict__ frac_nodes,
    const int32_t *__restrict__ node_unk, const int32_t *__restrict__ frac_unk, const double *__restrict__ p_bar,
    const double *__restrict__ aK, const double *__restrict__ rK, const double *__restrict__ AKK,
    const double *__restrict__ fside, const double *__restrict__ A5, const int64_t *__restrict__ slot_ptr,
    const int32_t *__restrict__ slots, double *__restrict__ A, double *__restrict__ Gb, double *__restrict__ b) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncell) return;
    const int32_t K = cells[t];
    const unsigned mask = fmask[K];
    const int m = 8 + __popc(mask);
    const int32_t *sl = slots + slot_ptr[K];
    const double inv = 1.0 / AKK[K];
    int32_t nid[8], row[8];
    double r[8], pb[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        nid[a] = hex8[8 * (int64_t)K + a];
        row[a] = node_unk[nid[a]];
        pb[a] = row[a] < 0 ? p_bar[nid[a]] : 0.0;
        r[a] = rK[(int64_t)a * nc + K];
    }
    // node-node block of M_K = a - r r^T / A_KK
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        if (row[a] < 0) continue;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const double v = aK[(int64_t)sym8(a, c) * nc + K] - r[a] * r[c] * inv;
            put(sl[a * m + c], v, row[a], pb[c], A, b);
        }
    }
    if (!mask) return;
    // fracture-face rows and columns of M_K
    double rs[6];
    int32_t sig[6];
    int sd[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        rs[f] = 0.0;
        sig[f] = -1;
        sd[f] = 0;
        if ((mask >> f) & 1u) {
            sig[f] = cell_frac[6 * (int64_t)K + f];
            sd[f] = (frac_cell[2 * (int64_t)sig[f]] == K) ? 0 : 1;
            rs[f] = fside[(2 * (int64_t)sig[f] + sd[f]) * 6 + 5];
        }
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        if (!((mask >> f) & 1u)) continue;
        const int j = 8 + __popc(mask & ((1u << f) - 1u));
        const int32_t frow = frac_unk[sig[f]];
        double *Af = frow >= nsys ? Gb : A;  // row of sigma
        const double *o = fside + (2 * (int64_t)sig[f] + sd[f]) * 6;
        double af[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) af[c] = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) af[hexf(f, i)] = o[1 + i];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const double v = af[c] - rs[f] * r[c] * inv;
            put(sl[j * m + c], v, frow, pb[c], Af, b);   // row sigma, column node c
            put(sl[c * m + j], v, row[c], 0.0, A, b);    // row node c, column sigma (-1: not stored)
        }
#pragma unroll
        for (int f2 = 0; f2 < 6; ++f2) {
            if (!((mask >> f2) & 1u)) continue;
            const int j2 = 8 + __popc(mask & ((1u << f2) - 1u));
            const double v = (f2 == f ? o[0] : 0.0) - rs[f] * rs[f2] * inv;
            put(sl[j * m + j2], v, frow, 0.0, Af, b);
        }
        // fracture block of sigma, added by its lower-index cell:
        // (sigma,sigma) += R, (sigma,s) = (s,sigma) += -rho_s, (s,s') += a_sigma
        if (sd[f] == 0) {
            const double *M = A5 + 25 * (int64_t)sig[f];
            int q[4];
            int32_t fn[4];
            double fpb[4];
            int32_t frw[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                q[i] = frac_slot[4 * (int64_t)sig[f] + i];
                fn[i] = frac_nodes[4 * (int64_t)sig[f] + i];
                frw[i] = node_unk[fn[i]];
                fpb[i] = frw[i] < 0 ? p_bar[fn[i]] : 0.0;
            }
            put(sl[j * m + j], M[0], frow, 0.0, Af, b);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                put(sl[j * m + q[i]], M[1 + i], frow, fpb[i], Af, b);
                if (frw[i] < 0) continue;
                put(sl[q[i] * m + j], M[5 * (1 + i)], frw[i], 0.0, A, b);
#pragma unroll
                for (int k = 0; k < 4; ++k) put(sl[q[i] * m + q[k]], M[5 * (1 + i) + 1 + k], frw[i], fpb[k], A, b);
            }
        }
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

void launch_scatter(hipStream_t s, int32_t ncell_color, const int32_t *cells, int32_t nc, int32_t nsys,
                    const int32_t *hex8, const uint8_t *fmask, const int32_t *cell_frac,
                    const int32_t *frac_cell, const int32_t *frac_slot, const int32_t *frac_nodes,
                    const int32_t *node_unk, const int32_t *frac_unk, const double *p_bar, const double *aK,
                    const double *rK, const double *AKK, const double *fside, const double *A5,
                    const int64_t *slot_ptr, const int32_t *slots, double *A, double *Gb, double *b) {
    if (ncell_color <= 0) return;
    hipLaunchKernelGGL(vag_scatter_kernel, dim3(nblk(ncell_color, 128)), dim3(128), 0, s, ncell_color,
                       cells, nc, nsys, hex8, fmask, cell_frac, frac_cell, frac_slot, frac_nodes, node_unk,
                       frac_unk, p_bar, aK, rK, AKK, fside, A5, slot_ptr, slots, A, Gb, b);
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
