// Darcy assembly and fluxes on general cells (cells given by their faces,
// §3.1; the tetrahedra, pyramids, prisms and hexahedra of §5.3-§5.5), one
// thread per cell or fracture face:
//
// gen_local_kernel      the local VAG matrix a_{K,nu}^{nu'} (eq VAGFluxMatrix)
//                       over the cell's nodes and fracture faces, from the
//                       sub-tetrahedra (x_K, x_sigma, s_e, s_e+1) of its faces,
//                       with non-fracture face centres interpolated by
//                       beta = 1/|V_sigma|; its row sums r, A_KK = sum r, and
//                       the Schur block M_K = a - r r^T / A_KK (eq eqschur)
// gen_frac_kernel       the P1 stiffness of d_f Lambda_f / mu on the triangles
//                       (x_sigma, s_e, s_e+1) of a fracture face
//                       (eq VAGFluxFracture), over (sigma, its nodes)
// gen_assemble_kernel   every stored entry of the system: the sum of the
//                       local entries that the symbolic phase listed for it
// gen_rhs_kernel        b = -sum of M p_bar over the Dirichlet columns
// gen_flux_kernel       u_K (eq eqschurcell) and F_{K,nu} per cell
// gen_frac_flux_kernel  F_{sigma,s} per fracture face
// gen_porous_kernel     porous volumes with alpha_{K,s} = 1/(2 |V_K|),
//                       alpha_{sigma,s} = 1/(2 |V_sigma|) (§3.2.1)
//
// Faces may be listed in either orientation: the k sub-tetrahedra of a face
// have signed volumes of one sign (checked), and |T| is their absolute value.
#include "vag_internal.h"

namespace vag {

namespace {

constexpr int kMaxM = kGenMaxNodes + kGenMaxFaces;  // unknowns of a cell

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
__device__ inline V3 node(const double *xyz, int32_t s) {
    return {xyz[3 * (int64_t)s], xyz[3 * (int64_t)s + 1], xyz[3 * (int64_t)s + 2]};
}

}  // namespace

// NV, NF, FK: the most nodes, faces and face nodes of a cell in the mesh, so
// that the thread's arrays (the local matrix over at most NV + NF unknowns)
// are no larger than the mesh needs: a tetrahedral mesh keeps 8 x 8 instead of
// 14 x 14 per thread
template <int NV, int NF, int FK>
__global__ __launch_bounds__(128) void gen_local_kernel(GenMesh g, const double *__restrict__ xyz,
                                                        const double *__restrict__ perm, double inv_mu,
                                                        double *__restrict__ loc, double *__restrict__ ga,
                                                        double *__restrict__ gr, double *__restrict__ AKKo,
                                                        double *__restrict__ volo, int *__restrict__ bad_cell) {
    constexpr int kM = NV + NF;
    const int32_t K = blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= g.nc) return;
    const int32_t p0 = g.cnode_ptr[K], nv = g.cnode_ptr[K + 1] - p0;
    V3 X[NV];
    V3 xK = {0, 0, 0};
    for (int i = 0; i < nv; ++i) {
        X[i] = node(xyz, g.cnode[p0 + i]);
        xK.x += X[i].x;
        xK.y += X[i].y;
        xK.z += X[i].z;
    }
    xK.x /= nv;
    xK.y /= nv;
    xK.z /= nv;
    double L[6];
    for (int i = 0; i < 6; ++i) L[i] = perm[6 * (int64_t)K + i] * inv_mu;
    // unknowns: the nodes (local order), then the fracture faces by local face
    int fu[NF];
    int m = nv;
    for (int f = 0; f < NF; ++f) fu[f] = g.cell_frac[kGenMaxFaces * (int64_t)K + f] >= 0 ? m++ : -1;
    double a[kM * kM];
    for (int i = 0; i < kM * kM; ++i) a[i] = 0.0;
    double vol = 0.0;
    bool bad = false;
    for (int f = 0; f < NF; ++f) {
        const int k = g.cface_k[kGenMaxFaces * (int64_t)K + f];
        if (k == 0) continue;
        int ln[FK];
        V3 xs = {0, 0, 0};
        for (int i = 0; i < k; ++i) {
            ln[i] = g.cface_loc[(kGenMaxFaces * (int64_t)K + f) * kGenMaxFaceNodes + i];
            xs.x += X[ln[i]].x;
            xs.y += X[ln[i]].y;
            xs.z += X[ln[i]].z;
        }
        xs.x /= k;
        xs.y /= k;
        xs.z /= k;
        const V3 av = sub(xs, xK);
        // orientation of the face seen from x_K: the sign of its sub-tetrahedra
        double dsum = 0.0;
        for (int e = 0; e < k; ++e)
            dsum += dot(av, cross(sub(X[ln[e]], xK), sub(X[ln[(e + 1) % k]], xK)));
        const double sg = dsum < 0.0 ? -1.0 : 1.0;
        // stiffness over (face centre, face nodes) from the face's sub-tetrahedra;
        // with J = [x_sigma - x_K, s1 - x_K, s2 - x_K] the gradients of the
        // barycentric coordinates of x_sigma, s1, s2 are (b x c, c x a, a x b) / det
        constexpr int W = FK + 1;
        double S[W * W];
        for (int i = 0; i < W * W; ++i) S[i] = 0.0;
        for (int e = 0; e < k; ++e) {
            const int i1 = 1 + e, i2 = 1 + (e + 1) % k;
            const V3 b = sub(X[ln[e]], xK), c = sub(X[ln[(e + 1) % k]], xK);
            const V3 uc = cross(b, c), u1 = cross(c, av), u2 = cross(av, b);
            const double det = sg * dot(av, uc);
            bad |= !(det > 0.0);
            vol += det * (1.0 / 6.0);
            const double w = 1.0 / (6.0 * det);  // |T| g_i . L g_j = (u_i . L u_j) / (6 |det|)
            const V3 Lc = tmul(L, uc), L1 = tmul(L, u1), L2 = tmul(L, u2);
            const double s00 = w * dot(uc, Lc), s01 = w * dot(uc, L1), s02 = w * dot(uc, L2);
            const double s11 = w * dot(u1, L1), s12 = w * dot(u1, L2), s22 = w * dot(u2, L2);
            S[0] += s00;
            S[i1] += s01;
            S[i1 * W] += s01;
            S[i2] += s02;
            S[i2 * W] += s02;
            S[i1 * W + i1] += s11;
            S[i1 * W + i2] += s12;
            S[i2 * W + i1] += s12;
            S[i2 * W + i2] += s22;
        }
        if (fu[f] < 0) {
            // non-fracture face: the centre value is the mean of the face's nodes
            const double be = 1.0 / k;
            for (int i = 0; i < k; ++i)
                for (int j = 0; j < k; ++j)
                    a[ln[i] * kM + ln[j]] +=
                        S[(1 + i) * W + 1 + j] + be * (S[1 + i] + S[1 + j]) + be * be * S[0];
        } else {
            const int t = fu[f];
            for (int i = 0; i < k; ++i) {
                for (int j = 0; j < k; ++j) a[ln[i] * kM + ln[j]] += S[(1 + i) * W + 1 + j];
                a[t * kM + ln[i]] += S[1 + i];
                a[ln[i] * kM + t] += S[1 + i];
            }
            a[t * kM + t] += S[0];
        }
    }
    double r[kM];
    double akk = 0.0;
    for (int i = 0; i < m; ++i) {
        double t = 0.0;
        for (int j = 0; j < m; ++j) t += a[i * kM + j];
        r[i] = t;
        akk += t;
    }
    const int64_t off = g.loc_off[K];
    for (int i = 0; i < m; ++i) {
        gr[g.unk_off[K] + i] = r[i];
        for (int j = 0; j < m; ++j) {
            ga[off + i * m + j] = a[i * kM + j];
            loc[off + i * m + j] = a[i * kM + j] - r[i] * r[j] / akk;
        }
    }
    AKKo[K] = akk;
    volo[K] = vol;
    if (bad) atomicMin(bad_cell, K);
}

__global__ __launch_bounds__(256) void gen_frac_kernel(GenMesh g, const double *__restrict__ xyz,
                                                       const double *__restrict__ fwidth,
                                                       const double *__restrict__ fperm, double inv_mu,
                                                       double *__restrict__ loc, double *__restrict__ areao) {
    const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= g.nf) return;
    const int32_t p0 = g.fnode_ptr[f], k = g.fnode_ptr[f + 1] - p0, k1 = k + 1;
    V3 P[kGenMaxFaceNodes];
    V3 xs = {0, 0, 0};
    for (int i = 0; i < k; ++i) {
        P[i] = node(xyz, g.fnode[p0 + i]);
        xs.x += P[i].x;
        xs.y += P[i].y;
        xs.z += P[i].z;
    }
    xs.x /= k;
    xs.y /= k;
    xs.z /= k;
    const double kap = fwidth[f] * fperm[f] * inv_mu;
    double A[(kGenMaxFaceNodes + 1) * (kGenMaxFaceNodes + 1)];
    for (int i = 0; i < k1 * k1; ++i) A[i] = 0.0;
    double area = 0.0;
    for (int e = 0; e < k; ++e) {
        // triangle (x_sigma, s_e, s_e+1): in-plane gradients of its barycentric
        // coordinates, grad lambda_i = n x (p_{i+2} - p_{i+1}) / |n|^2
        const V3 p[3] = {xs, P[e], P[(e + 1) % k]};
        const int id[3] = {0, 1 + e, 1 + (e + 1) % k};
        const V3 n = cross(sub(p[1], p[0]), sub(p[2], p[0]));
        const double nn = dot(n, n), ar = 0.5 * sqrt(nn);
        V3 gr3[3];
        for (int i = 0; i < 3; ++i) {
            const V3 c = cross(n, sub(p[(i + 2) % 3], p[(i + 1) % 3]));
            gr3[i] = {c.x / nn, c.y / nn, c.z / nn};
        }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) A[id[i] * k1 + id[j]] += kap * ar * dot(gr3[i], gr3[j]);
        area += ar;
    }
    const int64_t off = g.loc_off[g.nc + f];
    for (int i = 0; i < k1 * k1; ++i) loc[off + i] = A[i];
    areao[f] = area;
}

__global__ __launch_bounds__(256) void gen_assemble_kernel(int64_t stored, const int64_t *__restrict__ con_ptr,
                                                           const int64_t *__restrict__ con,
                                                           const double *__restrict__ loc, double *__restrict__ A) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= stored) return;
    double v = 0.0;
    for (int64_t c = con_ptr[q]; c < con_ptr[q + 1]; ++c) v += loc[con[c]];
    A[q] = v;
}

__global__ __launch_bounds__(256) void gen_rhs_kernel(int32_t nunk, const int32_t *__restrict__ bcon_ptr,
                                                      const int64_t *__restrict__ bcon,
                                                      const int32_t *__restrict__ bcon_node,
                                                      const double *__restrict__ loc,
                                                      const double *__restrict__ p_bar, double *__restrict__ b) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nunk) return;
    double v = 0.0;
    for (int32_t c = bcon_ptr[r]; c < bcon_ptr[r + 1]; ++c) v -= loc[bcon[c]] * p_bar[bcon_node[c]];
    b[r] = v;
}

__global__ __launch_bounds__(128) void gen_flux_kernel(GenMesh g, const double *__restrict__ ga,
                                                       const double *__restrict__ gr,
                                                       const double *__restrict__ AKK,
                                                       const double *__restrict__ u_node,
                                                       const double *__restrict__ u_frac,
                                                       double *__restrict__ u_cell, double *__restrict__ F) {
    const int32_t K = blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= g.nc) return;
    const int32_t p0 = g.cnode_ptr[K], nv = g.cnode_ptr[K + 1] - p0;
    double u[kMaxM];
    int fr[kGenMaxFaces];
    int m = 0;
    for (int i = 0; i < nv; ++i) u[m++] = u_node[g.cnode[p0 + i]];
    for (int f = 0; f < kGenMaxFaces; ++f) {
        const int32_t sg = g.cell_frac[kGenMaxFaces * (int64_t)K + f];
        if (sg >= 0) {
            fr[m - nv] = sg;
            u[m++] = u_frac[sg];
        }
    }
    const double *r = gr + g.unk_off[K];
    double t = 0.0;
    for (int i = 0; i < m; ++i) t += r[i] * u[i];
    const double uK = t / AKK[K];  // eq eqschurcell with zero cell right-hand side
    u_cell[K] = uK;
    const double *a = ga + g.loc_off[K];
    for (int i = 0; i < m; ++i) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += a[i * m + j] * (uK - u[j]);
        if (i < nv) {
            F[p0 + i] = s;
        } else {
            const int32_t sg = fr[i - nv];
            const int side = g.frac_cell[2 * (int64_t)sg] == K ? 0 : 1;
            F[g.ncn + 2 * (int64_t)sg + side] = s;
        }
    }
}

__global__ __launch_bounds__(256) void gen_frac_flux_kernel(GenMesh g, const double *__restrict__ loc,
                                                            const double *__restrict__ u_node,
                                                            const double *__restrict__ u_frac,
                                                            double *__restrict__ F) {
    const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= g.nf) return;
    const int32_t p0 = g.fnode_ptr[f], k = g.fnode_ptr[f + 1] - p0, k1 = k + 1;
    const double *A = loc + g.loc_off[g.nc + f];
    const double us = u_frac[f];
    for (int i = 0; i < k; ++i) {
        double s = 0.0;
        for (int j = 0; j < k; ++j) s += A[(1 + i) * k1 + 1 + j] * (us - u_node[g.fnode[p0 + j]]);
        F[g.ncn + 2 * (int64_t)g.nf + p0 + i] = s;
    }
}

// With pmax, a cell (fracture face) gives a node its share only if its
// permeability reaches pmax[node] (§3.2.1, nodes between rock types).
__global__ __launch_bounds__(256) void gen_porous_kernel(
    GenMesh g, const uint8_t *__restrict__ dirichlet, const uint8_t *__restrict__ frac_node,
    const int64_t *__restrict__ inc_ptr, const int32_t *__restrict__ inc_other, const double *__restrict__ vol,
    const double *__restrict__ poro, const double *__restrict__ area, const double *__restrict__ fwidth,
    const double *__restrict__ fporo, const double *__restrict__ perm, const double *__restrict__ fperm,
    const double *__restrict__ pmax, double *__restrict__ phi_cell, double *__restrict__ phi_frac,
    double *__restrict__ phi_node) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t off_f = g.nc, off_n = (int64_t)g.nc + g.nf;
    if (i >= off_n + g.nn) return;
    if (i < off_f) {
        const int32_t K = (int32_t)i, p0 = g.cnode_ptr[K], nv = g.cnode_ptr[K + 1] - p0;
        const double alpha = 0.5 / nv;
        const double mK = pmax ? perm_measure(perm, K) : 0.0;
        double sa = 0.0;
        for (int a = 0; a < nv; ++a) {
            const int32_t s = g.cnode[p0 + a];
            if (!dirichlet[s] && !frac_node[s] && (!pmax || mK >= pmax[s])) sa += alpha;
        }
        phi_cell[K] = (1.0 - sa) * (vol[K] * poro[K]);
    } else if (i < off_n) {
        const int32_t f = (int32_t)(i - off_f), p0 = g.fnode_ptr[f], k = g.fnode_ptr[f + 1] - p0;
        const double alpha = 0.5 / k;
        double sa = 0.0;
        for (int a = 0; a < k; ++a) {
            const int32_t s = g.fnode[p0 + a];
            if (!dirichlet[s] && (!pmax || fperm[f] >= pmax[s])) sa += alpha;
        }
        phi_frac[f] = (1.0 - sa) * (fwidth[f] * area[f] * fporo[f]);
    } else {
        // a node takes 1/(2 |V|) of each adjacent control volume it draws
        // from: the fracture faces around a fracture node, else the cells
        const int32_t s = (int32_t)(i - off_n);
        double p = 0.0;
        if (!dirichlet[s]) {
            const bool fn = frac_node[s] != 0;
            for (int64_t q = inc_ptr[i]; q < inc_ptr[i + 1]; ++q) {
                const int32_t o = inc_other[q];
                if (o < off_f && !fn) {
                    if (pmax && perm_measure(perm, o) < pmax[s]) continue;
                    const int nv = g.cnode_ptr[o + 1] - g.cnode_ptr[o];
                    p += (0.5 / nv) * (vol[o] * poro[o]);
                } else if (o >= off_f && o < off_n && fn) {
                    const int32_t f = o - (int32_t)off_f;
                    if (pmax && fperm[f] < pmax[s]) continue;
                    const int k = g.fnode_ptr[f + 1] - g.fnode_ptr[f];
                    p += (0.5 / k) * (fwidth[f] * area[f] * fporo[f]);
                }
            }
        }
        phi_node[s] = p;
    }
}

// the largest permeability around each node, from its incidence list
__global__ __launch_bounds__(256) void gen_node_pmax_kernel(GenMesh g, const uint8_t *__restrict__ frac_node,
                                                            const int64_t *__restrict__ inc_ptr,
                                                            const int32_t *__restrict__ inc_other,
                                                            const double *__restrict__ perm,
                                                            const double *__restrict__ fperm,
                                                            double *__restrict__ pmax) {
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.nn) return;
    const int64_t off_f = g.nc, off_n = (int64_t)g.nc + g.nf, i = off_n + s;
    const bool fn = frac_node[s] != 0;
    double m = -1.0;
    for (int64_t q = inc_ptr[i]; q < inc_ptr[i + 1]; ++q) {
        const int32_t o = inc_other[q];
        if (o < off_f && !fn) m = fmax(m, perm_measure(perm, o));
        else if (o >= off_f && o < off_n && fn) m = fmax(m, fperm[o - off_f]);
    }
    pmax[s] = m;
}

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

void launch_gen_local(hipStream_t s, const GenMesh &g, const double *xyz, const double *perm, double inv_mu,
                      double *loc, double *ga, double *gr, double *AKK, double *vol, int *bad_cell) {
    if (g.nc <= 0) return;
    const dim3 G(nblk(g.nc, 128)), B(128);
    if (g.max_nv <= 4 && g.max_nf <= 4 && g.max_fk <= 3)  // tetrahedra
        hipLaunchKernelGGL((gen_local_kernel<4, 4, 3>), G, B, 0, s, g, xyz, perm, inv_mu, loc, ga, gr, AKK, vol,
                           bad_cell);
    else if (g.max_nv <= 6 && g.max_nf <= 5)  // prisms, pyramids (and tetrahedra)
        hipLaunchKernelGGL((gen_local_kernel<6, 5, kGenMaxFaceNodes>), G, B, 0, s, g, xyz, perm, inv_mu, loc, ga,
                           gr, AKK, vol, bad_cell);
    else
        hipLaunchKernelGGL((gen_local_kernel<kGenMaxNodes, kGenMaxFaces, kGenMaxFaceNodes>), G, B, 0, s, g, xyz,
                           perm, inv_mu, loc, ga, gr, AKK, vol, bad_cell);
    VAG_HIP(hipGetLastError());
}
void launch_gen_frac_local(hipStream_t s, const GenMesh &g, const double *xyz, const double *fwidth,
                           const double *fperm, double inv_mu, double *loc, double *area) {
    if (g.nf <= 0) return;
    hipLaunchKernelGGL(gen_frac_kernel, dim3(nblk(g.nf, 256)), dim3(256), 0, s, g, xyz, fwidth, fperm, inv_mu, loc,
                       area);
    VAG_HIP(hipGetLastError());
}
void launch_gen_assemble(hipStream_t s, int64_t stored, const int64_t *con_ptr, const int64_t *con,
                         const double *loc, double *A) {
    if (stored <= 0) return;
    hipLaunchKernelGGL(gen_assemble_kernel, dim3(nblk(stored, 256)), dim3(256), 0, s, stored, con_ptr, con, loc, A);
    VAG_HIP(hipGetLastError());
}
void launch_gen_rhs(hipStream_t s, int32_t nunk, const int32_t *bcon_ptr, const int64_t *bcon,
                    const int32_t *bcon_node, const double *loc, const double *p_bar, double *b) {
    if (nunk <= 0) return;
    hipLaunchKernelGGL(gen_rhs_kernel, dim3(nblk(nunk, 256)), dim3(256), 0, s, nunk, bcon_ptr, bcon, bcon_node, loc,
                       p_bar, b);
    VAG_HIP(hipGetLastError());
}
void launch_gen_flux(hipStream_t s, const GenMesh &g, const double *loc, const double *ga, const double *gr,
                     const double *AKK, const double *u_node, const double *u_frac, double *u_cell, double *F) {
    if (g.nc > 0)
        hipLaunchKernelGGL(gen_flux_kernel, dim3(nblk(g.nc, 128)), dim3(128), 0, s, g, ga, gr, AKK, u_node, u_frac,
                           u_cell, F);
    if (g.nf > 0)
        hipLaunchKernelGGL(gen_frac_flux_kernel, dim3(nblk(g.nf, 256)), dim3(256), 0, s, g, loc, u_node, u_frac, F);
    VAG_HIP(hipGetLastError());
}
void launch_gen_porous(hipStream_t s, const GenMesh &g, const uint8_t *dirichlet, const uint8_t *frac_node,
                       const int64_t *inc_ptr, const int32_t *inc_other, const double *vol, const double *poro,
                       const double *area, const double *fwidth, const double *fporo, const double *perm,
                       const double *fperm, const double *pmax, double *phi_cell, double *phi_frac,
                       double *phi_node) {
    const int64_t total = (int64_t)g.nc + g.nf + g.nn;
    hipLaunchKernelGGL(gen_porous_kernel, dim3(nblk(total, 256)), dim3(256), 0, s, g, dirichlet, frac_node, inc_ptr,
                       inc_other, vol, poro, area, fwidth, fporo, perm, fperm, pmax, phi_cell, phi_frac, phi_node);
    VAG_HIP(hipGetLastError());
}
void launch_gen_node_pmax(hipStream_t s, const GenMesh &g, const uint8_t *frac_node, const int64_t *inc_ptr,
                          const int32_t *inc_other, const double *perm, const double *fperm, double *pmax) {
    if (g.nn <= 0) return;
    hipLaunchKernelGGL(gen_node_pmax_kernel, dim3(nblk(g.nn, 256)), dim3(256), 0, s, g, frac_node, inc_ptr,
                       inc_other, perm, fperm, pmax);
    VAG_HIP(hipGetLastError());
}

}  // namespace vag
