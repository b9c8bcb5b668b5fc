/*
 * FP64 CPU oracle for the hybrid-dimensional VAG scheme (Darcy flow with
 * fracture faces, then explicit first-order upwind transport).
 *
 * TEST INFRASTRUCTURE ONLY.  Tests, the smoke check and the CPU baseline leg of
 * the benchmark call this file; the product library never links or runs it and
 * shares no source with it.  It favours plain loops over speed: every quantity
 * is computed from its definition in the paper, in the paper's order.
 *
 * Paper: Xing, Masson, Lopez, "Parallel Vertex Approximate Gradient
 * discretization of hybrid dimensional Darcy flow and transport in discrete
 * fracture networks" (arXiv:1602.03641).
 *
 * Readings where the paper is silent (listed again in the design notes):
 *  - cell centre x_K = mean of the cell's nodes; face centre weights
 *    beta_{sigma,s} = 1/4 (quadrilateral faces);
 *  - Dirichlet data is given per node; a node without the flag gets the
 *    conservation equation of an interior node (homogeneous Neumann is natural
 *    in the Galerkin form), and in the transport formulas the Dirichlet set
 *    replaces V_ext;
 *  - volume fractions alpha_{K,s} = 1/(2*8) and alpha_{sigma,s} = 1/(2*4)
 *    (one rocktype for all matrix cells; fracture nodes take volume from the
 *    fracture only, as §3.2.1 requires);
 *  - Krylov stopping rule ||b - A x||_2 <= rtol ||b||_2 from x = 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "vag_oracle.h"

/* Faces of a VTK hexahedron, each listed cyclically (consecutive entries are
 * the face's edges) and oriented with the outward normal by the right-hand
 * rule, so every sub-tetrahedron (x_K, x_sigma, s_e, s_e+1) of a valid cell has
 * positive signed volume. */
static const int HEXF[6][4] = {
    {0, 4, 7, 3}, {1, 2, 6, 5}, {0, 1, 5, 4}, {3, 7, 6, 2}, {0, 3, 2, 1}, {4, 5, 6, 7}};

/* ------------------------------------------------------------------------ */
/* small dense helpers                                                       */
/* ------------------------------------------------------------------------ */

static double det3(const double J[3][3]) {
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

/* Gradients of the four barycentric coordinates of tetrahedron (p0,p1,p2,p3)
 * and its signed volume.  With J = [p1-p0, p2-p0, p3-p0] (columns), the
 * gradients of lambda_1..3 are the rows of J^{-1}; lambda_0 = 1 - sum. */
static double tet_gradients(const double *p0, const double *p1, const double *p2,
                            const double *p3, double g[4][3]) {
    double J[3][3];
    for (int r = 0; r < 3; ++r) {
        J[r][0] = p1[r] - p0[r];
        J[r][1] = p2[r] - p0[r];
        J[r][2] = p3[r] - p0[r];
    }
    double d = det3(J);
    /* inverse = adjugate / det; row i of J^{-1} is the gradient of lambda_{i+1} */
    double inv[3][3];
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / d;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / d;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / d;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / d;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / d;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / d;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / d;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / d;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / d;
    for (int c = 0; c < 3; ++c) {
        g[1][c] = inv[0][c];
        g[2][c] = inv[1][c];
        g[3][c] = inv[2][c];
        g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
    }
    return d / 6.0;
}

static void tensor_of(const double *p6, double L[3][3]) {
    L[0][0] = p6[0]; L[1][1] = p6[1]; L[2][2] = p6[2];
    L[0][1] = L[1][0] = p6[3];
    L[0][2] = L[2][0] = p6[4];
    L[1][2] = L[2][1] = p6[5];
}

/* ------------------------------------------------------------------------ */
/* topology: which local faces of each cell are fracture faces               */
/* ------------------------------------------------------------------------ */

static int same_set4(const int32_t *a, const int32_t *b) {
    for (int i = 0; i < 4; ++i) {
        int found = 0;
        for (int j = 0; j < 4; ++j) found |= (a[i] == b[j]);
        if (!found) return 0;
    }
    return 1;
}

/* Node -> cells lists (CSR), cells in increasing index. */
static void node_cells(const orc_problem *P, int64_t **ptr_out, int32_t **list_out) {
    int64_t nn = P->n_nodes, nc = P->n_cells;
    int64_t *ptr = (int64_t *)calloc((size_t)nn + 1, sizeof(int64_t));
    for (int64_t K = 0; K < nc; ++K)
        for (int a = 0; a < 8; ++a) ptr[P->hex8[8 * K + a] + 1]++;
    for (int64_t s = 0; s < nn; ++s) ptr[s + 1] += ptr[s];
    int32_t *list = (int32_t *)malloc(sizeof(int32_t) * (size_t)ptr[nn]);
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)nn);
    memcpy(fill, ptr, sizeof(int64_t) * (size_t)nn);
    for (int64_t K = 0; K < nc; ++K)
        for (int a = 0; a < 8; ++a) list[fill[P->hex8[8 * K + a]]++] = (int32_t)K;
    free(fill);
    *ptr_out = ptr;
    *list_out = list;
}

int orc_topology(const orc_problem *P, int32_t *cell_frac, int32_t *frac_cell,
                 int32_t *frac_lface) {
    int64_t nc = P->n_cells, nf = P->n_frac;
    for (int64_t i = 0; i < 6 * nc; ++i) cell_frac[i] = -1;
    for (int64_t i = 0; i < 2 * nf; ++i) frac_cell[i] = frac_lface[i] = -1;
    int64_t *ptr;
    int32_t *list;
    node_cells(P, &ptr, &list);
    int status = 0;
    for (int64_t f = 0; f < nf && !status; ++f) {
        const int32_t *fn = P->frac_nodes + 4 * f;
        int32_t s0 = fn[0];
        int nside = 0;
        for (int64_t q = ptr[s0]; q < ptr[s0 + 1]; ++q) {
            int32_t K = list[q];
            for (int lf = 0; lf < 6; ++lf) {
                int32_t cn[4];
                for (int i = 0; i < 4; ++i) cn[i] = P->hex8[8 * (int64_t)K + HEXF[lf][i]];
                if (!same_set4(cn, fn)) continue;
                if (cell_frac[6 * (int64_t)K + lf] >= 0) { status = -1; break; } /* listed twice */
                if (nside >= 2) { status = -2; break; }
                cell_frac[6 * (int64_t)K + lf] = (int32_t)f;
                frac_cell[2 * f + nside] = K;
                frac_lface[2 * f + nside] = lf;
                nside++;
            }
        }
        if (!status && nside == 0) status = -2; /* not a face of the mesh */
    }
    free(ptr);
    free(list);
    return status;
}

/* ------------------------------------------------------------------------ */
/* local VAG matrices                                                        */
/* ------------------------------------------------------------------------ */

/*
 * Matrix part of the VAG scheme in cell K (§3.1, definition of pi_T and the
 * matrix fluxes F_{K,nu}).
 *
 * 1. The cell is cut into the 24 tetrahedra T_{K,sigma,e} joining x_K to the
 *    triangles (x_sigma, e) of its faces.
 * 2. On that sub-mesh the P1 stiffness S = sum_T |T| G_T^T (Lambda_K / mu) G_T
 *    is accumulated over the 15 vertices {x_K, 8 nodes, 6 face centres}.
 * 3. Face centres of non-fracture faces are not unknowns: their value is the
 *    interpolation I_sigma(v) = sum_s beta_{sigma,s} v_s.  With the matrix
 *    Pm mapping the reduced unknowns (K, 8 nodes, the cell's fracture faces) to
 *    the 15 vertices, the reduced stiffness is Pm^T S Pm.
 * 4. a_{K,nu}^{nu'} = int_K Lambda/mu grad eta_nu . grad eta_nu' is its block
 *    over nu, nu' in V_K u F_{Gamma,K}.
 *
 * Output: m = 8 + (number of fracture faces of K); a is m x m row-major with the
 * 8 nodes in VTK slot order first, then the fracture faces by local face order.
 * Returns the cell volume |K|, or -1 if a sub-tetrahedron is not positive.
 */
double orc_cell_matrix(const orc_problem *P, int64_t K, const int32_t *cell_frac6, double *a,
                       int *m_out, double *full15) {
    const int32_t *cn = P->hex8 + 8 * K;
    double X[8][3];
    double xK[3] = {0, 0, 0};
    for (int i = 0; i < 8; ++i)
        for (int c = 0; c < 3; ++c) {
            X[i][c] = P->xyz[3 * (int64_t)cn[i] + c];
            xK[c] += X[i][c] / 8.0;
        }
    double L[3][3];
    tensor_of(P->perm + 6 * K, L);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) L[r][c] /= P->mu;

    double S[15][15];
    memset(S, 0, sizeof S);
    double vol = 0.0;
    int bad = 0;
    for (int f = 0; f < 6; ++f) {
        double xs[3] = {0, 0, 0};
        for (int i = 0; i < 4; ++i)
            for (int c = 0; c < 3; ++c) xs[c] += 0.25 * X[HEXF[f][i]][c];
        for (int e = 0; e < 4; ++e) {
            int s1 = HEXF[f][e], s2 = HEXF[f][(e + 1) % 4];
            double g[4][3];
            double v = tet_gradients(xK, xs, X[s1], X[s2], g);
            if (!(v > 0.0)) bad = 1;
            vol += v;
            int id[4] = {0, 9 + f, 1 + s1, 1 + s2};
            for (int i = 0; i < 4; ++i) {
                double Lg[3];
                for (int r = 0; r < 3; ++r) Lg[r] = L[r][0] * g[i][0] + L[r][1] * g[i][1] + L[r][2] * g[i][2];
                for (int j = 0; j < 4; ++j)
                    S[id[j]][id[i]] += v * (g[j][0] * Lg[0] + g[j][1] * Lg[1] + g[j][2] * Lg[2]);
            }
        }
    }
    if (full15) memcpy(full15, S, sizeof S);

    /* reduced unknowns: 0 = K, 1..8 = nodes, 9.. = fracture faces of K */
    int nfr = 0, fr_of_face[6];
    for (int f = 0; f < 6; ++f) fr_of_face[f] = (cell_frac6 && cell_frac6[f] >= 0) ? nfr++ : -1;
    int nr = 9 + nfr;
    double Pm[15][15];
    memset(Pm, 0, sizeof Pm);
    Pm[0][0] = 1.0;
    for (int s = 0; s < 8; ++s) Pm[1 + s][1 + s] = 1.0;
    for (int f = 0; f < 6; ++f) {
        if (fr_of_face[f] >= 0)
            Pm[9 + f][9 + fr_of_face[f]] = 1.0;
        else
            for (int i = 0; i < 4; ++i) Pm[9 + f][1 + HEXF[f][i]] += 0.25;
    }
    double SP[15][15], R[15][15];
    for (int i = 0; i < 15; ++i)
        for (int j = 0; j < nr; ++j) {
            double t = 0;
            for (int k = 0; k < 15; ++k) t += S[i][k] * Pm[k][j];
            SP[i][j] = t;
        }
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nr; ++j) {
            double t = 0;
            for (int k = 0; k < 15; ++k) t += Pm[k][i] * SP[k][j];
            R[i][j] = t;
        }
    int m = nr - 1;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) a[i * m + j] = R[1 + i][1 + j];
    *m_out = m;
    return bad ? -1.0 : vol;
}

/*
 * Fracture part (§3.1, fracture fluxes F_{sigma,s}): on the face sigma, the
 * trace of pi_T v is P1 on the 4 triangles (x_sigma, s_i, s_i+1).  The 5 x 5
 * stiffness over (sigma, s_1..s_4) of d_f Lambda_f / mu grad_tau . grad_tau is
 * accumulated triangle by triangle with in-plane gradients.  a_{sigma,s}^{s'}
 * is its node block.  Returns the face area |sigma|.
 */
double orc_frac_matrix(const orc_problem *P, int64_t f, double *A5) {
    const int32_t *fn = P->frac_nodes + 4 * f;
    double X[4][3], xs[3] = {0, 0, 0};
    for (int i = 0; i < 4; ++i)
        for (int c = 0; c < 3; ++c) {
            X[i][c] = P->xyz[3 * (int64_t)fn[i] + c];
            xs[c] += 0.25 * X[i][c];
        }
    double kappa = P->frac_width[f] * P->frac_perm[f] / P->mu;
    memset(A5, 0, sizeof(double) * 25);
    double area = 0.0;
    for (int e = 0; e < 4; ++e) {
        const double *p[3] = {xs, X[e], X[(e + 1) % 4]};
        int id[3] = {0, 1 + e, 1 + (e + 1) % 4};
        /* in-plane gradient of the barycentric coordinate of vertex i:
         * grad lambda_i = n x (p_{i+2} - p_{i+1}) / (2 A) with unit normal n */
        double e1[3], e2[3], nrm[3];
        for (int c = 0; c < 3; ++c) {
            e1[c] = p[1][c] - p[0][c];
            e2[c] = p[2][c] - p[0][c];
        }
        nrm[0] = e1[1] * e2[2] - e1[2] * e2[1];
        nrm[1] = e1[2] * e2[0] - e1[0] * e2[2];
        nrm[2] = e1[0] * e2[1] - e1[1] * e2[0];
        double twoA = sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
        for (int c = 0; c < 3; ++c) nrm[c] /= twoA;
        double g[3][3];
        for (int i = 0; i < 3; ++i) {
            const double *pa = p[(i + 1) % 3], *pb = p[(i + 2) % 3];
            double ed[3] = {pb[0] - pa[0], pb[1] - pa[1], pb[2] - pa[2]};
            g[i][0] = (nrm[1] * ed[2] - nrm[2] * ed[1]) / twoA;
            g[i][1] = (nrm[2] * ed[0] - nrm[0] * ed[2]) / twoA;
            g[i][2] = (nrm[0] * ed[1] - nrm[1] * ed[0]) / twoA;
        }
        double A = 0.5 * twoA;
        area += A;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                A5[id[i] * 5 + id[j]] += kappa * A * (g[i][0] * g[j][0] + g[i][1] * g[j][1] + g[i][2] * g[j][2]);
    }
    return area;
}

/* ------------------------------------------------------------------------ */
/* global system                                                             */
/* ------------------------------------------------------------------------ */

typedef struct { int64_t r, c; double v; } trip;

static int trip_cmp(const void *x, const void *y) {
    const trip *a = (const trip *)x, *b = (const trip *)y;
    if (a->r != b->r) return a->r < b->r ? -1 : 1;
    if (a->c != b->c) return a->c < b->c ? -1 : 1;
    return 0;
}

typedef struct {
    int64_t n;          /* unknowns: free nodes then fracture faces */
    int64_t *row_ptr;
    int64_t *col;
    double *val;
    double *b;
    int64_t *node_unk;  /* node -> unknown index, -1 for Dirichlet nodes */
    /* per-cell local data kept for cell recovery and fluxes */
    int *m;
    double **a;         /* a_K (m x m) */
    int32_t *cell_frac; /* [nc][6] */
    int32_t *frac_cell, *frac_lface;
    double *A5;         /* [nf][25] fracture 5x5 */
    double *cell_vol, *frac_area;
} orc_system;

static void free_system(orc_system *S, int64_t nc) {
    free(S->row_ptr); free(S->col); free(S->val); free(S->b); free(S->node_unk);
    if (S->a) for (int64_t K = 0; K < nc; ++K) free(S->a[K]);
    free(S->a); free(S->m); free(S->cell_frac); free(S->frac_cell); free(S->frac_lface);
    free(S->A5); free(S->cell_vol); free(S->frac_area);
    memset(S, 0, sizeof *S);
}

/*
 * Builds the system of §4.2 for a single process: the conservation equations
 * of cells, fracture faces and free nodes (§3.1), with the cell unknowns
 * eliminated by the Schur complement of the diagonal block A_cc
 * (equation eqschur), and the Dirichlet node values moved to the right-hand
 * side.  Unknown order: free nodes (by node index), then fracture faces.
 *
 * Cell K's equation is sum_nu F_{K,nu} = 0 with F_{K,nu} = sum_nu' a (u_K - u_nu'),
 * i.e. A_KK u_K - sum_nu r_nu u_nu = 0 with r_nu = sum_nu' a_{nu,nu'} and
 * A_KK = sum_nu r_nu.  The node and fracture-face equations carry -F_{K,nu},
 * so their cell column is -r_nu and their (nu, nu') block is a_{nu,nu'}.
 * Eliminating u_K adds -(-r_nu)(-r_nu')/A_KK to entry (nu, nu').
 * The fracture face equation adds sum_s F_{sigma,s}: (sigma,sigma) += R_sigma,
 * (sigma, s) and (s, sigma) += -rho_s, (s, s') += a_{sigma,s}^{s'}.
 */
static int build_system(const orc_problem *P, orc_system *S) {
    int64_t nn = P->n_nodes, nc = P->n_cells, nf = P->n_frac;
    memset(S, 0, sizeof *S);
    S->cell_frac = (int32_t *)malloc(sizeof(int32_t) * 6 * (size_t)nc);
    S->frac_cell = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(nf > 0 ? nf : 1));
    S->frac_lface = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(nf > 0 ? nf : 1));
    int st = orc_topology(P, S->cell_frac, S->frac_cell, S->frac_lface);
    if (st) return st;

    S->node_unk = (int64_t *)malloc(sizeof(int64_t) * (size_t)nn);
    int64_t nfree = 0;
    for (int64_t s = 0; s < nn; ++s) S->node_unk[s] = P->dirichlet[s] ? -1 : nfree++;
    S->n = nfree + nf;
    S->b = (double *)calloc((size_t)S->n + 1, sizeof(double));
    S->m = (int *)malloc(sizeof(int) * (size_t)nc);
    S->a = (double **)calloc((size_t)nc, sizeof(double *));
    S->cell_vol = (double *)malloc(sizeof(double) * (size_t)nc);
    S->A5 = (double *)malloc(sizeof(double) * 25 * (size_t)(nf > 0 ? nf : 1));
    S->frac_area = (double *)malloc(sizeof(double) * (size_t)(nf > 0 ? nf : 1));

    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t K = 0; K < nc; ++K) {
        double a[14 * 14];
        int m;
        double v = orc_cell_matrix(P, K, S->cell_frac + 6 * K, a, &m, NULL);
        if (v < 0) bad = 1;
        S->cell_vol[K] = v;
        S->m[K] = m;
        S->a[K] = (double *)malloc(sizeof(double) * (size_t)(m * m));
        memcpy(S->a[K], a, sizeof(double) * (size_t)(m * m));
    }
    if (bad) return -3;
    for (int64_t f = 0; f < nf; ++f) S->frac_area[f] = orc_frac_matrix(P, f, S->A5 + 25 * f);

    /* count triplets */
    int64_t ntr = 0;
    for (int64_t K = 0; K < nc; ++K) ntr += (int64_t)S->m[K] * S->m[K];
    ntr += 25 * nf;
    trip *T = (trip *)malloc(sizeof(trip) * (size_t)(ntr > 0 ? ntr : 1));
    int64_t nt = 0;

    for (int64_t K = 0; K < nc; ++K) {
        int m = S->m[K];
        const double *a = S->a[K];
        int64_t unk[14], nodeid[14];
        int q = 8;
        for (int i = 0; i < 8; ++i) {
            nodeid[i] = P->hex8[8 * K + i];
            unk[i] = S->node_unk[nodeid[i]];
        }
        for (int f = 0; f < 6; ++f)
            if (S->cell_frac[6 * K + f] >= 0) {
                nodeid[q] = -1;
                unk[q++] = nfree + S->cell_frac[6 * K + f];
            }
        double r[14], AKK = 0;
        for (int i = 0; i < m; ++i) {
            r[i] = 0;
            for (int j = 0; j < m; ++j) r[i] += a[i * m + j];
            AKK += r[i];
        }
        for (int i = 0; i < m; ++i) {
            if (unk[i] < 0) continue;
            for (int j = 0; j < m; ++j) {
                double v = a[i * m + j] - r[i] * r[j] / AKK;
                if (unk[j] >= 0) {
                    T[nt].r = unk[i]; T[nt].c = unk[j]; T[nt].v = v; nt++;
                } else {
                    S->b[unk[i]] -= v * P->p_bar[nodeid[j]];
                }
            }
        }
    }
    for (int64_t f = 0; f < nf; ++f) {
        const double *A5 = S->A5 + 25 * f;
        int64_t unk[5], nodeid[5];
        unk[0] = nfree + f; nodeid[0] = -1;
        for (int i = 0; i < 4; ++i) {
            nodeid[1 + i] = P->frac_nodes[4 * f + i];
            unk[1 + i] = S->node_unk[nodeid[1 + i]];
        }
        for (int i = 0; i < 5; ++i) {
            if (unk[i] < 0) continue;
            for (int j = 0; j < 5; ++j) {
                if (unk[j] >= 0) {
                    T[nt].r = unk[i]; T[nt].c = unk[j]; T[nt].v = A5[i * 5 + j]; nt++;
                } else {
                    S->b[unk[i]] -= A5[i * 5 + j] * P->p_bar[nodeid[j]];
                }
            }
        }
    }
    /* wells (§5.5): the face equation gains the inflow Q = WI (p_w - u_sigma) + q
     * on its right: WI on the diagonal, WI p_w + q into b */
    T = (trip *)realloc(T, sizeof(trip) * (size_t)(nt + P->n_wells + 1));
    for (int64_t k = 0; k < P->n_wells; ++k) {
        const int64_t row = nfree + P->well_face[k];
        T[nt].r = row; T[nt].c = row; T[nt].v = P->well_wi[k]; nt++;
        S->b[row] += P->well_wi[k] * P->well_pw[k] + P->well_q[k];
    }
    qsort(T, (size_t)nt, sizeof(trip), trip_cmp);
    S->row_ptr = (int64_t *)calloc((size_t)S->n + 1, sizeof(int64_t));
    S->col = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nt > 0 ? nt : 1));
    S->val = (double *)malloc(sizeof(double) * (size_t)(nt > 0 ? nt : 1));
    int64_t nnz = 0;
    for (int64_t t = 0; t < nt; ++t) {
        if (nnz > 0 && T[t].r == T[t - 1].r && T[t].c == S->col[nnz - 1]) {
            S->val[nnz - 1] += T[t].v;
        } else {
            S->col[nnz] = T[t].c;
            S->val[nnz] = T[t].v;
            S->row_ptr[T[t].r + 1]++;
            nnz++;
        }
    }
    for (int64_t i = 0; i < S->n; ++i) S->row_ptr[i + 1] += S->row_ptr[i];
    free(T);
    return 0;
}

static void spmv(const orc_system *S, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < S->n; ++i) {
        double t = 0;
        for (int64_t q = S->row_ptr[i]; q < S->row_ptr[i + 1]; ++q) t += S->val[q] * x[S->col[q]];
        y[i] = t;
    }
}

static double dot(int64_t n, const double *x, const double *y) {
    double t = 0;
    for (int64_t i = 0; i < n; ++i) t += x[i] * y[i];
    return t;
}

/* Conjugate gradients with the Jacobi (diagonal) preconditioner, x0 = 0. */
static int pcg(const orc_system *S, double *x, double rtol, int max_iter, double *relres) {
    int64_t n = S->n;
    double *r = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *z = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *p = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *q = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *dinv = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    for (int64_t i = 0; i < n; ++i) {
        double d = 0;
        for (int64_t k = S->row_ptr[i]; k < S->row_ptr[i + 1]; ++k)
            if (S->col[k] == i) d = S->val[k];
        dinv[i] = 1.0 / d;
        x[i] = 0;
        r[i] = S->b[i];
    }
    double bnorm = sqrt(dot(n, S->b, S->b));
    int it = 0;
    if (bnorm == 0.0) { *relres = 0; goto done; }
    for (int64_t i = 0; i < n; ++i) { z[i] = dinv[i] * r[i]; p[i] = z[i]; }
    double rz = dot(n, r, z);
    double rn = bnorm;
    while (rn > rtol * bnorm && it < max_iter) {
        spmv(S, p, q);
        double alpha = rz / dot(n, p, q);
        for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
        double rz2 = dot(n, r, z);
        double beta = rz2 / rz;
        rz = rz2;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rn = sqrt(dot(n, r, r));
        ++it;
    }
    /* report the true residual */
    spmv(S, x, q);
    {
        double t = 0;
        for (int64_t i = 0; i < n; ++i) t += (S->b[i] - q[i]) * (S->b[i] - q[i]);
        *relres = sqrt(t) / bnorm;
    }
done:
    free(r); free(z); free(p); free(q); free(dinv);
    return it;
}

/* ------------------------------------------------------------------------ */
/* exported entry points                                                     */
/* ------------------------------------------------------------------------ */

int64_t orc_system_size(const orc_problem *P, int64_t *n_out, int64_t *nnz_out) {
    orc_system S;
    int st = build_system(P, &S);
    if (!st) {
        *n_out = S.n;
        *nnz_out = S.row_ptr[S.n];
    }
    free_system(&S, P->n_cells);
    return st;
}

int orc_system_csr(const orc_problem *P, int64_t *row_ptr, int64_t *col, double *val, double *b) {
    orc_system S;
    int st = build_system(P, &S);
    if (!st) {
        memcpy(row_ptr, S.row_ptr, sizeof(int64_t) * (size_t)(S.n + 1));
        memcpy(col, S.col, sizeof(int64_t) * (size_t)S.row_ptr[S.n]);
        memcpy(val, S.val, sizeof(double) * (size_t)S.row_ptr[S.n]);
        memcpy(b, S.b, sizeof(double) * (size_t)S.n);
    }
    free_system(&S, P->n_cells);
    return st;
}

/*
 * Darcy solve (Algorithm paraimpdarcy on one process): assemble, eliminate the
 * cells, solve for nodes and fracture faces, then recover the cells by
 * eqschurcell and evaluate the fluxes of equations VAGFluxMatrix /
 * VAGFluxFracture.
 *
 * Outputs (caller allocated):
 *   u_node[n_nodes] (Dirichlet nodes carry p_bar), u_cell[n_cells], u_frac[n_frac]
 *   F_cell[n_cells][8]      F_{K,s} for the 8 nodes in VTK slot order
 *   F_cell_frac[n_frac][2]  F_{K,sigma} for the two cells of sigma (ascending
 *                           cell index; 0 where sigma has one cell)
 *   F_frac[n_frac][4]       F_{sigma,s} in the fracture face's node order
 *   cell_frac[n_cells][6], frac_cell[n_frac][2] (topology, may be NULL)
 */
int orc_solve_darcy(const orc_problem *P, double rtol, int max_iter, double *u_node, double *u_cell,
                    double *u_frac, double *F_cell, double *F_cell_frac, double *F_frac,
                    int *iters, double *relres) {
    orc_system S;
    int st = build_system(P, &S);
    if (st) { free_system(&S, P->n_cells); return st; }
    int64_t nn = P->n_nodes, nc = P->n_cells, nf = P->n_frac;
    int64_t nfree = S.n - nf;
    double *x = (double *)malloc(sizeof(double) * (size_t)(S.n + 1));
    *iters = pcg(&S, x, rtol, max_iter, relres);
    for (int64_t s = 0; s < nn; ++s) u_node[s] = S.node_unk[s] < 0 ? P->p_bar[s] : x[S.node_unk[s]];
    for (int64_t f = 0; f < nf; ++f) u_frac[f] = x[nfree + f];

    for (int64_t K = 0; K < nc; ++K) {
        int m = S.m[K];
        const double *a = S.a[K];
        double u[14], r[14], AKK = 0;
        int q = 8, fl[6];
        for (int i = 0; i < 8; ++i) u[i] = u_node[P->hex8[8 * K + i]];
        for (int f = 0; f < 6; ++f)
            if (S.cell_frac[6 * K + f] >= 0) { fl[q - 8] = f; u[q++] = u_frac[S.cell_frac[6 * K + f]]; }
        for (int i = 0; i < m; ++i) {
            r[i] = 0;
            for (int j = 0; j < m; ++j) r[i] += a[i * m + j];
            AKK += r[i];
        }
        /* eqschurcell with b_c = 0: u_K = (sum_nu r_nu u_nu) / A_KK */
        double t = 0;
        for (int i = 0; i < m; ++i) t += r[i] * u[i];
        double uK = t / AKK;
        u_cell[K] = uK;
        for (int i = 0; i < m; ++i) {
            double F = 0;
            for (int j = 0; j < m; ++j) F += a[i * m + j] * (uK - u[j]);
            if (i < 8) {
                F_cell[8 * K + i] = F;
            } else {
                int32_t f = S.cell_frac[6 * K + fl[i - 8]];
                int side = (S.frac_cell[2 * f] == K) ? 0 : 1;
                F_cell_frac[2 * f + side] = F;
            }
        }
    }
    for (int64_t f = 0; f < nf; ++f) {
        if (S.frac_cell[2 * f + 1] < 0) F_cell_frac[2 * f + 1] = 0.0;
        const double *A5 = S.A5 + 25 * f;
        for (int i = 0; i < 4; ++i) {
            double F = 0;
            for (int j = 0; j < 4; ++j)
                F += A5[(1 + i) * 5 + (1 + j)] * (u_frac[f] - u_node[P->frac_nodes[4 * f + j]]);
            F_frac[4 * f + i] = F;
        }
    }
    free(x);
    free_system(&S, nc);
    return 0;
}

/*
 * Residual of the system at given node and fracture-face pressures, without
 * assembling it: the conservation equations of §3.1 for the free nodes and the
 * fracture faces, written as b - A x of the cell-eliminated system (§4.2,
 * eq eqschur; faces kept as unknowns).  In each cell, u_K follows from
 * eq eqschurcell (zero cell source) and the fluxes F_{K,nu} from
 * eq VAGFluxMatrix; on each fracture face F_{sigma,s} from eq VAGFluxFracture;
 * a well adds its inflow Q = WI (p_w - u_sigma) + q to its face.
 *   res_node[s] = sum_K F_{K,s} + sum_sigma F_{sigma,s}          (free nodes)
 *   res_frac[f] = sum_K F_{K,sigma} - sum_s F_{sigma,s} + Q        (faces)
 * are the rows of b - A x.  b alone, the rows' Dirichlet columns and well
 * terms (-sum over Dirichlet nu' of the eliminated entry times p_bar, plus
 * WI p_w + q), goes to b_node / b_frac.  Dirichlet nodes get 0 in all four.
 * Inputs: u_node[n_nodes] (read at free nodes; Dirichlet nodes take p_bar),
 * u_frac[n_frac].  Returns 0, or the error of orc_topology / -3 for a cell
 * with a non-positive sub-tetrahedron.
 */
int orc_residual(const orc_problem *P, const double *u_node, const double *u_frac, double *res_node,
                 double *res_frac, double *b_node, double *b_frac) {
    int64_t nn = P->n_nodes, nc = P->n_cells, nf = P->n_frac;
    int32_t *cell_frac = (int32_t *)malloc(sizeof(int32_t) * 6 * (size_t)nc);
    int32_t *frac_cell = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(nf > 0 ? nf : 1));
    int32_t *frac_lface = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(nf > 0 ? nf : 1));
    int st = orc_topology(P, cell_frac, frac_cell, frac_lface);
    if (st) { free(cell_frac); free(frac_cell); free(frac_lface); return st; }
    for (int64_t s = 0; s < nn; ++s) res_node[s] = b_node[s] = 0.0;
    for (int64_t f = 0; f < nf; ++f) res_frac[f] = b_frac[f] = 0.0;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : bad)
    for (int64_t K = 0; K < nc; ++K) {
        double a[14 * 14];
        int m;
        if (orc_cell_matrix(P, K, cell_frac + 6 * K, a, &m, NULL) < 0) { bad = 1; continue; }
        double u[14], r[14], AKK = 0.0;
        int32_t node[14], face[14], dir[14];
        int q = 8;
        for (int i = 0; i < 8; ++i) {
            node[i] = P->hex8[8 * K + i];
            face[i] = -1;
            dir[i] = P->dirichlet[node[i]] != 0;
            u[i] = dir[i] ? P->p_bar[node[i]] : u_node[node[i]];
        }
        for (int lf = 0; lf < 6; ++lf)
            if (cell_frac[6 * K + lf] >= 0) {
                node[q] = -1;
                face[q] = cell_frac[6 * K + lf];
                dir[q] = 0;
                u[q] = u_frac[face[q]];
                ++q;
            }
        for (int i = 0; i < m; ++i) {
            r[i] = 0.0;
            for (int j = 0; j < m; ++j) r[i] += a[i * m + j];
            AKK += r[i];
        }
        double uK = 0.0;
        for (int i = 0; i < m; ++i) uK += r[i] * u[i];
        uK /= AKK;
        for (int i = 0; i < m; ++i) {
            if (dir[i]) continue;
            double F = 0.0, bD = 0.0;
            for (int j = 0; j < m; ++j) {
                F += a[i * m + j] * (uK - u[j]);
                if (dir[j]) bD -= (a[i * m + j] - r[i] * r[j] / AKK) * u[j];
            }
            double *rs = node[i] >= 0 ? res_node + node[i] : res_frac + face[i];
            double *bs = node[i] >= 0 ? b_node + node[i] : b_frac + face[i];
#pragma omp atomic
            *rs += F;
#pragma omp atomic
            *bs += bD;
        }
    }
    if (bad) { free(cell_frac); free(frac_cell); free(frac_lface); return -3; }
    for (int64_t f = 0; f < nf; ++f) {
        double A5[25];
        orc_frac_matrix(P, f, A5);
        double u[5];
        int dir[5];
        u[0] = u_frac[f];
        dir[0] = 0;
        for (int i = 0; i < 4; ++i) {
            int32_t sn = P->frac_nodes[4 * f + i];
            dir[1 + i] = P->dirichlet[sn] != 0;
            u[1 + i] = dir[1 + i] ? P->p_bar[sn] : u_node[sn];
        }
        for (int i = 0; i < 4; ++i) {
            double F = 0.0;  /* F_{sigma,s_i} */
            for (int j = 0; j < 4; ++j) F += A5[(1 + i) * 5 + 1 + j] * (u[0] - u[1 + j]);
            res_frac[f] -= F;
            if (!dir[1 + i]) res_node[P->frac_nodes[4 * f + i]] += F;
        }
        /* b: Dirichlet columns of the face's 5 x 5 block */
        for (int i = 0; i < 5; ++i) {
            if (dir[i]) continue;
            double bD = 0.0;
            for (int j = 0; j < 5; ++j)
                if (dir[j]) bD -= A5[i * 5 + j] * u[j];
            if (i == 0) b_frac[f] += bD;
            else b_node[P->frac_nodes[4 * f + i - 1]] += bD;
        }
    }
    for (int64_t k = 0; k < P->n_wells; ++k) {
        const int32_t f = P->well_face[k];
        res_frac[f] += P->well_wi[k] * (P->well_pw[k] - u_frac[f]) + P->well_q[k];
        b_frac[f] += P->well_wi[k] * P->well_pw[k] + P->well_q[k];
    }
    free(cell_frac); free(frac_cell); free(frac_lface);
    return 0;
}

/* Flow from each well into its fracture face: Q = WI (p_w - u_sigma) + q. */
int orc_well_rates(const orc_problem *P, const double *u_frac, double *Q) {
    for (int64_t k = 0; k < P->n_wells; ++k)
        Q[k] = P->well_wi[k] * (P->well_pw[k] - u_frac[P->well_face[k]]) + P->well_q[k];
    return 0;
}

/*
 * Porous volumes of the control volumes (§3.2.1).  Control volumes are the
 * cells, the fracture faces and the nodes without a Dirichlet flag; Dirichlet
 * nodes get 0.  Fracture nodes (nodes of a fracture face) take volume from the
 * fracture faces only; other nodes from the cells.  alpha_K,s = 1/16 and
 * alpha_sigma,s = 1/8 where a share is taken.
 *
 * alpha_rule 0: every adjacent cell (fracture face) gives its share.
 * alpha_rule 1: the rule of §3.2.1 for nodes between rock types: only the
 * adjacent cells (fracture faces) of largest permeability give a share, the
 * others none.  A cell's permeability is measured by the trace of its tensor
 * over 3, a fracture face's by its scalar permeability; all cells (faces)
 * that reach the largest value give their share.
 */
static double perm_measure(const double *L) { return (L[0] + L[1] + L[2]) / 3.0; }

int orc_porous_volumes(const orc_problem *P, int alpha_rule, double *phi_cell, double *phi_frac,
                       double *phi_node) {
    int64_t nn = P->n_nodes, nc = P->n_cells, nf = P->n_frac;
    const double alpha_cell = 1.0 / 16.0, alpha_frac = 1.0 / 8.0;
    uint8_t *is_frac_node = (uint8_t *)calloc((size_t)nn, 1);
    for (int64_t f = 0; f < nf; ++f)
        for (int i = 0; i < 4; ++i) is_frac_node[P->frac_nodes[4 * f + i]] = 1;
    /* largest permeability around each node: over the fracture faces at a
       fracture node, over the cells elsewhere */
    double *pmax = (double *)malloc(sizeof(double) * (size_t)(nn > 0 ? nn : 1));
    for (int64_t s = 0; s < nn; ++s) pmax[s] = -1.0;
    for (int64_t K = 0; K < nc; ++K) {
        double m = perm_measure(P->perm + 6 * K);
        for (int i = 0; i < 8; ++i) {
            int32_t s = P->hex8[8 * K + i];
            if (!is_frac_node[s] && m > pmax[s]) pmax[s] = m;
        }
    }
    for (int64_t f = 0; f < nf; ++f)
        for (int i = 0; i < 4; ++i) {
            int32_t s = P->frac_nodes[4 * f + i];
            if (P->frac_perm[f] > pmax[s]) pmax[s] = P->frac_perm[f];
        }
    for (int64_t s = 0; s < nn; ++s) phi_node[s] = 0.0;
    int32_t z6[6] = {-1, -1, -1, -1, -1, -1};
    for (int64_t K = 0; K < nc; ++K) {
        double a[14 * 14];
        int m;
        double vol = orc_cell_matrix(P, K, z6, a, &m, NULL);
        if (vol < 0) { free(is_frac_node); free(pmax); return -3; }
        double pore = vol * P->poro[K];
        double perm = perm_measure(P->perm + 6 * K);
        double sum_alpha = 0;
        for (int i = 0; i < 8; ++i) {
            int32_t s = P->hex8[8 * K + i];
            if (P->dirichlet[s] || is_frac_node[s]) continue;
            if (alpha_rule == 1 && perm < pmax[s]) continue;
            sum_alpha += alpha_cell;
            phi_node[s] += alpha_cell * pore;
        }
        phi_cell[K] = (1.0 - sum_alpha) * pore;
    }
    for (int64_t f = 0; f < nf; ++f) {
        double A5[25];
        double area = orc_frac_matrix(P, f, A5);
        double pore = P->frac_width[f] * area * P->frac_poro[f];
        double sum_alpha = 0;
        for (int i = 0; i < 4; ++i) {
            int32_t s = P->frac_nodes[4 * f + i];
            if (P->dirichlet[s]) continue;
            if (alpha_rule == 1 && P->frac_perm[f] < pmax[s]) continue;
            sum_alpha += alpha_frac;
            phi_node[s] += alpha_frac * pore;
        }
        phi_frac[f] = (1.0 - sum_alpha) * pore;
    }
    free(is_frac_node);
    free(pmax);
    return 0;
}

static double pos(double a) { return a > 0 ? a : 0.0; }
static double neg(double a) { return a < 0 ? a : 0.0; }

/*
 * CFL bound of equation eq_CFL: min over the cells, the fracture faces and the
 * free nodes of the porous volume over the sum of outgoing fluxes.  A control
 * volume without outflow contributes +infinity.  Returns the three partial
 * minima; the time step is cfl * min of them.
 */
int orc_cfl(const orc_problem *P, const double *F_cell, const double *F_cell_frac,
            const double *F_frac, const double *well_rate, const double *phi_cell,
            const double *phi_frac, const double *phi_node, double *dt3) {
    int64_t nn = P->n_nodes, nc = P->n_cells, nf = P->n_frac;
    int32_t *cell_frac = (int32_t *)malloc(sizeof(int32_t) * 6 * (size_t)nc);
    int32_t *frac_cell = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(nf > 0 ? nf : 1));
    int32_t *frac_lface = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(nf > 0 ? nf : 1));
    int st = orc_topology(P, cell_frac, frac_cell, frac_lface);
    if (st) { free(cell_frac); free(frac_cell); free(frac_lface); return st; }
    double *out_node = (double *)calloc((size_t)nn, sizeof(double));
    /* a producing well takes fluid out of its face */
    double *out_well = (double *)calloc((size_t)(nf > 0 ? nf : 1), sizeof(double));
    for (int64_t k = 0; well_rate && k < P->n_wells; ++k) out_well[P->well_face[k]] += pos(-well_rate[k]);
    double dtM = INFINITY, dtF = INFINITY, dtV = INFINITY;
    for (int64_t K = 0; K < nc; ++K) {
        double out = 0;
        for (int i = 0; i < 8; ++i) {
            out += pos(F_cell[8 * K + i]);
            out_node[P->hex8[8 * K + i]] += pos(-F_cell[8 * K + i]);
        }
        for (int lf = 0; lf < 6; ++lf) {
            int32_t f = cell_frac[6 * K + lf];
            if (f < 0) continue;
            int side = frac_cell[2 * f] == K ? 0 : 1;
            out += pos(F_cell_frac[2 * f + side]);
        }
        if (out > 0) dtM = fmin(dtM, phi_cell[K] / out);
    }
    for (int64_t f = 0; f < nf; ++f) {
        double out = 0;
        for (int i = 0; i < 4; ++i) {
            out += pos(F_frac[4 * f + i]);
            out_node[P->frac_nodes[4 * f + i]] += pos(-F_frac[4 * f + i]);
        }
        for (int side = 0; side < 2; ++side)
            if (frac_cell[2 * f + side] >= 0) out += pos(-F_cell_frac[2 * f + side]);
        out += out_well[f];
        if (out > 0) dtF = fmin(dtF, phi_frac[f] / out);
    }
    for (int64_t s = 0; s < nn; ++s)
        if (!P->dirichlet[s] && out_node[s] > 0) dtV = fmin(dtV, phi_node[s] / out_node[s]);
    dt3[0] = dtM; dt3[1] = dtF; dt3[2] = dtV;
    free(out_well);
    free(out_node); free(cell_frac); free(frac_cell); free(frac_lface);
    return 0;
}

/*
 * Explicit Euler upwind transport (§3.2.2, equations darcyfluxH and the
 * discrete conservation laws of each control volume), n_steps steps of size
 * dt; when last_dt > 0 the final step uses last_dt instead (§4.3, step 2).
 * c_cell / c_frac / c_node hold c^0 on entry and c^N on exit; Dirichlet nodes
 * are set to c_bar.
 *   H_{K,nu}     = c_K F_{K,nu}^+ + c_nu F_{K,nu}^-
 *   H_{sigma,s}  = c_sigma F_{sigma,s}^+ + c_s F_{sigma,s}^-
 *   cell:   phi_K (c_K^{n+1} - c_K^n)/dt + sum_nu H_{K,nu} = 0
 *   face:   phi_s (c^{n+1} - c^n)/dt + sum_s H_{sigma,s} - sum_K H_{K,sigma} = 0
 *   node:   phi_s (c^{n+1} - c^n)/dt - sum_K H_{K,s} - sum_sigma H_{sigma,s} = 0
 * A well perforating face sigma with inflow Q adds
 *   H_w = c_sigma max(-Q, 0) - c_inj max(Q, 0)
 * to the face's sum: production leaves at the face's concentration,
 * injection enters at c_inj.
 */
int orc_transport(const orc_problem *P, const double *F_cell, const double *F_cell_frac,
                  const double *F_frac, const double *well_rate, const double *phi_cell,
                  const double *phi_frac, const double *phi_node, double dt, int64_t n_steps,
                  double last_dt, double *c_cell, double *c_frac, double *c_node) {
    int64_t nn = P->n_nodes, nc = P->n_cells, nf = P->n_frac;
    int32_t *cell_frac = (int32_t *)malloc(sizeof(int32_t) * 6 * (size_t)nc);
    int32_t *frac_cell = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(nf > 0 ? nf : 1));
    int32_t *frac_lface = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(nf > 0 ? nf : 1));
    int st = orc_topology(P, cell_frac, frac_cell, frac_lface);
    if (st) { free(cell_frac); free(frac_cell); free(frac_lface); return st; }
    double *sK = (double *)malloc(sizeof(double) * (size_t)nc);
    double *sF = (double *)malloc(sizeof(double) * (size_t)(nf > 0 ? nf : 1));
    double *sV = (double *)malloc(sizeof(double) * (size_t)nn);
    for (int64_t s = 0; s < nn; ++s)
        if (P->dirichlet[s]) c_node[s] = P->c_bar[s];
    for (int64_t n = 0; n < n_steps; ++n) {
        double h = (n == n_steps - 1 && last_dt > 0) ? last_dt : dt;
        for (int64_t K = 0; K < nc; ++K) sK[K] = 0;
        for (int64_t f = 0; f < nf; ++f) sF[f] = 0;
        for (int64_t s = 0; s < nn; ++s) sV[s] = 0;
        for (int64_t K = 0; K < nc; ++K) {
            for (int i = 0; i < 8; ++i) {
                int32_t s = P->hex8[8 * K + i];
                double F = F_cell[8 * K + i];
                double H = c_cell[K] * pos(F) + c_node[s] * neg(F);
                sK[K] += H;
                sV[s] -= H;
            }
            for (int lf = 0; lf < 6; ++lf) {
                int32_t f = cell_frac[6 * K + lf];
                if (f < 0) continue;
                int side = frac_cell[2 * f] == K ? 0 : 1;
                double F = F_cell_frac[2 * f + side];
                double H = c_cell[K] * pos(F) + c_frac[f] * neg(F);
                sK[K] += H;
                sF[f] -= H;
            }
        }
        for (int64_t f = 0; f < nf; ++f)
            for (int i = 0; i < 4; ++i) {
                int32_t s = P->frac_nodes[4 * f + i];
                double F = F_frac[4 * f + i];
                double H = c_frac[f] * pos(F) + c_node[s] * neg(F);
                sF[f] += H;
                sV[s] -= H;
            }
        for (int64_t k = 0; well_rate && k < P->n_wells; ++k) {
            const int32_t f = P->well_face[k];
            sF[f] += c_frac[f] * pos(-well_rate[k]) - P->well_cinj[k] * pos(well_rate[k]);
        }
        for (int64_t K = 0; K < nc; ++K) c_cell[K] -= h / phi_cell[K] * sK[K];
        for (int64_t f = 0; f < nf; ++f) c_frac[f] -= h / phi_frac[f] * sF[f];
        for (int64_t s = 0; s < nn; ++s)
            if (!P->dirichlet[s]) c_node[s] -= h / phi_node[s] * sV[s];
    }
    free(sK); free(sF); free(sV); free(cell_frac); free(frac_cell); free(frac_lface);
    return 0;
}
