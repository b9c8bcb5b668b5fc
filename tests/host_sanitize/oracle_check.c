/*
 * Drives the C oracle (test infrastructure) through a whole run -- system,
 * Jacobi-PCG solve, residual, porous volumes (both volume rules), CFL bounds
 * and transport -- on a problem read from a file, for a build with the
 * address and undefined-behaviour sanitizers.  File layout (little endian):
 * int64 n_nodes, n_cells, n_frac, n_wells, n_steps; double mu, rtol; then
 * xyz, hex8, frac_nodes, frac_width, frac_perm, frac_poro, perm, poro,
 * dirichlet (uint8), p_bar, c_bar, well_face, well_wi, well_pw, well_q,
 * well_cinj.
 */
#include <stdio.h>
#include <stdlib.h>

#include "vag_oracle.h"

static void *rd(FILE *f, size_t size, int64_t n) {
    void *p = malloc(size * (size_t)(n > 0 ? n : 1));
    if (n > 0 && fread(p, size, (size_t)n, f) != (size_t)n) {
        fprintf(stderr, "short read\n");
        exit(3);
    }
    return p;
}

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t hdr[5];
    double dh[2];
    if (fread(hdr, 8, 5, f) != 5 || fread(dh, 8, 2, f) != 2) return 3;
    orc_problem P;
    const int64_t nn = hdr[0], nc = hdr[1], nf = hdr[2], nw = hdr[3], steps = hdr[4];
    P.n_nodes = nn;
    P.n_cells = nc;
    P.n_frac = nf;
    P.n_wells = nw;
    P.mu = dh[0];
    P.xyz = rd(f, 8, 3 * nn);
    P.hex8 = rd(f, 4, 8 * nc);
    P.frac_nodes = rd(f, 4, 4 * nf);
    P.frac_width = rd(f, 8, nf);
    P.frac_perm = rd(f, 8, nf);
    P.frac_poro = rd(f, 8, nf);
    P.perm = rd(f, 8, 6 * nc);
    P.poro = rd(f, 8, nc);
    P.dirichlet = rd(f, 1, nn);
    P.p_bar = rd(f, 8, nn);
    P.c_bar = rd(f, 8, nn);
    P.well_face = rd(f, 4, nw);
    P.well_wi = rd(f, 8, nw);
    P.well_pw = rd(f, 8, nw);
    P.well_q = rd(f, 8, nw);
    P.well_cinj = rd(f, 8, nw);
    fclose(f);

    int64_t n = 0, nnz = 0;
    if (orc_system_size(&P, &n, &nnz) != 0) return 6;
    int64_t *rp = malloc(8 * (size_t)(n + 1)), *col = malloc(8 * (size_t)nnz);
    double *val = malloc(8 * (size_t)nnz), *b = malloc(8 * (size_t)n);
    if (orc_system_csr(&P, rp, col, val, b)) return 7;
    double *un = calloc((size_t)nn, 8), *uc = calloc((size_t)nc, 8), *uf = calloc((size_t)(nf + 1), 8);
    double *Fc = calloc((size_t)(8 * nc), 8), *Fcf = calloc((size_t)(2 * nf + 2), 8), *Ff = calloc((size_t)(4 * nf + 4), 8);
    int iters = 0;
    double relres = 0;
    if (orc_solve_darcy(&P, dh[1], 100000, un, uc, uf, Fc, Fcf, Ff, &iters, &relres)) return 8;
    double *rn = calloc((size_t)nn, 8), *rf = calloc((size_t)(nf + 1), 8), *bn = calloc((size_t)nn, 8),
           *bf = calloc((size_t)(nf + 1), 8);
    if (orc_residual(&P, un, uf, rn, rf, bn, bf)) return 9;
    double *Q = calloc((size_t)(nw + 1), 8);
    if (nw && orc_well_rates(&P, uf, Q)) return 10;
    double *pc = calloc((size_t)nc, 8), *pf = calloc((size_t)(nf + 1), 8), *pn = calloc((size_t)nn, 8);
    for (int rule = 1; rule >= 0; --rule)
        if (orc_porous_volumes(&P, rule, pc, pf, pn)) return 11;
    double dt3[3];
    if (orc_cfl(&P, Fc, Fcf, Ff, nw ? Q : NULL, pc, pf, pn, dt3)) return 12;
    double dt = dt3[0];
    for (int k = 1; k < 3; ++k)
        if (dt3[k] < dt) dt = dt3[k];
    double *cc = calloc((size_t)nc, 8), *cf = calloc((size_t)(nf + 1), 8), *cn = calloc((size_t)nn, 8);
    if (orc_transport(&P, Fc, Fcf, Ff, nw ? Q : NULL, pc, pf, pn, 0.9 * dt, steps, 0.0, cc, cf, cn)) return 13;
    double sum = 0;
    for (int64_t i = 0; i < nc; ++i) sum += cc[i];
    printf("oracle: %lld unknowns, %lld nonzeros, %d iterations, residual %.2e, dt %.3e, sum c %.6f\n",
           (long long)n, (long long)nnz, iters, relres, dt, sum);
    free(rp); free(col); free(val); free(b); free(un); free(uc); free(uf); free(Fc); free(Fcf); free(Ff);
    free(rn); free(rf); free(bn); free(bf); free(Q); free(pc); free(pf); free(pn); free(cc); free(cf); free(cn);
    free((void *)P.xyz); free((void *)P.hex8); free((void *)P.frac_nodes); free((void *)P.frac_width);
    free((void *)P.frac_perm); free((void *)P.frac_poro); free((void *)P.perm); free((void *)P.poro);
    free((void *)P.dirichlet); free((void *)P.p_bar); free((void *)P.c_bar); free((void *)P.well_face);
    free((void *)P.well_wi); free((void *)P.well_pw); free((void *)P.well_q); free((void *)P.well_cinj);
    return 0;
}
