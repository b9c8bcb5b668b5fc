/*
 * FP64 CPU oracle for the hybrid-dimensional VAG scheme — TEST INFRASTRUCTURE.
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
 * it.  It shares no code with the GPU library.
 */
#ifndef VAG_ORACLE_H
#define VAG_ORACLE_H
#include <stdint.h>

typedef struct {
    int64_t n_nodes, n_cells, n_frac;
    const double *xyz;          /* [n_nodes][3] */
    const int32_t *hex8;        /* [n_cells][8] VTK order */
    const int32_t *frac_nodes;  /* [n_frac][4] cyclic */
    const double *frac_width;   /* [n_frac] d_f */
    const double *frac_perm;    /* [n_frac] Lambda_f */
    const double *frac_poro;    /* [n_frac] phi_f */
    const double *perm;         /* [n_cells][6] xx yy zz xy xz yz */
    const double *poro;         /* [n_cells] phi_m */
    double mu;
    const uint8_t *dirichlet;   /* [n_nodes] */
    const double *p_bar;        /* [n_nodes] */
    const double *c_bar;        /* [n_nodes] */
    /* Peaceman wells perforating fracture faces (§5.5): the flow from the well
     * into face sigma is Q = WI (p_w - u_sigma) + q, the injected fluid carries
     * concentration c_inj.  Each face is perforated at most once. */
    int64_t n_wells;
    const int32_t *well_face;   /* [n_wells] fracture face index */
    const double *well_wi;      /* [n_wells] well index WI (0: rate only) */
    const double *well_pw;      /* [n_wells] well pressure p_w */
    const double *well_q;       /* [n_wells] imposed rate q (injection > 0) */
    const double *well_cinj;    /* [n_wells] concentration of injected fluid */
} orc_problem;

int orc_topology(const orc_problem *P, int32_t *cell_frac, int32_t *frac_cell, int32_t *frac_lface);
double orc_cell_matrix(const orc_problem *P, int64_t K, const int32_t *cell_frac6, double *a,
                       int *m_out, double *full15);
double orc_frac_matrix(const orc_problem *P, int64_t f, double *A5);
int64_t orc_system_size(const orc_problem *P, int64_t *n_out, int64_t *nnz_out);
int orc_system_csr(const orc_problem *P, int64_t *row_ptr, int64_t *col, double *val, double *b);
int orc_solve_darcy(const orc_problem *P, double rtol, int max_iter, double *u_node, double *u_cell,
                    double *u_frac, double *F_cell, double *F_cell_frac, double *F_frac,
                    int *iters, double *relres);
int orc_residual(const orc_problem *P, const double *u_node, const double *u_frac, double *res_node,
                 double *res_frac, double *b_node, double *b_frac);
int orc_porous_volumes(const orc_problem *P, int alpha_rule, double *phi_cell, double *phi_frac,
                       double *phi_node);
int orc_well_rates(const orc_problem *P, const double *u_frac, double *Q);
int orc_cfl(const orc_problem *P, const double *F_cell, const double *F_cell_frac,
            const double *F_frac, const double *well_rate, const double *phi_cell,
            const double *phi_frac, const double *phi_node, double *dt3);
int orc_transport(const orc_problem *P, const double *F_cell, const double *F_cell_frac,
                  const double *F_frac, const double *well_rate, const double *phi_cell,
                  const double *phi_frac, const double *phi_node, double dt, int64_t n_steps,
                  double last_dt, double *c_cell, double *c_frac, double *c_node);
#endif
