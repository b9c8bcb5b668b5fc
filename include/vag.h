/*
 * libvag — hybrid-dimensional Vertex Approximate Gradient (VAG) Darcy flow and
 * explicit upwind transport in fractured porous media, on one AMD Instinct
 * MI355X (gfx950).
 *
 * The problem statement follows Xing, Masson, Lopez, "Parallel Vertex
 * Approximate Gradient discretization of hybrid dimensional Darcy flow and
 * transport in discrete fracture networks" (arXiv:1602.03641):
 *   - mesh D and conforming fracture faces F_Gamma ........ §3.1
 *   - Darcy unknowns u_K, u_s, u_sigma and the VAG fluxes .. §3.1, eqs VAGFluxMatrix,
 *                                                          VAGFluxFracture
 *   - cell elimination (Schur complement) .................. §4.2, eqs sysowndarcy,
 *                                                          eqschur, eqschurcell
 *   - control volumes and porous volumes ................... §3.2.1
 *   - explicit upwind steps and the CFL bound .............. §3.2.2, eqs darcyfluxH,
 *                                                          eq_CFL; §4.3
 *   - Krylov methods and preconditioners (CG, GMRES,
 *     BiCGStab; aggregation and classical AMG, block
 *     Jacobi ILU(0)) ....................................... §5.3
 *   - Peaceman wells on fracture faces .................... §5.5
 *
 * Conventions
 *   - All entry points are extern "C", take plain pointers and sizes, and never
 *     throw or abort: they return a vag_status (negative = error,
 *     VAG_WARN_NOT_CONVERGED = best iterate returned).  vag_last_error() gives
 *     the text of the last error of a handle (with the offending index where
 *     one exists).
 *   - Array arguments are caller-owned.  Input arrays are read during the call
 *     only (the library copies what it keeps).  Output arrays are written by the
 *     call.  A vag_mem argument says whether the pointers are host or device
 *     (HIP) memory; the same space applies to every array of the call.
 *   - A handle binds one HIP stream (the one given at creation, or the null
 *     stream).  All device work of the handle is queued on it.  Calls that
 *     return host data synchronise that stream.  A handle is not thread-safe;
 *     distinct handles are independent.
 *   - Index types are int32 (cells, nodes, fracture faces < 2^31); the
 *     assembled nodal system must have fewer than 2^31 nonzeros.
 */
#ifndef VAG_H
#define VAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VAG_OK = 0,
    VAG_WARN_NOT_CONVERGED = 1,
    VAG_ERR_ARG = -1,          /* invalid argument or inconsistent input */
    VAG_ERR_MESH = -2,         /* invalid mesh: non-positive sub-tetrahedron, unknown fracture face */
    VAG_ERR_UNSUPPORTED = -3,  /* valid request that the library does not support */
    VAG_ERR_OOM = -4,          /* device allocation failed */
    VAG_ERR_HIP = -5,          /* HIP runtime error */
    VAG_ERR_STATE = -6,        /* call out of order (e.g. transport before a pressure solve) */
    VAG_ERR_TIMEOUT = -7,      /* vag_server_wait: the job has not finished in time */
    VAG_ERR_CANCELLED = -8     /* the job was cancelled before it started */
} vag_status;

typedef enum { VAG_MEM_HOST = 0, VAG_MEM_DEVICE = 1 } vag_mem;

/* VAG_MIXED: the AMG hierarchy (every level's matrix) is stored and applied in
 * FP32 while the Krylov vectors, the system matrix products and residuals stay
 * FP64.  VAG_MIXED_IR: FP64 iterative refinement (residual b - A x and update
 * in FP64) around an FP32 CG or GMRES on the FP32 copy of A, preconditioned
 * by the FP32 hierarchy.  Assembly, elimination, fluxes and transport are
 * FP64 in every mode. */
typedef enum { VAG_FP64 = 0, VAG_MIXED = 1, VAG_MIXED_IR = 2 } vag_precision;
/* Krylov method for the eliminated system (§5.3 compares CG, GMRES and
 * BiCGStab): VAG_CG (the system is SPD), VAG_GMRES (restarted flexible GMRES(m), CGS2),
 * VAG_BICGSTAB (right-preconditioned BiCGStab, FP64 vectors; not with
 * VAG_MIXED_IR). */
typedef enum { VAG_CG = 0, VAG_GMRES = 1, VAG_BICGSTAB = 2 } vag_krylov;
/* Preconditioners (§5.3 compares algebraic multigrid and block Jacobi
 * ILU(0)): VAG_PC_JACOBI (diagonal), VAG_PC_AMG (aggregation AMG),
 * VAG_PC_BJILU0 (block Jacobi with an ILU(0) factor per block of
 * ilu_block_rows consecutive unknowns of the natural order, eliminated in that
 * order; not symmetric, so GMRES or BiCGStab only, FP64 only). */
typedef enum { VAG_PC_JACOBI = 0, VAG_PC_AMG = 1, VAG_PC_BJILU0 = 2 } vag_precond;

/*
 * Generalised polyhedral mesh (§3.1), in one of two forms.
 *
 * hex8 != NULL (the fast path): hexahedra, each listing its 8 nodes in VTK
 * order (bottom quad counter-clockwise seen from above, then the top quad);
 * faces may be non-planar.  Every one of the 24 sub-tetrahedra (x_K, x_sigma,
 * edge) must have positive volume.
 *
 * hex8 == NULL: general cells given by their faces.  cell_faces lists the
 * faces of each cell (CSR by cell_face_ptr, 4 to 6 faces), face_nodes the
 * nodes of each face in cyclic order (CSR by face_node_ptr, 3 or 4 nodes;
 * consecutive nodes are the face's edges); a face is shared by at most two
 * cells and may be listed in either orientation.  A cell has 4 to 8 nodes,
 * the union of its faces' nodes; its local node order is the order in which
 * they first appear along its faces (cell_faces order, each face's node
 * order).  This covers the tetrahedra, pyramids, prisms and hexahedra of the
 * paper's experiments (§5.4, §5.5).  On every face the k sub-tetrahedra
 * (x_K, x_sigma, s_e, s_e+1) must have volumes of one sign and none zero (a
 * cell star-shaped with respect to its centre).  Fracture-face groups are
 * never eliminated on this path (the faces stay unknowns), and
 * vag_transport_noalloc returns VAG_ERR_UNSUPPORTED.
 *
 * In both forms the cell centre is the mean of the cell's nodes and a face
 * centre the mean of the face's nodes (beta = 1/|V_sigma|).
 */
typedef struct {
    int64_t n_nodes;
    int64_t n_cells;
    const double *node_xyz;  /* [n_nodes][3] */
    const int32_t *hex8;     /* [n_cells][8], or NULL for the general form */
    /* general form (read when hex8 is NULL) */
    int64_t n_faces;
    const int64_t *cell_face_ptr;  /* [n_cells + 1] */
    const int32_t *cell_faces;     /* [cell_face_ptr[n_cells]] face indices */
    const int64_t *face_node_ptr;  /* [n_faces + 1] */
    const int32_t *face_nodes;     /* [face_node_ptr[n_faces]] node indices, cyclic per face */
} vag_mesh;

/*
 * Fracture faces F_Gamma (§3.1: the fracture network is a union of mesh faces),
 * each listed once.  With a hex8 mesh each is given by its 4 nodes in cyclic
 * order (face_nodes) and must be a face of one or two cells; with the general
 * form by its index in the mesh's face list (face_ids).  width = d_f, perm =
 * Lambda_f (isotropic in the plane), porosity = phi_f, each per fracture face.
 */
typedef struct {
    int64_t n_frac;
    const int32_t *face_nodes;  /* [n_frac][4], hex8 meshes */
    const double *width;        /* [n_frac] */
    const double *perm;         /* [n_frac] */
    const double *porosity;     /* [n_frac] */
    const int32_t *face_ids;    /* [n_frac], general meshes: indices into the mesh's faces */
} vag_fractures;

/* Matrix rock: symmetric positive definite Lambda_m per cell packed
 * [xx, yy, zz, xy, xz, yz] (checked at each vag_solve_pressure), porosity
 * phi_m per cell, constant viscosity mu. */
typedef struct {
    const double *perm;      /* [n_cells][6] */
    const double *porosity;  /* [n_cells] */
    double mu;
} vag_rock;

/*
 * Boundary data.  A node with node_dirichlet = 1 has pressure p_bar and, in the
 * transport, the fixed concentration c_bar (§3.1 last equation, §3.2.2).
 * Every other node carries the conservation equation of an interior node
 * (homogeneous Neumann where it lies on the boundary).  At least one node must
 * be Dirichlet.
 */
typedef struct {
    const uint8_t *node_dirichlet;  /* [n_nodes] 0/1 */
    const double *p_bar;            /* [n_nodes], read where flagged */
    const double *c_bar;            /* [n_nodes], read where flagged */
} vag_bc;

typedef struct {
    int precision;          /* vag_precision */
    int krylov;             /* vag_krylov */
    int precond;            /* vag_precond */
    double rtol;            /* stop when ||b - A x||_2 <= rtol ||b||_2, x0 = 0 */
    double inner_rtol;      /* VAG_MIXED: relative tolerance of each FP32 inner solve */
    int max_iter;           /* Krylov iterations (VAG_MIXED: inner iterations in total) */
    int gmres_restart;      /* GMRES basis size */
    int check_every;        /* iterations queued between host convergence checks */
    double cfl;             /* transport step = cfl * CFL bound (eq_CFL) */
    int amg_coarse_size;    /* stop coarsening below this many unknowns */
    int amg_max_levels;
    double amg_theta;       /* strength threshold |a_ij| >= theta sqrt(a_ii a_jj) */
    int amg_sweeps;         /* l1-Jacobi sweeps before and after the coarse correction on
                               the coarse levels (the finest level has one of each); default 1 */
    int eliminate_frac_faces;  /* 1: eliminate fracture-face groups onto the nodes
                                  (fixed at vag_create); 0: faces stay unknowns */
    int amg_aggregate_hops; /* radius of the aggregates: roots form a distance-2 (2, the
                               default) or distance-1 (1: smaller aggregates, more levels)
                               independent set of the strength graph; 0 = default */
    int amg_kcycle;         /* coarse levels 1..amg_kcycle (not the coarsest) take a K-cycle:
                               two flexible CG steps preconditioned by the V-cycle below, the
                               outer CG then in its flexible form (CG and flexible GMRES, not
                               with VAG_MIXED_IR; 0: V-cycles; default 2) */
    int ilu_block_rows;     /* VAG_PC_BJILU0: unknowns per block, 1..8192 (0: 128); blocks are
                               runs of the natural unknown order (vag_get_system's) */
    int amg_kind;           /* VAG_PC_AMG: 0 aggregation (default); 1 classical (strength
                               -a_ij >= amg_strong_theta max_k -a_ik, PMIS coarse points, direct
                               interpolation, Galerkin R A P; V-cycles, amg_kcycle ignored) */
    double amg_strong_theta;/* classical strength threshold in (0, 1); 0: 0.25 */
    int stream_loads;       /* row loops of the system matrix and the FP32 hierarchy read the
                               matrix entries with non-temporal loads: 0 for matrices above
                               128 MB (default), 1 always, 2 never; results are the same */
    int alpha_rule;         /* volume fractions of the node control volumes (§3.2.1):
                               0 (default): every adjacent cell gives a matrix node
                               alpha_K,s = 1/(2|V_K|) of its pore volume and every adjacent
                               fracture face gives a fracture node alpha_sigma,s = 1/(2|V_sigma|);
                               1: the rule for nodes between rock types, only the adjacent
                               cells (fracture faces) of largest permeability around the node
                               give their share, the others none (a cell's permeability: the
                               trace of its tensor over 3; ties all give) */
} vag_options;

typedef struct {
    int iterations;         /* Krylov iterations (total inner iterations in VAG_MIXED) */
    int outer_iterations;   /* refinement steps (VAG_MIXED), else 1 */
    double rel_residual;    /* final ||b - A x|| / ||b||, computed in FP64 */
    int64_t n_unknowns;     /* size of the nodal (+ fracture-face) system */
    int64_t nnz;
    int amg_levels;
    double amg_operator_complexity;
    double ms_assembly, ms_setup, ms_solve, ms_fluxes;  /* HIP-event times */
} vag_solve_info;

typedef struct {
    int64_t n_steps;        /* steps taken */
    double dt;              /* time step of the first n_steps-1 steps */
    double last_dt;         /* time step of the last step */
    double dt_bounds[3];    /* CFL minima over cells, fracture faces, nodes */
    double ms_setup, ms_steps;
    int64_t n_rows;         /* control volumes: cells + fracture faces + nodes */
    int64_t t_nnz;          /* off-diagonal entries of the upwind operator */
    int64_t t_stored;       /* stored entries including slice padding */
} vag_transport_info;

/* Kernels that vag_benchmark_kernel can time. */
typedef enum {
    VAG_KERNEL_SPMV = 0,            /* y = A x with the assembled system (Krylov operator) */
    VAG_KERNEL_TRANSPORT_STEP = 1,  /* one explicit upwind step */
    VAG_KERNEL_LOCAL = 2,           /* per-cell local VAG matrices */
    VAG_KERNEL_PRECOND = 3          /* one application of the preconditioner */
} vag_kernel;

typedef struct vag_handle vag_handle;

/* Library version string. */
const char *vag_version(void);

/* Fills *opt with defaults: FP64, CG, Jacobi, rtol 1e-8, cfl 0.9, fracture-face
 * groups eliminated. */
vag_status vag_default_options(vag_options *opt);

/*
 * Creates a handle: validates the mesh, matches fracture faces to cell faces,
 * numbers the unknowns (free nodes, then fracture faces), builds the sparsity
 * pattern of the cell-eliminated system (eq eqschur) with the slot of every
 * local-matrix entry in it (each row of the system is then gathered by one
 * thread, in a fixed order) and the node adjacency used by transport, and
 * copies all data to the device.  hip_stream may be NULL (null stream).
 * With opt->eliminate_frac_faces, the fracture faces are grouped by shared
 * cells (after the cell elimination the face-face block is block diagonal
 * over these groups) and every group of at most 32 faces whose cells have at
 * most 64 free nodes is eliminated exactly onto those nodes: the system then
 * holds the free nodes and the remaining faces only, with the extra node-node
 * couplings this creates; the eliminated face pressures are recovered after
 * the solve.  The solution is the same as with the faces kept.
 * Errors: VAG_ERR_ARG (null/size problems, fracture face listed twice, no
 * Dirichlet node), VAG_ERR_MESH (fracture face that is not a mesh face, face
 * with more than two cells, cell with a non-positive sub-tetrahedron —
 * detected at the first solve), VAG_ERR_OOM, VAG_ERR_HIP.
 */
vag_status vag_create(const vag_mesh *mesh, const vag_fractures *frac, const vag_rock *rock,
                      const vag_bc *bc, const vag_options *opt, vag_mem inputs_mem,
                      void *hip_stream, vag_handle **out);

/*
 * Replaces the numeric data (permeabilities, porosities, fracture widths,
 * boundary values) of a handle without touching its topology; NULL pointers
 * keep the current values.  Takes effect at the next vag_solve_pressure.
 */
vag_status vag_update(vag_handle *h, const vag_rock *rock, const vag_fractures *frac_props,
                      const double *p_bar, const double *c_bar, vag_mem mem);

/* Binds the handle to another HIP stream (NULL: the null stream).  Waits for
 * the work already queued on the old stream first. */
vag_status vag_set_stream(vag_handle *h, void *hip_stream);

/* Replaces the solver options of a handle (takes effect at the next solve). */
vag_status vag_set_options(vag_handle *h, const vag_options *opt);

/*
 * Darcy solve, Algorithm paraimpdarcy on one device: per-cell VAG matrices
 * (eq VAGFluxMatrix) and fracture matrices (eq VAGFluxFracture), elimination of
 * the cell unknowns (eq eqschur), Dirichlet columns to the right-hand side,
 * preconditioned Krylov solve, cell recovery (eq eqschurcell), then the fluxes
 * F_{K,nu} and F_{sigma,s} kept on the device for transport.
 * Returns VAG_WARN_NOT_CONVERGED with the last iterate if rtol is not reached;
 * VAG_ERR_ARG, before any solving, naming the first cell whose permeability
 * tensor is not symmetric positive definite (leading minors positive, entries
 * finite) or the first fracture face without positive width and permeability;
 * VAG_ERR_MESH naming a cell with a non-positive sub-tetrahedron.
 */
vag_status vag_solve_pressure(vag_handle *h, vag_solve_info *info);

/*
 * Explicit upwind transport (§3.2.2, eq darcyfluxH; §4.3): porous volumes of
 * the control volumes, time step dt = cfl * CFL bound (eq eq_CFL), then steps.
 * With t_final > 0: N = ceil(t_final/dt) steps, the last one t_final-(N-1) dt;
 * otherwise n_steps steps of dt.  The initial state is c0 (cell, fracture-face,
 * node arrays; NULL = continue from the current state, which is 0 after a
 * solve); Dirichlet nodes are held at c_bar.
 */
vag_status vag_transport(vag_handle *h, int64_t n_steps, double t_final, const double *c0_cell,
                         const double *c0_frac, const double *c0_node, vag_mem mem,
                         vag_transport_info *info);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * transport of vag_transport (time step dt = cfl * CFL bound, then n_steps
 * explicit upwind steps, or t_final as there) without the upwind operator that
 * vag_transport builds in memory it allocates.  Each step gathers the upwind
 * fluxes of every control volume from the handle's resident Darcy fluxes.
 * The call allocates nothing: the CFL reduction's partial minima and the time
 * step live in a static device array of the library (3 * 512 + 8 doubles,
 * about 12 KB, one copy per device, held until the process ends), the
 * concentration double buffer is the handle's own (from vag_create).
 *   c0_cell[n_cells], c0_frac[n_frac], c0_node[n_nodes]: initial state in
 *       device memory, read only; all NULL = continue from the handle's state
 *       (zero after a solve).  Dirichlet nodes are held at c_bar.
 *   c_cell, c_frac, c_node: the state after the steps, device memory,
 *       caller-owned, same sizes; any may be NULL.  The handle's concentration
 *       state (vag_get_concentration, a later transport call) is the result
 *       too.
 *   info: NULL, or filled as by vag_transport (t_nnz = t_stored = 0).  With
 *       info or t_final > 0 the call reads dt on the host and synchronises the
 *       handle's stream; otherwise it only queues work on that stream.
 * The result equals vag_transport's up to the order of the additions inside
 * each step.  Every call on a device shares that device's array and the
 * array keeps the last call's contents (each call writes every value it
 * reads before reading it), so calls whose work overlaps on one device
 * (handles on different streams or threads) race: serialise them.
 * Errors: as vag_transport; VAG_ERR_ARG if the reduction's scratch would
 * exceed the array.
 */
vag_status vag_transport_noalloc(vag_handle *h, int64_t n_steps, double t_final, const double *c0_cell,
                                 const double *c0_frac, const double *c0_node, double *c_cell, double *c_frac,
                                 double *c_node, vag_transport_info *info);

/*
 * Transport on given Darcy fluxes (layout of vag_get_fluxes) instead of those
 * of a pressure solve: the fluxes replace the handle's, porous volumes are
 * computed from its geometry and porosities, and vag_transport may follow.
 * Pressures stay unavailable until the next vag_solve_pressure.
 */
vag_status vag_set_fluxes(vag_handle *h, const double *F_cell, const double *F_cell_frac, const double *F_frac,
                          vag_mem mem);

/* Peaceman wells (§5.5) perforating fracture faces: the flow from well k
 * into face face[k] is Q_k = wi[k] (p_w[k] - u_sigma) + q[k] (wi = 0: a well
 * at imposed rate q; q = 0: a well at pressure p_w), and the injected fluid
 * (Q_k > 0) carries concentration c_inj[k]; produced fluid (Q_k < 0) leaves
 * at the face's concentration and counts in the face's CFL outflow.  Each
 * face is perforated at most once; wi >= 0; arrays of n values in mem,
 * copied.  n = 0 removes the wells.  Takes effect at the next
 * vag_solve_pressure.  Hexahedral and general meshes alike: face[k] indexes
 * the fracture faces in the order vag_fractures lists them.  VAG_ERR_ARG
 * for a face out of range or perforated twice, a negative WI or a value that
 * is not finite. */
vag_status vag_set_wells(vag_handle *h, int64_t n, const int32_t *face, const double *wi, const double *p_w,
                         const double *q, const double *c_inj, vag_mem mem);
/* Q_k of the last solve (or of vag_set_well_rates), n values. */
vag_status vag_get_well_rates(vag_handle *h, double *Q, vag_mem mem);
/* Well rates for a transport on given fluxes: call after vag_set_fluxes
 * (which sets them to zero). */
vag_status vag_set_well_rates(vag_handle *h, const double *Q, vag_mem mem);
/* Peaceman well index of a fracture face of size dx (along the face) x dz
 * (along the well) and width d_f with permeability lambda_f, for a well of
 * radius r_w (§5.5, the face expanded to a dx x d_f x dz box):
 * 2 pi dz lambda_f / ln(r0 / r_w), r0 = D exp(-2 pi dz / C),
 * C = 4/3 (dx dz / d_f + dx d_f / dz + dz d_f / dx), D = sqrt(dx^2 + d_f^2) / 2.
 * 0 for non-positive arguments or r0 <= r_w. */
double vag_peaceman_wi(double dx, double dz, double d_f, double lambda_f, double r_w);

/* Pressures: u_node[n_nodes] (Dirichlet nodes carry p_bar), u_cell[n_cells],
 * u_frac[n_frac].  Any pointer may be NULL. */
vag_status vag_get_pressure(vag_handle *h, double *u_node, double *u_cell, double *u_frac,
                            vag_mem mem);

/* Fluxes: F_cell[n_cells][8] = F_{K,s} in VTK node order; F_cell_frac[n_frac][2]
 * = F_{K,sigma} for the cells of sigma by ascending cell index (0 for a missing
 * second cell); F_frac[n_frac][4] = F_{sigma,s} in the face's input node order.
 * General meshes: F_cell holds, cell after cell, F_{K,s} for the cell's nodes
 * in its local node order (sum over the cells of their node counts values),
 * F_frac, face after face, F_{sigma,s} for each fracture face's nodes in the
 * order of face_nodes (sum of their node counts values). */
vag_status vag_get_fluxes(vag_handle *h, double *F_cell, double *F_cell_frac, double *F_frac,
                          vag_mem mem);

/* Sizes of the F_cell and F_frac arrays of vag_get_fluxes / vag_set_fluxes:
 * 8 n_cells and 4 n_frac for hex8 meshes, the sums of the cells' and of the
 * fracture faces' node counts for general meshes. */
vag_status vag_flux_layout(const vag_handle *h, int64_t *n_cell_flux, int64_t *n_frac_flux);

/* Porous volumes phi_K, phi_sigma, phi_s (0 at Dirichlet nodes). */
vag_status vag_get_porous_volumes(vag_handle *h, double *phi_cell, double *phi_frac,
                                  double *phi_node, vag_mem mem);

/* Concentrations after the last transport call. */
vag_status vag_get_concentration(vag_handle *h, double *c_cell, double *c_frac, double *c_node,
                                 vag_mem mem);

/* Size of the assembled system of eq eqschur, after the elimination of the
 * fracture-face groups when enabled. */
vag_status vag_system_size(vag_handle *h, int64_t *n, int64_t *nnz);

/* z = M^-1 r with the preconditioner that the last vag_solve_pressure set up
 * (Jacobi: D^-1 r; AMG: one cycle from zero, K-cycles included; block-Jacobi
 * ILU(0): the forward and backward substitutions of every block).  r and z
 * hold n = vag_system_size values, in the unknown order of vag_get_system,
 * both in the memory space mem; caller-owned, r is only read.  For tests and
 * for callers that run a Krylov method of their own; synchronises the
 * handle's stream and overwrites the Krylov work vectors (the pressures and
 * fluxes of the last solve are kept).  VAG_ERR_STATE before the first solve,
 * VAG_ERR_UNSUPPORTED with VAG_MIXED_IR. */
vag_status vag_apply_preconditioner(vag_handle *h, const double *r, double *z, vag_mem mem);

/* Copies the assembled system (after a solve): CSR row_ptr[n+1], col[nnz]
 * (int64), val[nnz], b[n].  Unknown order: free nodes by node index, then the
 * fracture faces that are not eliminated, by face index (the device stores the
 * rows in another order, sorted by length inside windows). */
vag_status vag_get_system(vag_handle *h, int64_t *row_ptr, int64_t *col, double *val, double *b,
                          vag_mem mem);

/*
 * Measurement helper: launches `kernel` `reps` times back to back on the
 * handle's stream with the handle's current data (after a solve; the transport
 * step also needs a transport call) and returns the mean duration of one
 * launch from HIP events.  Scratch vectors only are written.
 */
vag_status vag_benchmark_kernel(vag_handle *h, int kernel, int reps, double *ms_per_launch);

/* AMG hierarchy of the last solve: number of levels and, per level (up to
 * max_levels; any array may be NULL), rows, nonzero entries and stored
 * entries (sliced ELL including padding). */
vag_status vag_amg_levels(vag_handle *h, int *nlev, int64_t *rows, int64_t *nnz, int64_t *stored, int max_levels);

/* Level `level` of the last solve's AMG hierarchy as host CSR arrays: the
 * matrix A_l (n x n, columns ascending, slice padding left out) and the
 * interpolation P_l (n x n_coarse) that carries level l + 1 back to level l
 * (aggregation: one entry 1 per row; none on the coarsest level), and for the
 * classical hierarchy the coarse index of each row (-1: fine point; every
 * entry -1 for aggregation).  Level 0 uses the unknown order of
 * vag_get_system.  sizes[4] receives n, nnz(A_l), n_coarse, nnz(P_l); call
 * with null arrays first to size them (caller-owned, any may be NULL).
 * VAG_ERR_STATE without an AMG solve, VAG_ERR_ARG for a level out of range. */
vag_status vag_amg_level_csr(vag_handle *h, int level, int64_t *sizes, int64_t *a_ptr, int64_t *a_col,
                             double *a_val, int64_t *p_ptr, int64_t *p_col, double *p_val,
                             int32_t *coarse_index);

/* Device bytes held by the handle. */
size_t vag_footprint_bytes(const vag_handle *h);

/* Text of the handle's last error ("" if none); for a NULL handle, of the last
 * failed vag_create in this thread. */
const char *vag_last_error(const vag_handle *h);

/* Releases the handle (after waiting for its stream).  Its device blocks go
 * back to the library's per-device cache and its pinned host blocks to the
 * library's free list, both kept for later handles of the process
 * (vag_trim_memory returns the cached device blocks to the system). */
void vag_destroy(vag_handle *h);

/* Returns the cached (unused) device blocks of the current device to the
 * system.  Waits for the device to be idle first.  Errors: VAG_ERR_HIP. */
vag_status vag_trim_memory(void);

/*
 * Upper bound of the device bytes a handle of these sizes holds after a solve
 * and a transport call with these options (opt NULL = defaults); used for
 * admission by footprint.
 */
size_t vag_estimate_footprint(int64_t n_nodes, int64_t n_cells, int64_t n_frac, const vag_options *opt);
/* The same for a mesh in either form (host arrays): a hex8 mesh as above; a
 * mesh given by its faces adds its local matrices (from each cell's face and
 * node counts) and flux incidences.  0 for an inconsistent mesh. */
size_t vag_estimate_footprint_mesh(const vag_mesh *mesh, int64_t n_frac, const vag_options *opt);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of independent Darcy + transport jobs.       */
/* ------------------------------------------------------------------------ */
/*
 * A server owns n_workers host threads, each with its own HIP stream on the
 * device that is current when the server is created.  Submitted jobs wait in
 * one FIFO queue; the head job starts on the first free worker as soon as its
 * estimated footprint (vag_estimate_footprint_mesh) fits in what the running jobs
 * and the cached handles leave of hbm_budget.  Jobs on different workers run
 * concurrently, so their kernels overlap on the device.  The transport steps
 * of jobs below 2^18 control volumes are batched per launch: per size class
 * (below 2^16, 2^17, 2^18 control volumes) a host thread launches, tick after
 * tick on a stream of its own, one kernel that takes one step of every job of
 * the class in its transport phase (up to 8 jobs a launch); a job joins once
 * its upwind operator is built and leaves after its last step, while its
 * worker takes the next job (larger jobs' steps fill the device alone and
 * their worker launches them).  Every row of a job gets the arithmetic, in
 * the same order, of the job run alone on a lone handle, so its results are
 * bitwise those of the job run alone.
 *
 * A job with a nonzero mesh_key keeps its handle (matrices, AMG hierarchy and
 * all buffers) resident after it finishes; a later job with the same key and
 * the same sizes reuses it with vag_update (topology and fracture set must be
 * the same: the key is the caller's promise), skipping the symbolic phase and
 * the allocations.  Idle cached handles count against the budget and are
 * destroyed, least recently used first, when a job needs their room.
 */
typedef struct vag_server vag_server;

typedef struct {
    const vag_mesh *mesh;
    const vag_fractures *frac;      /* NULL: no fracture */
    const vag_rock *rock;
    const vag_bc *bc;
    const vag_options *opt;         /* NULL: defaults */
    int64_t n_steps;                /* transport after the solve, as vag_transport */
    double t_final;
    uint64_t mesh_key;              /* 0: no handle reuse */
    /* Host output buffers, written by the worker; NULL = not wanted.  They must
     * stay valid until vag_server_wait returns for this job. */
    double *u_node, *u_cell, *u_frac;   /* [n_nodes], [n_cells], [n_frac] */
    double *c_cell, *c_frac, *c_node;   /* concentrations after the steps */
} vag_job;

typedef struct {
    int status;                     /* vag_status of the job */
    char message[200];              /* vag_last_error text when status != VAG_OK */
    vag_solve_info solve;
    vag_transport_info transport;
    double t_submit, t_start, t_end;  /* seconds on the server's steady clock */
    int worker;                     /* worker that ran the job, -1 if it never ran */
    int reused;                     /* 1 if a cached handle was reused */
    size_t footprint_estimate, footprint_bytes;
    double ms_create;               /* wall time of vag_create (host symbolic phase, uploads) */
    double ms_run;                  /* wall time from the start of the job to its outputs on the host */
} vag_job_result;

typedef struct {
    int64_t submitted, queued, running, finished;
    size_t budget, bytes_in_use, peak_bytes_in_use, cached_bytes;
    int cached_handles;
    int64_t step_launches;  /* batched transport launches so far */
    int64_t job_steps;      /* transport steps of all jobs so far (>= step_launches) */
} vag_server_stats;

/* hbm_budget 0: 80 % of the free device memory at creation.  n_workers in
 * [1, 16].  Errors: VAG_ERR_ARG, VAG_ERR_HIP. */
vag_status vag_server_create(size_t hbm_budget, int n_workers, vag_server **out);

/* Copies the job's input arrays (host memory) and queues it; returns at once.
 * The mesh may take either form (hex8, or faces with fracture face_ids).
 * VAG_ERR_OOM when the job's estimate exceeds the whole budget, VAG_ERR_ARG
 * for missing inputs or face lists whose offsets do not start at 0 and never
 * decrease (the rest of the mesh is checked by vag_create when the job runs). */
vag_status vag_server_submit(vag_server *s, const vag_job *job, uint64_t *job_id);

/* Waits up to timeout_s seconds (< 0: no limit) for the job.  VAG_OK: *res is
 * filled, the outputs are written and the id is released.  VAG_ERR_TIMEOUT:
 * still queued or running.  VAG_ERR_ARG: unknown id. */
vag_status vag_server_wait(vag_server *s, uint64_t job_id, double timeout_s, vag_job_result *res);

/* Cancels a job that has not started (its wait then reports
 * VAG_ERR_CANCELLED); VAG_ERR_STATE if it already started. */
vag_status vag_server_cancel(vag_server *s, uint64_t job_id);

vag_status vag_server_get_stats(vag_server *s, vag_server_stats *st);

/* Seconds on the server's steady clock (the clock of t_submit etc.). */
double vag_server_clock(vag_server *s);

/* Cancels queued jobs, waits for running ones, releases everything. */
void vag_server_destroy(vag_server *s);

#ifdef __cplusplus
}
#endif
#endif /* VAG_H */
