// Internal declarations of libvag: device buffers, the handle, the symbolic
// phase and the kernel launchers.  Nothing here crosses the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "vag.h"

namespace vag {

// Loads of the entries of a large matrix, read once per pass: marked
// non-temporal so that they do not push out of the caches the vector entries
// that neighbouring rows gather again.  A matrix that fits the last-level
// cache (256 MB) together with its vectors is read with ordinary loads, since
// it is read again by the next pass.
constexpr int64_t kStreamBytes = int64_t(128) << 20;
// mode (vag_options.stream_loads): 0 automatic (above kStreamBytes), 1 always, 2 never
inline bool stream_matrix(int64_t stored, int value_bytes, int mode) {
    if (mode == 1) return true;
    if (mode == 2) return false;
    return stored * (value_bytes + 4) > kStreamBytes;
}
template <bool NT, class T>
__device__ __forceinline__ T ld_matrix(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// ---------------------------------------------------------------------------
// errors: thrown inside the library, turned into a vag_status at the ABI
// ---------------------------------------------------------------------------
// Named ranges on the host timeline of a profiler's marker trace (rocprofv3
// --marker-trace); a range is closed on every exit of its scope, exceptions
// included.  Phases holds one open range at a time: next() closes the
// current one and opens the next.
class Phases {
public:
    explicit Phases(const char *name) { next(name); }
    void next(const char *name) {
        if (open_) roctxRangePop();
        roctxRangePushA(name);
        open_ = true;
    }
    ~Phases() {
        if (open_) roctxRangePop();
    }
    Phases(const Phases &) = delete;
    Phases &operator=(const Phases &) = delete;

private:
    bool open_ = false;
};

struct Error : std::runtime_error {
    vag_status status;
    Error(vag_status s, const std::string &m) : std::runtime_error(m), status(s) {}
};

#define VAG_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            throw ::vag::Error(e_ == hipErrorOutOfMemory ? VAG_ERR_OOM : VAG_ERR_HIP,  \
                               std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

// Faces of a VTK hexahedron, cyclic and outward oriented (right-hand rule), so
// that every sub-tetrahedron (x_K, x_sigma, s_e, s_e+1) of a valid cell has a
// positive signed volume.
__host__ __device__ constexpr int hexf(int f, int i) {
    constexpr int t[24] = {0, 4, 7, 3, 1, 2, 6, 5, 0, 1, 5, 4, 3, 7, 6, 2, 0, 3, 2, 1, 4, 5, 6, 7};
    return t[f * 4 + i];
}
// packed upper triangle of a symmetric 8x8 block
__host__ __device__ constexpr int sym8(int i, int j) {
    return i <= j ? i * 8 - i * (i - 1) / 2 + (j - i) : j * 8 - j * (j - 1) / 2 + (i - j);
}
// packed upper triangle of a symmetric 5x5 block
__host__ __device__ constexpr int sym5(int i, int j) {
    return i <= j ? i * 5 - i * (i - 1) / 2 + (j - i) : j * 5 - j * (j - 1) / 2 + (i - j);
}

constexpr int kSliceRows = 64;      // SELL slice height = one wavefront
constexpr int kReduceBlocks = 512;  // fixed grid of the deterministic reductions
constexpr int kReduceThreads = 256;
constexpr int kKrylovThreads = 1024;  // block size of the Krylov kernels (and of their partials' producers)

// ---------------------------------------------------------------------------
// device buffer
// ---------------------------------------------------------------------------
// Device memory comes from a per-device cache of blocks: hipFree would
// synchronise the whole device at every handle destruction, serialising the
// independent handles that run side by side on their own streams.  A block
// returns to the cache only after the stream of its owner has been
// synchronised, so no queued kernel of the old owner can touch it once
// another handle takes it.
void *dev_alloc(size_t bytes);
void dev_free(void *p, hipStream_t owner_stream);
// Pinned host blocks from a process-wide free list (same reason: hipHostFree
// synchronises the device).  bytes must be the size given to pinned_get.
void *pinned_get(size_t bytes);
void pinned_put(void *p, size_t bytes);

struct Tracker {
    size_t bytes = 0;
    hipStream_t stream = nullptr;  // the stream the buffers are used on
};

template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    Tracker *tr = nullptr;
    void alloc(size_t count, Tracker &t) {
        release();
        tr = &t;
        n = count;
        if (count) {
            p = static_cast<T *>(dev_alloc(count * sizeof(T)));
            t.bytes += count * sizeof(T);
        }
    }
    void release() {
        if (p) {
            dev_free(p, tr ? tr->stream : nullptr);
            if (tr) tr->bytes -= n * sizeof(T);
        }
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
    ~DBuf() { release(); }
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
};

// ---------------------------------------------------------------------------
// symbolic phase (host): topology-only data structures
// ---------------------------------------------------------------------------
// A std::vector whose resize leaves new elements uninitialised (no zero
// fill), for large host arrays written in full right afterwards.
template <class T>
struct DefaultInitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = DefaultInitAlloc<U>;
    };
    DefaultInitAlloc() = default;
    template <class U>
    DefaultInitAlloc(const DefaultInitAlloc<U> &) noexcept {}
    template <class U>
    void construct(U *p) noexcept {
        ::new ((void *)p) U;
    }
    template <class U, class... A>
    void construct(U *p, A &&...a) {
        ::new ((void *)p) U(std::forward<A>(a)...);
    }
};
template <class T>
using uvector = std::vector<T, DefaultInitAlloc<T>>;

struct Symbolic {
    // nunk: rows of the assembled system (free nodes, kept fracture faces);
    // nx: all nodal and face unknowns (eliminated faces numbered after nunk)
    int32_t nn = 0, nc = 0, nf = 0, nfree = 0, nunk = 0, nx = 0;
    int64_t nnz = 0;
    std::vector<uint8_t> fmask;        // [nc] bit f = local face f is a fracture face
    std::vector<int32_t> cell_frac;    // [nc*6] fracture index of local face, -1
    std::vector<int32_t> frac_cell;    // [nf*2] cells of sigma, ascending, -1 if absent
    std::vector<int32_t> frac_slot;    // [nf*4] slot (0..7) in frac_cell[.,0] of input node i
    std::vector<int32_t> node_unk;     // [nn] unknown index, -1 for Dirichlet nodes
    std::vector<uint8_t> frac_node;    // [nn] node of some fracture face
    std::vector<int32_t> node_cell_ptr, node_cell;  // node -> cell*8+slot, ascending
    std::vector<int32_t> node_frac_ptr, node_frac;  // node -> frac*4+i, ascending
    // CSR pattern of the eliminated system (sorted rows).  col_on_host false:
    // the device built the columns (straight into the sliced-ELL layout) and
    // col is empty until a host consumer downloads them; row_ptr is there.
    std::vector<int32_t> row_ptr;
    uvector<int32_t> col;
    bool col_on_host = true;
    // node row (natural numbering, before the renumbering) -> eliminated
    // groups holding that node: the fill of its row
    std::vector<int32_t> node_grp_ptr, node_grp;
    std::vector<int64_t> sell_ptr;                   // sliced-ELL slice pointers of that pattern
    std::vector<int32_t> unk_node, unk_face;         // row -> free node (rows < nfree), -> kept face
    std::vector<int32_t> sys_old, sys_new;           // system row renumbering: new -> natural, natural -> new
    std::vector<int32_t> face_grp, face_loc;         // [nf] eliminated group of sigma and index in it, or -1
    std::vector<int32_t> frac_unk;                   // [nf] unknown index of sigma (>= nunk: eliminated)
    // Fracture-face groups eliminated onto the nodes: faces linked through a
    // shared cell, ordered by colour (groups of one colour share no free node).
    // Group G: faces grp_face[grp_ptr[G]..], free nodes of its cells
    // grp_node[grp_nptr[G]..] (system unknowns, ascending), a dense block of
    // g x (g + m) values at grp_off[G], and the system positions of its m x m
    // node pairs at grp_pos[grp_poff[G]..].
    int32_t ngroup = 0, ngcolor = 0, grp_max_g = 0, grp_max_m = 0;
    std::vector<int32_t> grp_ptr, grp_face, grp_nptr, grp_node, grp_pos, gcolor_ptr;
    std::vector<int64_t> grp_off, grp_poff;
};

// General cells (cell -> faces, face -> nodes): what the symbolic phase of a
// general mesh adds to Symbolic (whose node and face numbering, pattern and
// renumbering it shares; cell_frac holds 6 entries per cell, frac_cell 2 per
// fracture face, frac_node the fracture-node flags).
constexpr int kGenMaxFaces = 6;      // faces of a cell
constexpr int kGenMaxNodes = 8;      // nodes of a cell
constexpr int kGenMaxFaceNodes = 4;  // nodes of a face
struct GenSym {
    int64_t ncn = 0;                 // sum over cells of their node counts
    int64_t nfn = 0;                 // sum over fracture faces of their node counts
    int64_t nflux = 0;               // ncn + 2 nf + nfn: the flux array [cell-node | cell-face | face-node]
    int max_nv = 0, max_nf = 0, max_fk = 0;  // the most nodes, faces and face nodes of a cell
    std::vector<int32_t> cnode_ptr;  // [nc + 1] cell -> its nodes, local order
    std::vector<int32_t> cnode;      // [ncn] global node indices
    std::vector<uint8_t> cface_k;    // [6 nc] node count of local face f (0: no such face)
    std::vector<uint8_t> cface_loc;  // [24 nc] local node indices of local face f, cyclic as given
    std::vector<int32_t> fnode_ptr;  // [nf + 1] fracture face -> its nodes
    std::vector<int32_t> fnode;      // [nfn] global node indices, the face's cyclic order
    std::vector<int32_t> unk_off;    // [nc + 1] prefix of the cells' unknown counts m (row sums r)
    std::vector<int64_t> loc_off;    // [nc + nf + 1] blocks in the local value array: m x m per cell
                                     // (the Schur block M), then (k + 1)^2 per fracture face
    std::vector<int64_t> con_ptr;    // [stored + 1] contributions to each sliced-ELL slot of the system
    std::vector<int64_t> con;        // local value indices, in a fixed order
    std::vector<int32_t> bcon_ptr;   // [nunk + 1] Dirichlet-column contributions to each row of b
    std::vector<int64_t> bcon;       // local value index
    std::vector<int32_t> bcon_node;  // the Dirichlet node of that column
    std::vector<int64_t> inc_ptr;    // [nc + nf + nn + 1] control volume -> its fluxes
    std::vector<int32_t> inc_edge;   // flux index << 1 | 1 if the control volume is the flux's far end
    std::vector<int32_t> inc_other;  // the control volume at the other end
};
// Builds Symbolic and GenSym for a general mesh; throws vag::Error on invalid
// or unsupported input (sizes of cells and faces, orientation is checked on
// the device).  face_ids: the fracture faces as face indices.
void build_symbolic_general(int64_t nn, int64_t nc, int64_t nface, const int64_t *cell_face_ptr,
                            const int32_t *cell_faces, const int64_t *face_node_ptr, const int32_t *face_nodes,
                            int64_t nf, const int32_t *face_ids, const uint8_t *dirichlet, Symbolic &S,
                            GenSym &G);
// Renumbering of the system rows (longest first inside windows) and the
// sliced-ELL slice pointers of the CSR pattern in S (shared by both paths).
void finish_symbolic_pattern(Symbolic &S, const std::vector<const int32_t *> *row_src = nullptr,
                             bool columns = true);
// the renumbering and layout from the row lengths the device found (natural
// row order), without columns
void finish_symbolic_lengths(Symbolic &S, const int32_t *len);

// Rows are sorted by length inside windows of this many rows (slice padding).
constexpr int kSortWindow = 512;

// Limits of an eliminated fracture-face group (larger groups stay unknowns).
constexpr int kGroupMaxFaces = 32;
constexpr int kGroupMaxNodes = 64;

// Builds the symbolic data; throws vag::Error on invalid input.
// With eliminate, fracture-face groups within the limits above are
// eliminated; otherwise every face stays an unknown.  With rows_on_device,
// it stops before the pattern (the caller builds the rows on the device and
// then calls finish_symbolic_lengths); otherwise the host builds it.
void build_symbolic(int64_t nn, int64_t nc, int64_t nf, const int32_t *hex8,
                    const int32_t *frac_nodes, const uint8_t *dirichlet, bool eliminate, Symbolic &S,
                    bool rows_on_device = false);

// ---------------------------------------------------------------------------
// kernel launchers (defined in the .hip files)
// ---------------------------------------------------------------------------
// Sliced ELL: slices of 64 rows (one wavefront), entries of a slice stored
// column-major (entry k of row r at ptr[r/64] + 64 k + r%64), slice width = its
// longest row; padding entries point at their own row with value 0.
template <class V>
struct Sell {
    int32_t n = 0;
    const int64_t *ptr = nullptr;
    const int32_t *col = nullptr;
    const V *val = nullptr;
    // optional diagonal held apart in FP64 (the stored diagonal entries are
    // then zero): the FP32 copies keep each row's FP64 row sum this way
    const double *dg = nullptr;
    // optional 16-bit column offsets, one base per group of 64 stored entries
    // (one level of a slice): where the slice's first group has cbase >= 0,
    // the column of entry q is cbase[q / 64] + col16[q] (the row loops read 2
    // bytes per entry instead of 4); other kernels keep reading col
    const uint16_t *col16 = nullptr;
    const int32_t *cbase = nullptr;
    // the row loops read val and the columns with non-temporal loads
    bool nt = false;
};
// col16 and cbase (one per 64 stored entries) of a sliced-ELL pattern: a
// slice each of whose levels holds real columns within 65536 of the level's
// least gets that least as the level's base, else -1 for all its levels
void launch_sell_pack(hipStream_t s, int32_t n, const int64_t *ptr, const int32_t *col, const int32_t *row_len,
                      uint16_t *col16, int32_t *cbase);

struct PcgState {       // device-resident scalars of a Krylov solve
    double tol2, bnorm2, rr, pad;
    int iter, done, converged, pad2;
};

// Partials of the CG scalars, double-buffered by iteration parity:
// pq at [0, G), rz[p] at [(1+p) G, (2+p) G), rr[p] at [(3+p) G, (4+p) G).
struct PcgParts {
    double *base;
    int G;
    __host__ __device__ double *pq() const { return base; }
    __host__ __device__ double *rz(int k) const { return base + (size_t)(1 + (k & 1)) * G; }
    __host__ __device__ double *rr(int k) const { return base + (size_t)(3 + (k & 1)) * G; }
    // flexible CG: z_{k+1} . q_k (written by the preconditioner's last sweep)
    __host__ __device__ double *zq() const { return base + (size_t)5 * G; }
};

// assembly
void launch_local(hipStream_t s, int32_t nc, const double *xyz, const int32_t *hex8, const double *perm,
                  double mu, const uint8_t *fmask, const int32_t *cell_frac, const int32_t *frac_cell,
                  double *aK, double *rK, double *AKK, double *vol, double *fside, int *bad_cell);
void launch_frac_local(hipStream_t s, int32_t nf, const double *xyz, const int32_t *frac_nodes,
                       const double *width, const double *perm, double mu, double *A5, double *area);
// Arguments of the row-by-row assembly kernels (device pointers).
struct AsmArgs {
    int32_t nc, nfree, nsys;
    const int32_t *hex8, *node_unk, *frac_unk, *unk_node, *unk_face;
    const int32_t *node_cell_ptr, *node_cell, *node_frac_ptr, *node_frac;
    const uint8_t *fmask;
    const int32_t *cell_frac, *frac_cell, *frac_nodes;
    const double *aK, *rK, *AKK, *fside, *A5, *p_bar;
    const int64_t *sell_ptr;
    const int32_t *sell_col, *row_len;
    const int32_t *grp_ptr, *grp_face, *grp_nptr, *grp_node, *face_grp, *face_loc;
    const int64_t *grp_off;
    double *A, *Gb, *b;
    int *bad;  // receives INT_MIN if a position is missing from the pattern
    // slot of column c of M_K in the row of each node_cell entry q:
    // node_pos[8 q + c] (0xffff: a Dirichlet column); null before it is built
    const uint16_t *node_pos;
};
// Node rows, kept-face rows, eliminated-face rows (into the group blocks).
void launch_assemble(hipStream_t s, const AsmArgs &g, int32_t nkept, int32_t nelim);
// The system pattern of a hexahedral mesh on the device: row bounds, then the
// rows themselves (natural numbering and order, sorted, at off), then their
// renumbering (see pattern.hip).
struct PatArgs {
    int32_t nn, nf, nunk;
    const int32_t *hex8, *node_cell_ptr, *node_cell, *node_unk, *frac_unk, *cell_frac, *frac_cell;
    const uint8_t *fmask;
    const int32_t *node_grp_ptr, *node_grp, *grp_nptr, *grp_node;
};
// node_cell_ptr (nn + 1) and node_cell (8 nc: K * 8 + a, ascending per node)
// of a hexahedral mesh; work: nn + 2 (nn / 1024 + 2) ints
void launch_node_cell(hipStream_t s, int32_t nn, int64_t nc, const int32_t *hex8, int32_t *ptr, int32_t *cells,
                      int32_t *work);
void launch_pattern_bound(hipStream_t s, const PatArgs &g, int32_t *ub);
// out[0..n] = exclusive scan of in (out[n] the total), n > 0; sums: n / 1024 + 2
void launch_scan64(hipStream_t s, int32_t n, const int32_t *in, int64_t *out, int64_t *sums);
void launch_pattern_rows(hipStream_t s, const PatArgs &g, const int64_t *off, int32_t *raw, int32_t *len);
// col (row_ptr layout) = the rows of raw (natural order and numbering, sorted,
// at off) renumbered by sys_new and sorted, row r from natural row sys_old[r]
void launch_pattern_sort(hipStream_t s, int32_t n, const int32_t *row_ptr, const int32_t *sys_old,
                         const int64_t *off, const int32_t *raw, const int32_t *sys_new, int32_t *col);
// Sliced-ELL columns, row lengths and diagonal positions from the CSR pattern.
void launch_sell_fill(hipStream_t s, int32_t n, int64_t nslice, const int32_t *row_ptr, const int32_t *col,
                      const int64_t *sell_ptr, int32_t *sell_col, int32_t *row_len, int32_t *diag_pos);
// bad[0] = the least cell whose tensor is not symmetric positive definite,
// bad[1] = the least fracture face without positive width and permeability
// (both left as they were where none fails)
void launch_check_coef(hipStream_t s, int32_t nc, const double *perm, int32_t nf, const double *fwidth,
                       const double *fperm, int *bad);
// node_pos (see AsmArgs) for the rows of the free nodes, once per handle.
void launch_node_pos(hipStream_t s, const AsmArgs &g, uint16_t *node_pos);
// System positions of the node pairs of each eliminated group.
void launch_grp_pos(hipStream_t s, const AsmArgs &g, int32_t ngroup, const int64_t *grp_poff, int32_t *grp_pos);
// Eliminates groups [first, first+ngroup) (one colour) onto the node rows.
// bad receives -1-G for a group whose face block is not positive definite.
void launch_group_elim(hipStream_t s, int32_t first, int32_t ngroup, int max_g, int max_m, const int32_t *grp_ptr,
                       const int32_t *grp_face, const int32_t *grp_nptr, const int32_t *grp_node,
                       const int64_t *grp_off, const int64_t *grp_poff, const int32_t *grp_pos,
                       const int32_t *frac_unk, double *Gb, double *A, double *b, int *bad);
// x of the eliminated faces from the solved node unknowns.
void launch_group_back(hipStream_t s, int32_t ngroup, const int32_t *grp_ptr, const int32_t *grp_face,
                       const int32_t *grp_nptr, const int32_t *grp_node, const int64_t *grp_off,
                       const int32_t *frac_unk, const double *Gb, const double *b, double *x);
void launch_diag_inv(hipStream_t s, int32_t n, const int32_t *diag_pos, const double *A, double *dinv);

// BiCGStab (bicgstab.hip): parts holds 8 * bcg_grid(n) doubles
int bcg_grid(int64_t n);
void launch_bcg_init(hipStream_t s, Sell<double> A, bool zero_x, int k0, const double *b, double *x, double *r,
                     double *rhat, double *parts);
void launch_bcg_start(hipStream_t s, int32_t n, double *parts, PcgState *st, double rtol, int k0);
void launch_bcg_direction(hipStream_t s, int32_t n, int k, int k0, const double *r, double *p, const double *v,
                          double *parts, PcgState *st, bool update);
void launch_bcg_spmv_v(hipStream_t s, Sell<double> A, const double *phat, double *v, const double *rhat,
                       double *parts, const PcgState *st);
void launch_bcg_s(hipStream_t s, int32_t n, int k, const double *r, const double *v, const double *phat, double *sv,
                  double *x, double *parts, PcgState *st);
void launch_bcg_spmv_t(hipStream_t s, Sell<double> A, const double *shat, double *t, const double *sv, double *parts,
                       const PcgState *st);
void launch_bcg_update(hipStream_t s, int32_t n, int k, const double *phat, const double *shat, const double *sv,
                       const double *t, const double *rhat, double *x, double *r, double *parts, PcgState *st);

// Krylov
int pcg_grid(int64_t n);
void launch_fill(hipStream_t s, int64_t n, double v, double *x);
void launch_copy(hipStream_t s, int64_t n, const double *src, double *dst);
void launch_jacobi(hipStream_t s, int64_t n, const double *dinv, const double *r, double *z);
void launch_spmv(hipStream_t s, Sell<double> A, const double *x, double *y);
void launch_residual_norm(hipStream_t s, Sell<double> A, const double *x, const double *b, double *r,
                          double *parts, double *out2 /* [2]: ||b-Ax||^2, ||b||^2 */);
// x = 0, r = b, parts rr(-1) = b.b; with dinv also z = D^-1 b, p = z and parts rz(-1)
void launch_pcg_init(hipStream_t s, int32_t n, const double *b, const double *dinv, double *x, double *r,
                     double *z, PcgParts P);
// one block: tolerance rtol^2 rr(k0-1), state reset to iteration k0
void launch_pcg_start(hipStream_t s, PcgParts P, PcgState *st, double rtol, int k0);
// warm start at iteration k0 from the current x (see krylov.hip)
void launch_pcg_init_warm(hipStream_t s, Sell<double> A, int k0, const double *b, const double *x, double *r,
                          const double *dinv, double *z, PcgParts P);
// convergence test on rr(k-1); then p = z + beta p (beta = rz(k-1)/rz(k-2), 0 at k = 0;
// flexible: beta = -zq/pq, which keeps p A-orthogonal to the previous
// direction when the preconditioner changes from one application to the next)
template <class T>
void launch_pcg_direction(hipStream_t s, int32_t n, int k, int k0, const T *z, T *p, PcgParts P, PcgState *st,
                          bool update, bool flexible = false);
// q = A p, partials of p.q
template <class V, class T>
void launch_pcg_spmv(hipStream_t s, Sell<V> A, const T *p, T *q, PcgParts P, const PcgState *st);
// alpha = rz(k-1) / p.q; x += alpha p; r -= alpha q; Jacobi: z = D^-1 r and partials rz(k), rr(k)
void launch_pcg_update(hipStream_t s, int32_t n, int k, double *x, double *r, double *z, const double *p,
                       const double *q, const double *dinv, PcgParts P, PcgState *st);
// same without the preconditioner: partials rr(k) only
template <class T>
void launch_pcg_update_xr(hipStream_t s, int32_t n, int k, T *x, T *r, const T *p, const T *q, PcgParts P,
                          PcgState *st, const T *dinv = nullptr, T *x0 = nullptr);
// partials rz(k) = r.z
template <class T>
void launch_pcg_dot_rz(hipStream_t s, int32_t n, int k, const T *r, const T *z, PcgParts P, const PcgState *st);
// x = 0, r = b, partials rr(-1) = b.b
template <class T>
void launch_pcg_init_plain(hipStream_t s, int32_t n, const T *b, T *x, T *r, PcgParts P);
// FP64 refinement helpers: out[0] = ||r||^2; r32 = r / ||r||; x += ||r|| d32
void launch_norm2(hipStream_t s, int32_t n, const double *r, double *parts, double *out);
void launch_normalize_to_float(hipStream_t s, int32_t n, const double *r, const double *nrm2, float *r32);
void launch_correct(hipStream_t s, int32_t n, double *x, const float *d32, const double *nrm2);

// recovery, fluxes, transport
void launch_node_pressure(hipStream_t s, int32_t nn, const int32_t *node_unk, const double *x,
                          const double *p_bar, double *u_node);
void launch_cell_flux(hipStream_t s, int32_t nc, const int32_t *hex8, const uint8_t *fmask,
                      const int32_t *cell_frac, const int32_t *frac_cell, const double *aK,
                      const double *rK, const double *AKK, const double *fside, const double *u_node,
                      const double *u_frac, double *u_cell, double *F_cell, double *F_cell_frac);
void launch_frac_flux(hipStream_t s, int32_t nf, const int32_t *frac_nodes, const double *A5,
                      const double *u_node, const double *u_frac, double *F_frac);
// Porous volumes (§3.2.1).  pmax == nullptr: every adjacent cell (fracture
// face) gives a node its share; else only those whose permeability reaches
// pmax[node] (launch_node_pmax), the rule for nodes between rock types.
void launch_porous(hipStream_t s, int32_t nc, int32_t nf, int32_t nn, const int32_t *hex8,
                   const int32_t *frac_nodes, const uint8_t *dirichlet, const uint8_t *frac_node,
                   const int32_t *node_cell_ptr, const int32_t *node_cell, const int32_t *node_frac_ptr,
                   const int32_t *node_frac, const double *vol, const double *poro, const double *area,
                   const double *fwidth, const double *fporo, const double *perm, const double *fperm,
                   const double *pmax, double *phi_cell, double *phi_frac, double *phi_node);
// pmax[s]: the largest permeability around node s, over the fracture faces at
// a fracture node, over the cells elsewhere (a cell's permeability: the trace
// of its tensor over 3)
void launch_node_pmax(hipStream_t s, int32_t nn, const uint8_t *frac_node, const int32_t *node_cell_ptr,
                      const int32_t *node_cell, const int32_t *node_frac_ptr, const int32_t *node_frac,
                      const double *perm, const double *fperm, double *pmax);
__device__ __forceinline__ double perm_measure(const double *perm, int64_t K) {
    return (perm[6 * K] + perm[6 * K + 1] + perm[6 * K + 2]) / 3.0;
}
void launch_cfl(hipStream_t s, int32_t nc, int32_t nf, int32_t nn, const int32_t *hex8,
                const uint8_t *fmask, const int32_t *cell_frac, const int32_t *frac_cell,
                const uint8_t *dirichlet, const int32_t *node_cell_ptr, const int32_t *node_cell,
                const int32_t *node_frac_ptr, const int32_t *node_frac, const double *F_cell,
                const double *F_cell_frac, const double *F_frac,
                const double *wout /* [nf] volume produced by a well per face, or null */,
                const double *phi_cell, const double *phi_frac, const double *phi_node, double cfl,
                double *parts, double *dt_out /* [4]: dtM, dtF, dtV, dt */);
void launch_upwind_count(hipStream_t s, int32_t nc, int32_t nf, int32_t nn, const uint8_t *fmask,
                         const int32_t *cell_frac, const int32_t *frac_cell, const uint8_t *dirichlet,
                         const int32_t *node_cell_ptr, const int32_t *node_cell,
                         const int32_t *node_frac_ptr, const int32_t *node_frac, const double *F_cell,
                         const double *F_cell_frac, const double *F_frac, const double *wsrc, int32_t *slice_width,
                         uint16_t *meta, int32_t *slice_nnz);
// slice_ptr = exclusive scan of per_width * slice_width (64 for padded
// sliced ELL, 1 for counts of packed entries); with slice_nnz, *total = its sum
void launch_slice_scan(hipStream_t s, int32_t nslice, const int32_t *slice_width, int per_width, int64_t *slice_ptr,
                       const int32_t *slice_nnz = nullptr, unsigned long long *total = nullptr);
void launch_upwind_fill(hipStream_t s, int32_t nc, int32_t nf, int32_t nn, const int32_t *hex8,
                        const uint8_t *fmask, const int32_t *cell_frac, const int32_t *frac_cell,
                        const int32_t *frac_nodes, const uint8_t *dirichlet, const int32_t *node_cell_ptr,
                        const int32_t *node_cell, const int32_t *node_frac_ptr, const int32_t *node_frac,
                        const double *F_cell, const double *F_cell_frac, const double *F_frac,
                        const double *wsrc, const double *wout, const double *phi_cell, const double *phi_frac,
                        const double *phi_node,
                        const double *dt, const int64_t *slice_ptr, const uint16_t *meta, int32_t *tcol,
                        double *tval, double *tdiag);
// Upwind operator: 64-row slices (rows sorted longest first, meta = source
// lane << 8 | entry count per slot), entries packed by level (jagged
// diagonals) from slice_ptr[slice]; 16-bit columns from tbase[slice] where
// tbase >= 0, else the 32-bit tcol.
// The sweep splits the slices into two segments, A = [0, sa) (cells and
// fracture faces) and B = [sa, nslice) (nodes), and gives XCD x of the 8 the
// slices [xlo[x], xlo[x+1]) of A and [ylo[x], ylo[x+1]) of B, runs of equal
// cost (bytes moved) in each segment.  The XCD interleaves its two runs in
// proportion, so that the cells and the nodes of one region of the mesh
// (both numbered along the mesh) are swept together and the gathers of each
// hit the lines the other has brought into that XCD's L2; the cost balance
// keeps every XCD equally busy when rows differ in length along the
// numbering (cells of 4 nodes, nodes of 24 cells).
struct UpwindOp {
    int32_t nrow;
    const int64_t *slice_ptr;
    const uint16_t *meta;
    const int32_t *tcol;
    const uint16_t *tcol16;
    const int32_t *tbase;
    const double *tval, *tdiag;
    int32_t xlo[9], ylo[9];
};
// tcol16 and tbase from tcol (after launch_upwind_fill)
void launch_upwind_pack(hipStream_t s, const UpwindOp &T, uint16_t *tcol16, int32_t *tbase);
// xlo[0..8] and ylo[0..8] (at xlo + 9) from slice_ptr (after the slice scan)
void launch_xcd_split(hipStream_t s, int32_t nslice, int32_t sa, const int64_t *slice_ptr, int32_t *xlo);
// backward: sweep each XCD's slices in reverse order (alternate steps)
void launch_transport_step(hipStream_t s, const UpwindOp &T, const double *c_in, double *c_out, double theta,
                           bool backward);
// blocks of one step's launch over T (a multiple of 8)
int32_t transport_step_blocks(const UpwindOp &T);
// One step of up to kBatchJobs operators in one launch (served jobs): each
// operator's rows get exactly the arithmetic of launch_transport_step.
constexpr int kBatchJobs = 8;
struct TransportJob {
    UpwindOp T;
    const double *c_in;
    double *c_out;
    double theta;
    int32_t backward;
};
struct TransportBatch {
    int32_t n;
    int32_t blk[kBatchJobs + 1];  // first block of each job (set by the launcher)
    TransportJob job[kBatchJobs];
};
static_assert(sizeof(TransportBatch) <= 2048, "kernel argument block");
void launch_transport_batch(hipStream_t s, TransportBatch &B);

}  // namespace vag

// The server's side of a served job's transport: begin prepares it (time
// step, upwind operator, initial state) on the handle's stream and gives the
// step count; job(k) describes step k for a batched launch and moves the
// handle to the next state; the server records event 6 before the job's
// first step and event 7 after its last, on the stream it launches on; end
// waits for event 7 and reports.
extern "C" {
vag_status vag_serving_transport_begin(vag_handle *h, int64_t n_steps, double t_final, int64_t *N);
void vag_serving_transport_job(vag_handle *h, int64_t k, vag::TransportJob *J);
hipEvent_t vag_serving_event(vag_handle *h, int i);
vag_status vag_serving_transport_end(vag_handle *h, vag_transport_info *info);
}

namespace vag {
// Peaceman wells (wells.hip).  wsrc[f] = c_inj Q^+ (tracer injected into face
// f per unit time), wout[f] = Q^- (volume produced); the upwind operator's
// injection entries point at the constant control volume (index nc + nf + nn,
// concentration 1) that follows the state vector.
struct WellAsm {
    int32_t nunk;
    const int32_t *frac_unk, *diag_pos, *face_grp, *face_loc, *grp_ptr, *grp_nptr;
    const int64_t *grp_off;
    double *A, *Gb, *b;
};
void launch_well_assemble(hipStream_t s, int32_t nw, const int32_t *wface, const double *wi, const double *pw,
                          const double *q, const WellAsm &g);
void launch_well_rates(hipStream_t s, int32_t nw, const int32_t *wface, const double *wi, const double *pw,
                       const double *q, const double *cinj, const double *u_frac, const double *given, double *rate,
                       double *fsrc, double *fout);
void launch_set_dirichlet(hipStream_t s, int32_t nn, int32_t offset, const uint8_t *dirichlet,
                          const double *c_bar, double *c);
// One explicit step gathered per control volume from the fluxes (no upwind
// operator); dt = dt[3], theta as in launch_transport_step.
void launch_transport_gather(hipStream_t s, int32_t nc, int32_t nf, int32_t nn, const int32_t *hex8,
                             const uint8_t *fmask, const int32_t *cell_frac, const int32_t *frac_cell,
                             const int32_t *frac_nodes, const uint8_t *dirichlet, const int32_t *node_cell_ptr,
                             const int32_t *node_cell, const int32_t *node_frac_ptr, const int32_t *node_frac,
                             const double *F_cell, const double *F_cell_frac, const double *F_frac,
                             const double *wsrc, const double *wout, const double *phi_cell, const double *phi_frac,
                             const double *phi_node, const double *dt, double theta, const double *c_in,
                             double *c_out);
// General cells (general.hip, transport.hip).  Local value array: the m x m
// Schur blocks M_K = a - r r^T / A_KK of the cells and the (k+1)^2 fracture
// blocks, at GenSym::loc_off; ga holds the cells' a with the same offsets,
// gr their row sums at unk_off.
struct GenMesh {
    int32_t nc, nf, nn;
    int max_nv, max_nf, max_fk;  // the largest cell shape (sizes the local-matrix kernel's arrays)
    const int32_t *cnode_ptr, *cnode;
    const uint8_t *cface_k, *cface_loc;
    const int32_t *cell_frac, *frac_cell, *fnode_ptr, *fnode, *unk_off;
    const int64_t *loc_off;
    int64_t ncn;  // start of the cell-face section of the flux array (the fracture-face section follows 2 nf later)
};
void launch_gen_local(hipStream_t s, const GenMesh &g, const double *xyz, const double *perm, double inv_mu,
                      double *loc, double *ga, double *gr, double *AKK, double *vol, int *bad_cell);
void launch_gen_frac_local(hipStream_t s, const GenMesh &g, const double *xyz, const double *fwidth,
                           const double *fperm, double inv_mu, double *loc, double *area);
// A at every sliced-ELL slot = sum of its contributions; b = -sum M p_bar over
// the Dirichlet columns
void launch_gen_assemble(hipStream_t s, int64_t stored, const int64_t *con_ptr, const int64_t *con,
                         const double *loc, double *A);
void launch_gen_rhs(hipStream_t s, int32_t nunk, const int32_t *bcon_ptr, const int64_t *bcon,
                    const int32_t *bcon_node, const double *loc, const double *p_bar, double *b);
void launch_gen_flux(hipStream_t s, const GenMesh &g, const double *loc, const double *ga, const double *gr,
                     const double *AKK, const double *u_node, const double *u_frac, double *u_cell, double *F);
void launch_gen_porous(hipStream_t s, const GenMesh &g, const uint8_t *dirichlet, const uint8_t *frac_node,
                       const int64_t *inc_ptr, const int32_t *inc_other, const double *vol, const double *poro,
                       const double *area, const double *fwidth, const double *fporo, const double *perm,
                       const double *fperm, const double *pmax, double *phi_cell, double *phi_frac,
                       double *phi_node);
void launch_gen_node_pmax(hipStream_t s, const GenMesh &g, const uint8_t *frac_node, const int64_t *inc_ptr,
                          const int32_t *inc_other, const double *perm, const double *fperm, double *pmax);
// transport on the incidence lists (every control volume alike)
struct GenInc {
    int32_t nc, nf, nn;
    const int64_t *ptr;
    const int32_t *edge, *other;
    const uint8_t *dirichlet;
};
void launch_gen_cfl(hipStream_t s, const GenInc &I, const double *F, const double *wout, const double *phi_cell,
                    const double *phi_frac, const double *phi_node, double cfl, double *parts, double *dt_out);
void launch_gen_upwind_count(hipStream_t s, const GenInc &I, const double *F, const double *wsrc,
                             int32_t *slice_width, uint16_t *meta, int32_t *slice_nnz);
void launch_gen_upwind_fill(hipStream_t s, const GenInc &I, const double *F, const double *wsrc, const double *wout,
                            const double *phi_cell, const double *phi_frac, const double *phi_node, const double *dt,
                            const int64_t *slice_ptr, const uint16_t *meta, int32_t *tcol, double *tval,
                            double *tdiag);

// Device address of the current device's copy of the allocation-free entry
// point's static scratch array (looked up once per device) and its size in
// doubles.
double *noalloc_scratch(size_t *doubles);

}  // namespace vag
