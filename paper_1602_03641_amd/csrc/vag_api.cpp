// C-ABI of libvag: handle lifecycle and orchestration of the device phases.
// Every entry point catches internal errors and returns a vag_status.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>

#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "amg.h"
#include "ilu.h"
#include "gmres.h"
#include "vag_internal.h"

using namespace vag;

namespace vag {

namespace {
struct DevCache {
    std::multimap<size_t, void *> free;          // block size -> free blocks
    std::unordered_map<void *, size_t> size_of;  // every block handed out or cached
};
std::mutex g_dev_mu;
DevCache g_dev[64];
int current_device() {
    int dev = 0;
    VAG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) throw Error(VAG_ERR_UNSUPPORTED, "device index beyond 63");
    return dev;
}
}  // namespace

void *dev_alloc(size_t bytes) {
    const size_t want = (bytes + 4095) & ~(size_t)4095;
    const int dev = current_device();
    {
        std::lock_guard<std::mutex> lk(g_dev_mu);
        DevCache &c = g_dev[dev];
        // the smallest cached block that fits, if it wastes at most a quarter
        auto it = c.free.lower_bound(want);
        if (it != c.free.end() && it->first <= want + want / 4 + (1u << 16)) {
            void *p = it->second;
            c.free.erase(it);
            return p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipErrorOutOfMemory) {
        // give the cached blocks back and try once more
        (void)hipGetLastError();
        VAG_HIP(hipDeviceSynchronize());
        std::vector<void *> drop;
        {
            std::lock_guard<std::mutex> lk(g_dev_mu);
            DevCache &c = g_dev[dev];
            for (auto &kv : c.free) {
                drop.push_back(kv.second);
                c.size_of.erase(kv.second);
            }
            c.free.clear();
        }
        for (void *q : drop) (void)hipFree(q);
        e = hipMalloc(&p, want);
    }
    VAG_HIP(e);
    std::lock_guard<std::mutex> lk(g_dev_mu);
    g_dev[dev].size_of[p] = want;
    return p;
}

void dev_free(void *p, hipStream_t owner_stream) {
    if (!p) return;
    // the owner's queued work may still use the block
    (void)hipStreamSynchronize(owner_stream);
    const int dev = current_device();
    std::lock_guard<std::mutex> lk(g_dev_mu);
    DevCache &c = g_dev[dev];
    auto it = c.size_of.find(p);
    if (it == c.size_of.end()) return;  // not ours: leave it alone
    c.free.emplace(it->second, p);
}

// Frees the cached blocks of the current device (the device must be idle).
void dev_trim() {
    const int dev = current_device();
    std::vector<void *> drop;
    {
        std::lock_guard<std::mutex> lk(g_dev_mu);
        DevCache &c = g_dev[dev];
        for (auto &kv : c.free) {
            drop.push_back(kv.second);
            c.size_of.erase(kv.second);
        }
        c.free.clear();
    }
    for (void *q : drop) VAG_HIP(hipFree(q));
}

namespace {
std::mutex g_pinned_mu;
std::multimap<size_t, void *> g_pinned_free;  // size class -> free blocks
size_t pinned_class(size_t bytes) {
    size_t c = 256;
    while (c < bytes) c <<= 1;
    return c;
}
}  // namespace

void *pinned_get(size_t bytes) {
    const size_t c = pinned_class(bytes);
    {
        std::lock_guard<std::mutex> lk(g_pinned_mu);
        auto it = g_pinned_free.find(c);
        if (it != g_pinned_free.end()) {
            void *p = it->second;
            g_pinned_free.erase(it);
            return p;
        }
    }
    void *p = nullptr;
    VAG_HIP(hipHostMalloc(&p, c));
    return p;
}

void pinned_put(void *p, size_t bytes) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    g_pinned_free.emplace(pinned_class(bytes), p);
}

// What a run of transport steps needs: step count, the last step's fraction
// of dt, and the figures the info reports.
struct TransportPlan {
    int64_t N = 0, total = 0;
    double dt = 0, last_dt = 0, theta_last = 1.0, dtb[3] = {};
};

}  // namespace vag

struct vag_handle {
    hipStream_t stream = nullptr;
    vag_options opt{};
    std::string err;
    Tracker tr;
    Symbolic S;
    double mu = 1.0;

    // topology
    DBuf<double> xyz;
    DBuf<int32_t> hex8, cell_frac, frac_cell, frac_slot, frac_nodes, node_unk, node_cell_ptr, node_cell,
        node_frac_ptr, node_frac, sell_col, row_len, diag_pos, unk_node, unk_face, sell_cbase;
    DBuf<uint16_t> sell_col16;  // 16-bit column offsets of the slices that allow them
    DBuf<int64_t> sell_ptr;
    // eliminated fracture-face groups
    DBuf<int32_t> frac_unk, grp_ptr, grp_face, grp_nptr, grp_node, grp_pos, face_grp, face_loc;
    DBuf<uint16_t> node_pos;  // slots of the cell-matrix columns in the node rows
    DBuf<int64_t> grp_off, grp_poff;
    DBuf<double> Gb;
    DBuf<uint8_t> fmask, dirichlet, frac_node;
    // numeric inputs
    DBuf<double> perm, poro, fwidth, fperm, fporo, p_bar, c_bar;
    // assembly
    DBuf<double> aK, rK, AKK, vol, fside, A5, area, A, b, dinv;
    DBuf<int> bad;
    DBuf<int> coef_bad;  // [2]: first cell / fracture face with invalid coefficients
    // Krylov
    DBuf<double> x, r, z, p, q, parts, rparts, scal;
    DBuf<PcgState> pcg;  // [0] the solve, [1] kernel timing (never done)
    // results
    DBuf<double> u_node, u_cell, u_frac, F_cell, F_cell_frac, F_frac, phi_cell, phi_frac, phi_node;
    // transport
    DBuf<int32_t> slice_width, slice_nnz, tcol, tbase;
    DBuf<uint16_t> tcol16;
    DBuf<uint16_t> tmeta;
    DBuf<int64_t> slice_ptr;
    DBuf<int32_t> xsplit;  // [18] the XCDs' runs of slices of the upwind operator (xlo, then ylo)
    DBuf<double> pmax;     // [nn] largest permeability around each node (alpha_rule 1)
    int32_t xlo[18] = {};  // host copy, passed to the sweep by value
    DBuf<double> tval, tdiag, cbuf0, cbuf1, dt4;
    DBuf<int64_t> tscan;  // per-block sums of the slice offsets' scan
    // pinned: [0] entry count of the upwind operator, from [2] the 18 ints of xsplit
    static constexpr int kCntWords = 16;
    unsigned long long *h_cnt = nullptr;
    int32_t *h_xsplit() { return reinterpret_cast<int32_t *>(h_cnt + 2); }
    int cur = 0;
    bool solved = false, have_flux = false, have_c = false;
    bool have_op = false;  // the upwind operator of the last vag_transport exists
    std::unique_ptr<vag::TransportPlan> plan;  // a served transport whose steps the server runs

    Amg amg;
    Ilu ilu;                 // block-Jacobi ILU(0)
    // general cells (mesh given by faces): tables of GenSym on the device,
    // local values, the cells' a and row sums, the flux array
    // [cell-node | cell-face | face-node]
    bool general = false;
    GenSym G;
    DBuf<int32_t> g_cnode_ptr, g_cnode, g_fnode_ptr, g_fnode, g_unk_off, g_bcon_ptr, g_bcon_node, g_inc_edge,
        g_inc_other;
    DBuf<uint8_t> g_cface_k, g_cface_loc;
    DBuf<int64_t> g_loc_off, g_con_ptr, g_con, g_bcon, g_inc_ptr;
    DBuf<double> gloc, ga, gr, Fall;
    GenMesh gmesh() const {
        return GenMesh{S.nc,        S.nf,      S.nn,      G.max_nv,      G.max_nf,      G.max_fk,
                       g_cnode_ptr.p, g_cnode.p, g_cface_k.p, g_cface_loc.p, cell_frac.p, frac_cell.p,
                       g_fnode_ptr.p, g_fnode.p, g_unk_off.p, g_loc_off.p, G.ncn};
    }
    GenInc ginc() const { return GenInc{S.nc, S.nf, S.nn, g_inc_ptr.p, g_inc_edge.p, g_inc_other.p, dirichlet.p}; }
    // the three flux sections (hexahedra: their own arrays)
    double *flux_cell() { return general ? Fall.p : F_cell.p; }
    double *flux_cell_frac() { return general ? Fall.p + G.ncn : F_cell_frac.p; }
    double *flux_frac() { return general ? Fall.p + G.ncn + 2 * (int64_t)S.nf : F_frac.p; }
    int64_t n_flux_cell() const { return general ? G.ncn : 8 * (int64_t)S.nc; }
    int64_t n_flux_frac() const { return general ? G.nfn : 4 * (int64_t)S.nf; }
    // Peaceman wells: perforations, rates of the last solve, per-face terms
    int32_t nw = 0;
    DBuf<int32_t> wface;
    DBuf<double> wwi, wpw, wq, wcinj, wrate, wgiven, wsrc, wout;
    const double *well_src() const { return nw ? wsrc.p : nullptr; }
    const double *well_out() const { return nw ? wout.p : nullptr; }
    DBuf<int> ilu_bad;       // 1 + natural row of a zero pivot, else 0
    DBuf<float> b32, x32, r32, z32, p32, q32;  // inner single-precision solve (VAG_MIXED)
    // GMRES(m) work: FP64 basis (VAG_FP64 / VAG_MIXED) or FP32 basis (inner solves of VAG_MIXED_IR)
    DBuf<double> gmV, gmZ, gmw, gmt, gmparts, gmnparts, gmhd;
    DBuf<float> gmV32, gmZ32, gmw32, gmt32;
    // BiCGStab work (p, phat, v are p, z, q)
    DBuf<double> bcg_rhat, bcg_s, bcg_shat, bcg_t, bcg_parts;
    double *h_gm = nullptr;
    int h_gm_m = 0;
    int last_outer = 1, last_inner = 0;
    PcgState *h_pcg = nullptr;
    double *h_scal = nullptr;
    hipEvent_t ev[8] = {};

    Sell<double> Asell() const { return with_col16(A.p); }
    // the system pattern with the matrix values v
    Sell<double> with_col16(const double *v) const {
        Sell<double> m{S.nunk, sell_ptr.p, sell_col.p, v};
        m.col16 = sell_col16.p;
        m.cbase = sell_cbase.p;
        m.nt = stream_matrix((int64_t)A.n, sizeof(double), opt.stream_loads);
        return m;
    }
    UpwindOp upwind() const {
        UpwindOp T{S.nc + S.nf + S.nn, slice_ptr.p, tmeta.p, tcol.p, tcol16.p, tbase.p, tval.p, tdiag.p, {}, {}};
        for (int x = 0; x < 9; ++x) {
            T.xlo[x] = xlo[x];
            T.ylo[x] = xlo[9 + x];
        }
        return T;
    }
    double *c_cur() { return cur ? cbuf1.p : cbuf0.p; }
    double *c_next() { return cur ? cbuf0.p : cbuf1.p; }

    ~vag_handle() {
        pinned_put(h_pcg, sizeof(PcgState));
        pinned_put(h_scal, 16 * sizeof(double));
        pinned_put(h_cnt, kCntWords * sizeof(unsigned long long));
        pinned_put(h_gm, (3 * (size_t)(h_gm_m + 1) + 1) * sizeof(double));
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace {

thread_local std::string g_create_error;

template <class F>
vag_status guard(vag_handle *h, F &&fn) {
    try {
        fn();
        if (h) h->err.clear();
        return VAG_OK;
    } catch (const Error &e) {
        if (h) h->err = e.what();
        return e.status;
    } catch (const std::bad_alloc &) {
        if (h) h->err = "host allocation failed";
        return VAG_ERR_OOM;
    } catch (const std::exception &e) {
        if (h) h->err = e.what();
        return VAG_ERR_ARG;
    }
}

hipMemcpyKind kind_in(vag_mem m) { return m == VAG_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }
hipMemcpyKind kind_out(vag_mem m) { return m == VAG_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }

template <class T>
void upload(vag_handle *h, DBuf<T> &d, const T *src, size_t n, vag_mem mem) {
    if (!n) return;
    if (!src) throw Error(VAG_ERR_ARG, "null input array");
    if (d.n < n) d.alloc(n, h->tr);
    VAG_HIP(hipMemcpyAsync(d.p, src, n * sizeof(T), kind_in(mem), h->stream));
    if (mem == VAG_MEM_HOST) VAG_HIP(hipStreamSynchronize(h->stream));
}

template <class T, class A>
void upload_vec(vag_handle *h, DBuf<T> &d, const std::vector<T, A> &v) {
    d.alloc(v.size(), h->tr);
    if (v.empty()) return;
    // on the handle's stream: a worker stream created non-blocking is not
    // ordered after the null stream that hipMemcpy would use
    VAG_HIP(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, h->stream));
    VAG_HIP(hipStreamSynchronize(h->stream));
}

template <class T>
void download(vag_handle *h, T *dst, const DBuf<T> &d, size_t n, vag_mem mem) {
    if (!dst || !n) return;
    VAG_HIP(hipMemcpyAsync(dst, d.p, n * sizeof(T), kind_out(mem), h->stream));
}

// host copy of an input that may live in device memory
template <class T>
std::vector<T> host_copy(const T *src, size_t n, vag_mem mem, hipStream_t s) {
    std::vector<T> v(n);
    if (n) {
        if (!src) throw Error(VAG_ERR_ARG, "null input array");
        if (mem == VAG_MEM_DEVICE) {
            VAG_HIP(hipMemcpyAsync(v.data(), src, n * sizeof(T), hipMemcpyDeviceToHost, s));
            VAG_HIP(hipStreamSynchronize(s));
        } else
            std::memcpy(v.data(), src, n * sizeof(T));
    }
    return v;
}

void check_options(const vag_options &o) {
    if (!(o.rtol > 0) || o.max_iter < 0 || !(o.cfl > 0) || o.check_every <= 0)
        throw Error(VAG_ERR_ARG, "invalid options (rtol, max_iter, cfl or check_every)");
    if (o.precision != VAG_FP64 && o.precision != VAG_MIXED && o.precision != VAG_MIXED_IR)
        throw Error(VAG_ERR_ARG, "unknown precision");
    if (o.precision != VAG_FP64 && o.precond != VAG_PC_AMG)
        throw Error(VAG_ERR_UNSUPPORTED, "mixed precision needs the AMG preconditioner");
    if (o.precision == VAG_MIXED_IR && !(o.inner_rtol > 0 && o.inner_rtol < 1))
        throw Error(VAG_ERR_ARG, "inner_rtol must lie in (0, 1)");
    if (o.amg_kcycle < 0 || o.amg_kcycle > 12) throw Error(VAG_ERR_ARG, "amg_kcycle must lie in [0, 12]");
    if (o.amg_kind != 0 && o.amg_kind != 1) throw Error(VAG_ERR_ARG, "amg_kind must be 0 (aggregation) or 1 (classical)");
    if (!(o.amg_strong_theta >= 0 && o.amg_strong_theta < 1))
        throw Error(VAG_ERR_ARG, "amg_strong_theta must lie in [0, 1) (0: default)");
    if (o.amg_aggregate_hops < 0 || o.amg_aggregate_hops > 2)
        throw Error(VAG_ERR_ARG, "amg_aggregate_hops must be 0 (default), 1 or 2");
    if (o.krylov != VAG_CG && o.krylov != VAG_GMRES && o.krylov != VAG_BICGSTAB)
        throw Error(VAG_ERR_ARG, "unknown Krylov method");
    if (o.stream_loads < 0 || o.stream_loads > 2)
        throw Error(VAG_ERR_ARG, "stream_loads must be 0 (automatic), 1 (always) or 2 (never)");
    if (o.alpha_rule < 0 || o.alpha_rule > 1)
        throw Error(VAG_ERR_ARG, "alpha_rule must be 0 (every adjacent cell or face) or 1 (largest permeability)");
    if (o.krylov == VAG_BICGSTAB && o.precision == VAG_MIXED_IR)
        throw Error(VAG_ERR_UNSUPPORTED, "BiCGStab runs in FP64 (with the FP64 or FP32 hierarchy), not as an inner solver");
    if (o.krylov == VAG_GMRES && (o.gmres_restart < 1 || o.gmres_restart > 1024))
        throw Error(VAG_ERR_ARG, "gmres_restart must lie in [1, 1024]");
    if (o.precond != VAG_PC_JACOBI && o.precond != VAG_PC_AMG && o.precond != VAG_PC_BJILU0)
        throw Error(VAG_ERR_ARG, "unknown preconditioner");
    if (o.precond == VAG_PC_BJILU0 && o.krylov == VAG_CG)
        throw Error(VAG_ERR_UNSUPPORTED, "block-Jacobi ILU(0) is not symmetric: use GMRES or BiCGStab");
    if (o.ilu_block_rows < 0 || o.ilu_block_rows > kIluMaxBlock)
        throw Error(VAG_ERR_ARG, "ilu_block_rows must lie in [0, " + std::to_string(kIluMaxBlock) + "]");
}

// z = M^{-1} r for the handle's preconditioner (see Amg::apply for x_ready, rz)
void precond_apply(vag_handle *h, const double *r, double *z, const PcgState *st, bool x_ready = false,
                   double *rz = nullptr, double *zq = nullptr, const double *qv = nullptr);

// device pointers of the assembly kernels
AsmArgs asm_args(vag_handle *h) {
    const Symbolic &S = h->S;
    AsmArgs g{};
    g.nc = S.nc;
    g.nfree = S.nfree;
    g.nsys = S.nunk;
    g.hex8 = h->hex8.p;
    g.node_unk = h->node_unk.p;
    g.frac_unk = h->frac_unk.p;
    g.unk_node = h->unk_node.p;
    g.unk_face = h->unk_face.p;
    g.node_cell_ptr = h->node_cell_ptr.p;
    g.node_cell = h->node_cell.p;
    g.node_frac_ptr = h->node_frac_ptr.p;
    g.node_frac = h->node_frac.p;
    g.fmask = h->fmask.p;
    g.cell_frac = h->cell_frac.p;
    g.frac_cell = h->frac_cell.p;
    g.frac_nodes = h->frac_nodes.p;
    g.aK = h->aK.p;
    g.rK = h->rK.p;
    g.AKK = h->AKK.p;
    g.fside = h->fside.p;
    g.A5 = h->A5.p;
    g.p_bar = h->p_bar.p;
    g.node_pos = h->node_pos.p;
    g.sell_ptr = h->sell_ptr.p;
    g.sell_col = h->sell_col.p;
    g.row_len = h->row_len.p;
    g.grp_ptr = h->grp_ptr.p;
    g.grp_face = h->grp_face.p;
    g.grp_nptr = h->grp_nptr.p;
    g.grp_node = h->grp_node.p;
    g.face_grp = h->face_grp.p;
    g.face_loc = h->face_loc.p;
    g.grp_off = h->grp_off.p;
    g.A = h->A.p;
    g.Gb = h->Gb.p;
    g.b = h->b.p;
    g.bad = h->bad.p;
    return g;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) ms = 0.f;
    return ms;
}

}  // namespace

namespace {
void precond_apply(vag_handle *h, const double *r, double *z, const PcgState *st, bool x_ready, double *rz,
                   double *zq, const double *qv) {
    if (h->opt.precond == VAG_PC_AMG && h->opt.precision == VAG_MIXED)
        h->amg.apply_mixed(h->stream, r, z, st, x_ready, rz, zq, qv);
    else if (h->opt.precond == VAG_PC_AMG)
        h->amg.apply(h->stream, r, z, st, x_ready, rz, zq, qv);
    else if (h->opt.precond == VAG_PC_BJILU0)
        h->ilu.apply(h->stream, r, z, st);
    else
        launch_jacobi(h->stream, h->S.nunk, h->dinv.p, r, z);
}

AmgOptions amg_options(const vag_options &o) {
    AmgOptions a;
    if (o.amg_theta > 0) a.theta = o.amg_theta;
    if (o.amg_coarse_size > 0) a.coarse_size = o.amg_coarse_size;
    if (o.amg_max_levels > 0) a.max_levels = o.amg_max_levels;
    if (o.amg_sweeps > 0) a.sweeps = o.amg_sweeps;
    if (o.amg_aggregate_hops > 0) a.hops = o.amg_aggregate_hops;
    a.kind = o.amg_kind;
    if (o.amg_strong_theta > 0) a.strong_theta = o.amg_strong_theta;
    // K-cycles make the preconditioner nonlinear: CG runs in its flexible form
    // and GMRES is flexible; BiCGStab and the FP32 inner solves keep V-cycles
    a.kcycle = ((o.krylov == VAG_CG || o.krylov == VAG_GMRES) && o.precision != VAG_MIXED_IR) ? o.amg_kcycle : 0;
    return a;
}

// Preconditioned CG from x = 0 on the device; the host only queues iterations
// and reads the state every check_every iterations.  When the recurrence
// residual meets rtol but the true residual does not (rounding drift), CG
// restarts from the current x with the remaining reduction as its target.
void run_pcg(vag_handle *h) {
    hipStream_t s = h->stream;
    const int32_t n = h->S.nunk;
    const PcgParts P{h->parts.p, pcg_grid(n)};
    PcgState *st = h->pcg.p;
    const bool jacobi = h->opt.precond == VAG_PC_JACOBI;
    // the aggregation V-cycle takes D^-1 r from the update kernel and returns
    // the partials of r.z; the classical one runs apart
    const bool fused = !jacobi && h->amg.nlev > 1 && !h->amg.classical();
    const bool flexible = fused && h->amg.nonlinear();
    const Sell<double> A = h->Asell();
    const int max_iter = h->opt.max_iter;
    int k = 0, k0 = 0;
    double rtol = h->opt.rtol, bb = -1.0;
    for (int restart = 0;; ++restart) {
        if (restart == 0) {
            launch_pcg_init(s, n, h->b.p, jacobi ? h->dinv.p : nullptr, h->x.p, h->r.p, h->z.p, P);
        } else {
            launch_pcg_init_warm(s, A, k0, h->b.p, h->x.p, h->r.p, jacobi ? h->dinv.p : nullptr, h->z.p, P);
        }
        if (!jacobi) {
            precond_apply(h, h->r.p, h->z.p, nullptr);
            launch_pcg_dot_rz<double>(s, n, k0 - 1, h->r.p, h->z.p, P, nullptr);
        }
        launch_pcg_start(s, P, st, rtol, k0);
        for (;;) {
            const int kend = std::min(k + h->opt.check_every, max_iter);
            for (; k < kend; ++k) {
                launch_pcg_direction<double>(s, n, k, k0, h->z.p, h->p.p, P, st, true, flexible);
                launch_pcg_spmv<double, double>(s, A, h->p.p, h->q.p, P, st);
                if (jacobi) {
                    launch_pcg_update(s, n, k, h->x.p, h->r.p, h->z.p, h->p.p, h->q.p, h->dinv.p, P, st);
                } else {
                    if (fused) {
                        // the update also writes the V-cycle's first iterate D^-1 r, and
                        // the V-cycle's last sweep the partials of r.z
                        launch_pcg_update_xr<double>(s, n, k, h->x.p, h->r.p, h->p.p, h->q.p, P, st,
                                                     h->amg.L[0]->dinv.p, h->amg.L[0]->xa.p);
                        precond_apply(h, h->r.p, h->z.p, st, true, P.rz(k), flexible ? P.zq() : nullptr,
                                      flexible ? h->q.p : nullptr);
                    } else {
                        launch_pcg_update_xr<double>(s, n, k, h->x.p, h->r.p, h->p.p, h->q.p, P, st);
                        precond_apply(h, h->r.p, h->z.p, st);
                        launch_pcg_dot_rz<double>(s, n, k, h->r.p, h->z.p, P, st);
                    }
                }
            }
            if (k >= max_iter) launch_pcg_direction<double>(s, n, k, k0, h->z.p, h->p.p, P, st, false);
            VAG_HIP(hipMemcpyAsync(h->h_pcg, st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
            VAG_HIP(hipStreamSynchronize(s));
            if (h->h_pcg->done || k >= max_iter) break;
        }
        k = h->h_pcg->iter;
        if (!h->h_pcg->converged || k >= max_iter) break;
        // true residual check
        launch_residual_norm(s, A, h->x.p, h->b.p, h->q.p, h->rparts.p, h->scal.p);
        VAG_HIP(hipMemcpyAsync(h->h_scal, h->scal.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        VAG_HIP(hipStreamSynchronize(s));
        if (bb < 0) bb = h->h_scal[1];
        const double rr = h->h_scal[0];
        if (rr <= h->opt.rtol * h->opt.rtol * bb) break;
        if (restart >= 3) {  // the true residual stays above rtol (rounding floor): report it
            h->h_pcg->converged = 0;
            break;
        }
        rtol = std::min(0.5, h->opt.rtol * std::sqrt(bb / rr));
        k0 = k;
    }
    h->last_inner = h->h_pcg->iter;
    h->last_outer = 1;
}

// Right-preconditioned BiCGStab from x = 0 with device-resident scalars; the
// host reads the state every check_every iterations.  A true-residual check
// and up to three warm restarts, as for CG.
void run_bicgstab(vag_handle *h) {
    hipStream_t s = h->stream;
    const int32_t n = h->S.nunk;
    const size_t nv = (size_t)std::max(n, 1);
    for (auto *v : {&h->bcg_rhat, &h->bcg_s, &h->bcg_shat, &h->bcg_t}) ensure(*v, nv, h->tr);
    ensure(h->bcg_parts, 8 * (size_t)kReduceBlocks, h->tr);
    double *parts = h->bcg_parts.p;
    PcgState *st = h->pcg.p;
    const Sell<double> A = h->Asell();
    const int max_iter = h->opt.max_iter;
    int k = 0, k0 = 0;
    double rtol = h->opt.rtol, bb = -1.0;
    for (int restart = 0;; ++restart) {
        launch_bcg_init(s, A, restart == 0, k0, h->b.p, h->x.p, h->r.p, h->bcg_rhat.p, parts);
        launch_bcg_start(s, n, parts, st, rtol, k0);
        for (;;) {
            const int kend = std::min(k + h->opt.check_every, max_iter);
            for (; k < kend; ++k) {
                launch_bcg_direction(s, n, k, k0, h->r.p, h->p.p, h->q.p, parts, st, true);
                precond_apply(h, h->p.p, h->z.p, st);
                launch_bcg_spmv_v(s, A, h->z.p, h->q.p, h->bcg_rhat.p, parts, st);
                launch_bcg_s(s, n, k, h->r.p, h->q.p, h->z.p, h->bcg_s.p, h->x.p, parts, st);
                precond_apply(h, h->bcg_s.p, h->bcg_shat.p, st);
                launch_bcg_spmv_t(s, A, h->bcg_shat.p, h->bcg_t.p, h->bcg_s.p, parts, st);
                launch_bcg_update(s, n, k, h->z.p, h->bcg_shat.p, h->bcg_s.p, h->bcg_t.p, h->bcg_rhat.p, h->x.p,
                                  h->r.p, parts, st);
            }
            // convergence test of the last residual without a new direction
            launch_bcg_direction(s, n, k, k0, h->r.p, h->p.p, h->q.p, parts, st, false);
            VAG_HIP(hipMemcpyAsync(h->h_pcg, st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
            VAG_HIP(hipStreamSynchronize(s));
            if (h->h_pcg->done || k >= max_iter) break;
        }
        k = h->h_pcg->iter;
        if (!h->h_pcg->converged || k >= max_iter) break;
        launch_residual_norm(s, A, h->x.p, h->b.p, h->q.p, h->rparts.p, h->scal.p);
        VAG_HIP(hipMemcpyAsync(h->h_scal, h->scal.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        VAG_HIP(hipStreamSynchronize(s));
        if (bb < 0) bb = h->h_scal[1];
        const double rr = h->h_scal[0];
        if (rr <= h->opt.rtol * h->opt.rtol * bb) break;
        if (restart >= 3) {  // the true residual stays above rtol (rounding floor): report it
            h->h_pcg->converged = 0;
            break;
        }
        rtol = std::min(0.5, h->opt.rtol * std::sqrt(bb / rr));
        k0 = k;
    }
    h->last_inner = h->h_pcg->iter;
    h->last_outer = 1;
}

// Scratch of GMRES(m) on n unknowns with vectors of type T.
template <class T>
GmresWork<T> gmres_work(vag_handle *h, int32_t n, DBuf<T> &V, DBuf<T> &Z, DBuf<T> &w, DBuf<T> &t) {
    const int m = h->opt.gmres_restart;
    Tracker &tr = h->tr;
    ensure(V, (size_t)(m + 1) * (size_t)std::max(n, 1), tr);
    ensure(Z, (size_t)m * (size_t)std::max(n, 1), tr);
    ensure(w, (size_t)std::max(n, 1), tr);
    ensure(t, (size_t)std::max(n, 1), tr);
    ensure(h->gmparts, (size_t)(m + 1) * gmres_grid(n), tr);
    ensure(h->gmnparts, (size_t)gmres_grid(n), tr);
    ensure(h->gmhd, (size_t)3 * (m + 1) + 1, tr);
    if (h->h_gm_m < m) {
        pinned_put(h->h_gm, (3 * (size_t)(h->h_gm_m + 1) + 1) * sizeof(double));
        h->h_gm = nullptr;
        h->h_gm = static_cast<double *>(pinned_get((3 * (size_t)(m + 1) + 1) * sizeof(double)));
        h->h_gm_m = m;
    }
    GmresWork<T> W;
    W.V = V.p;
    W.Z = Z.p;
    W.w = w.p;
    W.t = t.p;
    W.parts = h->gmparts.p;
    W.nparts = h->gmnparts.p;
    W.hd = h->gmhd.p;
    W.hh = h->h_gm;
    return W;
}

// Flexible GMRES(m) from x = 0 in FP64 (the preconditioner may be
// the FP32 hierarchy of VAG_MIXED).
void run_gmres(vag_handle *h) {
    hipStream_t s = h->stream;
    const int32_t n = h->S.nunk;
    const GmresWork<double> W = gmres_work<double>(h, n, h->gmV, h->gmZ, h->gmw, h->gmt);
    launch_fill(s, n, 0.0, h->x.p);
    launch_residual_norm(s, h->Asell(), h->x.p, h->b.p, h->r.p, h->rparts.p, h->scal.p);
    VAG_HIP(hipMemcpyAsync(h->h_scal, h->scal.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    VAG_HIP(hipStreamSynchronize(s));
    const double tol = h->opt.rtol * std::sqrt(h->h_scal[1]);
    const GmresResult R = gmres_solve<double, double>(
        s, h->Asell(), h->b.p, h->x.p, tol, h->opt.gmres_restart, h->opt.max_iter, W,
        [&](const double *in, double *out) { precond_apply(h, in, out, nullptr); });
    h->h_pcg->iter = R.iterations;
    h->h_pcg->converged = R.converged;
    h->h_pcg->done = 1;
    h->last_inner = R.iterations;
    h->last_outer = 1;
}

// FP64 iterative refinement: r = b - A x in FP64; the correction solves
// A d = r / ||r|| by CG or GMRES in FP32 (the FP32 copy of A, FP64 diagonal)
// preconditioned by the FP32 hierarchy of A, to inner_rtol, then x += ||r|| d
// in FP64.  Stops when ||r|| <= rtol ||b||.  The hierarchy is that of A
// itself: its piecewise-constant interpolation carries the constants, the
// near-null space of A, which a diagonally rescaled matrix would not have.
void run_mixed(vag_handle *h) {
    hipStream_t s = h->stream;
    const int32_t n = h->S.nunk;
    const PcgParts P{h->parts.p, pcg_grid(n)};
    PcgState *st = h->pcg.p;
    Tracker &tr = h->tr;
    for (auto *v : {&h->b32, &h->x32, &h->r32, &h->z32, &h->p32, &h->q32}) ensure(*v, (size_t)std::max(n, 1), tr);
    h->amg.stream_mode = h->opt.stream_loads;
    h->amg.make_fp32(s, tr, nullptr);
    const Sell<float> A32 = h->amg.L[0]->A32;
    launch_fill(s, n, 0.0, h->x.p);
    launch_residual_norm(s, h->Asell(), h->x.p, h->b.p, h->r.p, h->rparts.p, h->scal.p);
    VAG_HIP(hipMemcpyAsync(h->h_scal, h->scal.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    VAG_HIP(hipStreamSynchronize(s));
    const double bb = h->h_scal[1];
    double rr = h->h_scal[0];
    const double tol2 = h->opt.rtol * h->opt.rtol * bb;
    int inner_total = 0, outer = 0;
    bool converged = (rr <= tol2);
    while (!converged && inner_total < h->opt.max_iter) {
        ++outer;
        launch_norm2(s, n, h->r.p, h->rparts.p, h->scal.p + 2);
        launch_normalize_to_float(s, n, h->r.p, h->scal.p + 2, h->b32.p);
        if (h->opt.krylov == VAG_GMRES) {
            // inner FP32 GMRES, ||b32|| = 1: one cycle of at most m iterations that
            // stops when the Arnoldi estimate of its residual reaches inner_rtol.
            // The true FP32 residual of an FP32 iterate cannot fall much below
            // ||A|| ||x|| eps_32 / ||b|| (about 1e-2 at contrast 1e6), so restarts
            // from it would stall; the FP64 refinement takes over instead.
            const GmresWork<float> W = gmres_work<float>(h, n, h->gmV32, h->gmZ32, h->gmw32, h->gmt32);
            VAG_HIP(hipMemsetAsync(h->x32.p, 0, (size_t)n * sizeof(float), s));
            const int cycle = std::min(h->opt.gmres_restart, h->opt.max_iter - inner_total);
            const GmresResult R = gmres_solve<float, float>(
                s, A32, h->b32.p, h->x32.p, h->opt.inner_rtol, h->opt.gmres_restart, cycle, W,
                [&](const float *in, float *out) { h->amg.apply32(s, in, out, nullptr); });
            inner_total += std::max(R.iterations, 1);
            launch_correct(s, n, h->x.p, h->x32.p, h->scal.p + 2);
            launch_residual_norm(s, h->Asell(), h->x.p, h->b.p, h->r.p, h->rparts.p, h->scal.p);
            VAG_HIP(hipMemcpyAsync(h->h_scal, h->scal.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
            VAG_HIP(hipStreamSynchronize(s));
            rr = h->h_scal[0];
            converged = (rr <= tol2);
            continue;
        }
        launch_pcg_init_plain<float>(s, n, h->b32.p, h->x32.p, h->r32.p, P);
        h->amg.apply32(s, h->r32.p, h->z32.p, nullptr);
        launch_pcg_dot_rz<float>(s, n, -1, h->r32.p, h->z32.p, P, nullptr);
        launch_pcg_start(s, P, st, h->opt.inner_rtol, 0);
        const int budget = h->opt.max_iter - inner_total;
        int k = 0;
        for (;;) {
            const int kend = std::min(k + h->opt.check_every, budget);
            for (; k < kend; ++k) {
                launch_pcg_direction<float>(s, n, k, 0, h->z32.p, h->p32.p, P, st, true);
                launch_pcg_spmv<float, float>(s, A32, h->p32.p, h->q32.p, P, st);
                launch_pcg_update_xr<float>(s, n, k, h->x32.p, h->r32.p, h->p32.p, h->q32.p, P, st);
                h->amg.apply32(s, h->r32.p, h->z32.p, st);
                launch_pcg_dot_rz<float>(s, n, k, h->r32.p, h->z32.p, P, st);
            }
            if (k >= budget) launch_pcg_direction<float>(s, n, k, 0, h->z32.p, h->p32.p, P, st, false);
            VAG_HIP(hipMemcpyAsync(h->h_pcg, st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
            VAG_HIP(hipStreamSynchronize(s));
            if (h->h_pcg->done || k >= budget) break;
        }
        inner_total += std::max(h->h_pcg->iter, 1);
        launch_correct(s, n, h->x.p, h->x32.p, h->scal.p + 2);
        launch_residual_norm(s, h->Asell(), h->x.p, h->b.p, h->r.p, h->rparts.p, h->scal.p);
        VAG_HIP(hipMemcpyAsync(h->h_scal, h->scal.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        VAG_HIP(hipStreamSynchronize(s));
        rr = h->h_scal[0];
        converged = (rr <= tol2);
    }
    h->h_pcg->iter = inner_total;
    h->h_pcg->converged = converged;
    h->h_pcg->done = 1;
    h->last_inner = inner_total;
    h->last_outer = outer;
}

// Porous volumes of the control volumes (§3.2.1) on the handle's stream;
// with alpha_rule 1 the largest permeability around each node first.
void porous_volumes(vag_handle *h, hipStream_t s) {
    const Symbolic &S = h->S;
    const double *pmax = nullptr;
    if (h->opt.alpha_rule == 1) {
        ensure(h->pmax, (size_t)std::max(S.nn, 1), h->tr);
        if (h->general)
            launch_gen_node_pmax(s, h->gmesh(), h->frac_node.p, h->g_inc_ptr.p, h->g_inc_other.p, h->perm.p,
                                 h->fperm.p, h->pmax.p);
        else
            launch_node_pmax(s, S.nn, h->frac_node.p, h->node_cell_ptr.p, h->node_cell.p, h->node_frac_ptr.p,
                             h->node_frac.p, h->perm.p, h->fperm.p, h->pmax.p);
        pmax = h->pmax.p;
    }
    if (h->general)
        launch_gen_porous(s, h->gmesh(), h->dirichlet.p, h->frac_node.p, h->g_inc_ptr.p, h->g_inc_other.p, h->vol.p,
                          h->poro.p, h->area.p, h->fwidth.p, h->fporo.p, h->perm.p, h->fperm.p, pmax, h->phi_cell.p,
                          h->phi_frac.p, h->phi_node.p);
    else
        launch_porous(s, S.nc, S.nf, S.nn, h->hex8.p, h->frac_nodes.p, h->dirichlet.p, h->frac_node.p,
                      h->node_cell_ptr.p, h->node_cell.p, h->node_frac_ptr.p, h->node_frac.p, h->vol.p, h->poro.p,
                      h->area.p, h->fwidth.p, h->fporo.p, h->perm.p, h->fperm.p, pmax, h->phi_cell.p, h->phi_frac.p,
                      h->phi_node.p);
}
}  // namespace

namespace {
// From host memory a copy holds the calling thread; so vag_create sends the
// per-node and per-cell coefficients up from a thread (and stream) of their
// own while it builds the system pattern, and waits for them at its end.
struct InputUploads {
    struct Copy {
        void *dst;
        const void *src;
        size_t bytes;
    };
    std::vector<Copy> copies;
    std::thread th;
    bool failed = false;
    template <class T>
    void add(vag_handle *h, DBuf<T> &d, const T *src, size_t n) {
        if (!n) return;
        if (!src) throw Error(VAG_ERR_ARG, "null input array");
        if (d.n < n) d.alloc(n, h->tr);
        copies.push_back(Copy{d.p, src, n * sizeof(T)});
    }
    void start() {
        int dev = 0;
        VAG_HIP(hipGetDevice(&dev));
        th = std::thread([this, dev] {
            hipStream_t us = nullptr;
            bool ok = hipSetDevice(dev) == hipSuccess && hipStreamCreateWithFlags(&us, hipStreamNonBlocking) == hipSuccess;
            for (const Copy &c : copies)
                ok = ok && hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyHostToDevice, us) == hipSuccess;
            if (us) {
                ok = hipStreamSynchronize(us) == hipSuccess && ok;
                (void)hipStreamDestroy(us);
            }
            failed = !ok;
        });
    }
    void finish() {
        if (th.joinable()) th.join();
        if (failed) throw Error(VAG_ERR_HIP, "uploading the coefficients failed");
    }
    ~InputUploads() {
        if (th.joinable()) th.join();
    }
};
}  // namespace

extern "C" {

const char *vag_version(void) { return "libvag 0.1 (gfx950)"; }

vag_status vag_default_options(vag_options *o) {
    if (!o) return VAG_ERR_ARG;
    std::memset(o, 0, sizeof *o);
    o->precision = VAG_FP64;
    o->krylov = VAG_CG;
    o->precond = VAG_PC_JACOBI;
    o->rtol = 1e-8;
    o->inner_rtol = 1e-4;
    o->max_iter = 20000;
    o->gmres_restart = 100;
    o->check_every = 16;
    o->cfl = 0.9;
    o->amg_coarse_size = 1000;
    o->amg_max_levels = 12;
    o->amg_theta = 0.02;
    o->amg_sweeps = 1;
    o->amg_kcycle = 2;
    o->eliminate_frac_faces = 1;
    return VAG_OK;
}

namespace {
// The system pattern of a hexahedral mesh, built on the device from what the
// host symbolic phase left (natural numbering): row bounds, scan, rows and
// their lengths; the host then renumbers the rows from the lengths alone
// (finish_symbolic_lengths), and the rows are mapped and sorted into rp/cl
// (CSR, system numbering).  Needs h->hex8 and the node -> cell lists on the
// device; uploads fmask, cell_frac and frac_cell for good.
void device_pattern(vag_handle *h, DBuf<int32_t> &rp, DBuf<int32_t> &cl) {
    Symbolic &S = h->S;
    hipStream_t s = h->stream;
    const int32_t n = S.nunk;
    upload_vec(h, h->fmask, S.fmask);
    upload_vec(h, h->cell_frac, S.cell_frac);
    upload_vec(h, h->frac_cell, S.frac_cell);
    std::vector<int32_t> len((size_t)n);
    DBuf<int32_t> raw;
    DBuf<int64_t> off;
    if (n > 0) {
        DBuf<int32_t> nu, fu, ngp_ptr, ngp, gnp, gn, ub, dlen;
        upload_vec(h, nu, S.node_unk);
        upload_vec(h, fu, S.frac_unk);
        upload_vec(h, ngp_ptr, S.node_grp_ptr);
        upload_vec(h, ngp, S.node_grp);
        upload_vec(h, gnp, S.grp_nptr);
        upload_vec(h, gn, S.grp_node);
        const PatArgs g{S.nn,     S.nf,        n,         h->hex8.p,       h->node_cell_ptr.p,
                        h->node_cell.p, nu.p,  fu.p,      h->cell_frac.p,  h->frac_cell.p,
                        h->fmask.p, ngp_ptr.p, ngp.p,     gnp.p,           gn.p};
        ub.alloc(n, h->tr);
        dlen.alloc(n, h->tr);
        off.alloc((size_t)n + 1, h->tr);
        DBuf<int64_t> sums;
        sums.alloc((size_t)n / 1024 + 2, h->tr);
        launch_pattern_bound(s, g, ub.p);
        launch_scan64(s, n, ub.p, off.p, sums.p);
        int64_t total = 0;
        VAG_HIP(hipMemcpyAsync(&total, off.p + n, sizeof total, hipMemcpyDeviceToHost, s));
        VAG_HIP(hipStreamSynchronize(s));
        raw.alloc((size_t)std::max<int64_t>(total, 1), h->tr);
        launch_pattern_rows(s, g, off.p, raw.p, dlen.p);
        VAG_HIP(hipMemcpyAsync(len.data(), dlen.p, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        VAG_HIP(hipStreamSynchronize(s));
    }
    finish_symbolic_lengths(S, len.data());
    upload_vec(h, rp, S.row_ptr);
    cl.alloc((size_t)std::max<int64_t>(S.nnz, 1), h->tr);
    if (n > 0) {
        DBuf<int32_t> so, sn;
        upload_vec(h, so, S.sys_old);
        upload_vec(h, sn, S.sys_new);
        launch_pattern_sort(s, n, rp.p, so.p, off.p, raw.p, sn.p, cl.p);
        VAG_HIP(hipStreamSynchronize(s));  // before the temporaries go
    }
}

// The sorted CSR columns on the host for the few host consumers (the
// block-ILU build, the system export), read back from the sliced-ELL columns
// where the device built the pattern.
void host_pattern(vag_handle *h) {
    Symbolic &S = h->S;
    if (S.col_on_host) return;
    const int32_t n = S.nunk;
    std::vector<int32_t> sc((size_t)std::max<int64_t>(S.sell_ptr.back(), 1)), rl((size_t)std::max(n, 1));
    VAG_HIP(hipMemcpyAsync(sc.data(), h->sell_col.p, sc.size() * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    VAG_HIP(hipMemcpyAsync(rl.data(), h->row_len.p, rl.size() * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    VAG_HIP(hipStreamSynchronize(h->stream));
    uvector<int32_t> col((size_t)S.nnz);
    for (int32_t r = 0; r < n; ++r) {
        const int32_t len = S.row_ptr[r + 1] - S.row_ptr[r];
        if (rl[r] != len) throw Error(VAG_ERR_HIP, "device pattern does not match its row lengths");
        const int64_t base = S.sell_ptr[r / kSliceRows] + r % kSliceRows;
        for (int32_t k = 0; k < len; ++k) col[(size_t)S.row_ptr[r] + k] = sc[base + (int64_t)k * kSliceRows];
    }
    S.col.swap(col);
    S.col_on_host = true;
}
}  // namespace

vag_status vag_create(const vag_mesh *mesh, const vag_fractures *frac, const vag_rock *rock, const vag_bc *bc,
                      const vag_options *opt, vag_mem mem, void *hip_stream, vag_handle **out) {
    if (!out) return VAG_ERR_ARG;
    *out = nullptr;
    vag_handle *h = nullptr;
    try {
        h = new vag_handle();
    } catch (...) {
        g_create_error = "host allocation failed";
        return VAG_ERR_OOM;
    }
    vag_status st = guard(h, [&] {
        Phases ph("vag.create");
        if (!mesh || !rock || !bc) throw Error(VAG_ERR_ARG, "mesh, rock and bc are required");
        if (!(rock->mu > 0)) throw Error(VAG_ERR_ARG, "viscosity must be positive");
        h->stream = reinterpret_cast<hipStream_t>(hip_stream);
        h->tr.stream = h->stream;
        if (opt) h->opt = *opt; else vag_default_options(&h->opt);
        check_options(h->opt);
        const int64_t nn = mesh->n_nodes, nc = mesh->n_cells, nf = frac ? frac->n_frac : 0;
        if (nn <= 0 || nc <= 0 || nf < 0) throw Error(VAG_ERR_ARG, "empty mesh");
        auto dir = host_copy(bc->node_dirichlet, (size_t)nn, mem, h->stream);
        h->general = mesh->hex8 == nullptr;
        DBuf<int32_t> pat_rp, pat_cl;  // the system pattern (CSR), for the sliced-ELL columns
        InputUploads inputs;           // once the host symbolic phase has accepted the mesh
        auto start_inputs = [&] {
            if (mem != VAG_MEM_HOST) return;
            inputs.add(h, h->xyz, mesh->node_xyz, 3 * (size_t)nn);
            inputs.add(h, h->perm, rock->perm, 6 * (size_t)nc);
            inputs.add(h, h->poro, rock->porosity, (size_t)nc);
            if (nf) {
                inputs.add(h, h->fwidth, frac->width, (size_t)nf);
                inputs.add(h, h->fperm, frac->perm, (size_t)nf);
                inputs.add(h, h->fporo, frac->porosity, (size_t)nf);
            }
            inputs.add(h, h->p_bar, bc->p_bar, (size_t)nn);
            if (bc->c_bar) inputs.add(h, h->c_bar, bc->c_bar, (size_t)nn);
            inputs.start();
        };
        if (!h->general) {
            // the caller's host array as it is; device arrays come over first
            std::vector<int32_t> hex8_copy;
            const int32_t *hex8 = mesh->hex8;
            if (mem == VAG_MEM_DEVICE) {
                hex8_copy = host_copy(mesh->hex8, 8 * (size_t)nc, mem, h->stream);
                hex8 = hex8_copy.data();
            }
            if (nf && !frac->face_nodes) throw Error(VAG_ERR_ARG, "hex8 meshes give fracture faces by face_nodes");
            std::vector<int32_t> fnodes =
                nf ? host_copy(frac->face_nodes, 4 * (size_t)nf, mem, h->stream) : std::vector<int32_t>();
            build_symbolic(nn, nc, nf, hex8, fnodes.data(), dir.data(), h->opt.eliminate_frac_faces != 0, h->S,
                           true);
            start_inputs();
            upload(h, h->hex8, mesh->hex8, 8 * (size_t)nc, mem);
            upload_vec(h, h->frac_nodes, fnodes);
            upload_vec(h, h->frac_slot, h->S.frac_slot);
            {
                DBuf<int32_t> work;
                work.alloc((size_t)nn + 2 * ((size_t)nn / 1024 + 2), h->tr);
                h->node_cell_ptr.alloc((size_t)nn + 1, h->tr);
                h->node_cell.alloc(8 * (size_t)nc, h->tr);
                launch_node_cell(h->stream, (int32_t)nn, nc, h->hex8.p, h->node_cell_ptr.p, h->node_cell.p, work.p);
                VAG_HIP(hipStreamSynchronize(h->stream));  // before work goes
            }
            upload_vec(h, h->node_frac_ptr, h->S.node_frac_ptr);
            upload_vec(h, h->node_frac, h->S.node_frac);
            device_pattern(h, pat_rp, pat_cl);
        } else {
            if (!mesh->cell_face_ptr || !mesh->cell_faces || !mesh->face_node_ptr || !mesh->face_nodes ||
                mesh->n_faces <= 0)
                throw Error(VAG_ERR_ARG, "a mesh without hex8 needs cell_face_ptr, cell_faces, face_node_ptr, "
                                         "face_nodes and n_faces");
            if (nf && !frac->face_ids) throw Error(VAG_ERR_ARG, "general meshes give fracture faces by face_ids");
            const int64_t nF = mesh->n_faces;
            if (nF >= INT32_MAX / 4) throw Error(VAG_ERR_ARG, "mesh sizes out of range");
            const auto cfp = host_copy(mesh->cell_face_ptr, (size_t)nc + 1, mem, h->stream);
            const auto fnp = host_copy(mesh->face_node_ptr, (size_t)nF + 1, mem, h->stream);
            if (cfp[0] != 0 || fnp[0] != 0 || cfp[nc] < 0 || fnp[nF] < 0 || cfp[nc] > 6 * (int64_t)nc ||
                fnp[nF] > 4 * nF)
                throw Error(VAG_ERR_ARG, "cell_face_ptr / face_node_ptr out of range");
            for (int64_t K = 0; K < nc; ++K)
                if (cfp[K + 1] < cfp[K]) throw Error(VAG_ERR_ARG, "cell_face_ptr is not ascending");
            for (int64_t f = 0; f < nF; ++f)
                if (fnp[f + 1] < fnp[f]) throw Error(VAG_ERR_ARG, "face_node_ptr is not ascending");
            const auto cf = host_copy(mesh->cell_faces, (size_t)cfp[nc], mem, h->stream);
            const auto fnd = host_copy(mesh->face_nodes, (size_t)fnp[nF], mem, h->stream);
            const std::vector<int32_t> fid =
                nf ? host_copy(frac->face_ids, (size_t)nf, mem, h->stream) : std::vector<int32_t>();
            build_symbolic_general(nn, nc, nF, cfp.data(), cf.data(), fnp.data(), fnd.data(), nf, fid.data(),
                                   dir.data(), h->S, h->G);
            start_inputs();
            const GenSym &G = h->G;
            upload_vec(h, h->g_cnode_ptr, G.cnode_ptr);
            upload_vec(h, h->g_cnode, G.cnode);
            upload_vec(h, h->g_cface_k, G.cface_k);
            upload_vec(h, h->g_cface_loc, G.cface_loc);
            upload_vec(h, h->g_fnode_ptr, G.fnode_ptr);
            upload_vec(h, h->g_fnode, G.fnode);
            upload_vec(h, h->g_unk_off, G.unk_off);
            upload_vec(h, h->g_loc_off, G.loc_off);
            upload_vec(h, h->g_con_ptr, G.con_ptr);
            upload_vec(h, h->g_con, G.con);
            upload_vec(h, h->g_bcon_ptr, G.bcon_ptr);
            upload_vec(h, h->g_bcon, G.bcon);
            upload_vec(h, h->g_bcon_node, G.bcon_node);
            upload_vec(h, h->g_inc_ptr, G.inc_ptr);
            upload_vec(h, h->g_inc_edge, G.inc_edge);
            upload_vec(h, h->g_inc_other, G.inc_other);
            h->gloc.alloc(std::max<int64_t>(G.loc_off.back(), 1), h->tr);
            h->ga.alloc(std::max<int64_t>(G.loc_off[nc], 1), h->tr);
            h->gr.alloc(std::max<int32_t>(G.unk_off.back(), 1), h->tr);
            h->Fall.alloc(std::max<int64_t>(G.nflux, 1), h->tr);
            launch_fill(h->stream, std::max<int64_t>(G.nflux, 1), 0.0, h->Fall.p);
        }
        const Symbolic &S = h->S;
        h->mu = rock->mu;

        if (mem != VAG_MEM_HOST) upload(h, h->xyz, mesh->node_xyz, 3 * (size_t)nn, mem);
        upload_vec(h, h->dirichlet, dir);
        if (h->general) {
            upload_vec(h, h->fmask, S.fmask);
            upload_vec(h, h->cell_frac, S.cell_frac);
            upload_vec(h, h->frac_cell, S.frac_cell);
            upload_vec(h, pat_rp, S.row_ptr);
            upload_vec(h, pat_cl, S.col);
        }
        upload_vec(h, h->node_unk, S.node_unk);
        upload_vec(h, h->frac_node, S.frac_node);
        upload_vec(h, h->sell_ptr, S.sell_ptr);
        upload_vec(h, h->unk_node, S.unk_node);
        upload_vec(h, h->unk_face, S.unk_face);
        upload_vec(h, h->frac_unk, S.frac_unk);
        upload_vec(h, h->face_grp, S.face_grp);
        upload_vec(h, h->face_loc, S.face_loc);
        upload_vec(h, h->grp_ptr, S.grp_ptr);
        upload_vec(h, h->grp_face, S.grp_face);
        upload_vec(h, h->grp_nptr, S.grp_nptr);
        upload_vec(h, h->grp_node, S.grp_node);
        upload_vec(h, h->grp_off, S.grp_off);
        upload_vec(h, h->grp_poff, S.grp_poff);
        {
            // sliced-ELL columns from the CSR pattern, on the device
            DBuf<int32_t> &rp = pat_rp, &cl = pat_cl;
            const int64_t nslice = (int64_t)S.sell_ptr.size() - 1;
            h->sell_col.alloc(std::max<int64_t>(S.sell_ptr.back(), 1), h->tr);
            h->row_len.alloc(std::max(S.nunk, 1), h->tr);
            h->diag_pos.alloc(std::max(S.nunk, 1), h->tr);
            launch_sell_fill(h->stream, S.nunk, nslice, rp.p, cl.p, h->sell_ptr.p, h->sell_col.p, h->row_len.p,
                             h->diag_pos.p);
            h->sell_col16.alloc(std::max<int64_t>(S.sell_ptr.back(), 1), h->tr);
            h->sell_cbase.alloc(std::max<int64_t>(S.sell_ptr.back() / 64, 1), h->tr);
            launch_sell_pack(h->stream, S.nunk, h->sell_ptr.p, h->sell_col.p, h->row_len.p, h->sell_col16.p,
                             h->sell_cbase.p);
            VAG_HIP(hipStreamSynchronize(h->stream));
            rp.release();
            cl.release();
        }
        h->Gb.alloc(std::max<int64_t>(S.grp_off.back(), 1), h->tr);

        if (mem != VAG_MEM_HOST) {
            upload(h, h->perm, rock->perm, 6 * (size_t)nc, mem);
            upload(h, h->poro, rock->porosity, (size_t)nc, mem);
            if (nf) {
                upload(h, h->fwidth, frac->width, (size_t)nf, mem);
                upload(h, h->fperm, frac->perm, (size_t)nf, mem);
                upload(h, h->fporo, frac->porosity, (size_t)nf, mem);
            }
            upload(h, h->p_bar, bc->p_bar, (size_t)nn, mem);
            if (bc->c_bar) upload(h, h->c_bar, bc->c_bar, (size_t)nn, mem);
        }
        if (!bc->c_bar) {
            h->c_bar.alloc(nn, h->tr);
            launch_fill(h->stream, nn, 0.0, h->c_bar.p);
        }

        const size_t n = S.nx;  // vectors hold the eliminated faces too
        if (!h->general) {
            h->aK.alloc(36 * (size_t)nc, h->tr);
            h->rK.alloc(8 * (size_t)nc, h->tr);
            h->fside.alloc(12 * (size_t)std::max<int64_t>(nf, 1), h->tr);
            h->A5.alloc(25 * (size_t)std::max<int64_t>(nf, 1), h->tr);
        }
        h->AKK.alloc(nc, h->tr);
        h->vol.alloc(nc, h->tr);
        h->area.alloc(std::max<int64_t>(nf, 1), h->tr);
        h->A.alloc(std::max<int64_t>(S.sell_ptr.back(), 1), h->tr);
        h->b.alloc(n, h->tr);
        h->dinv.alloc(n, h->tr);
        h->bad.alloc(1, h->tr);
        h->coef_bad.alloc(2, h->tr);
        for (auto *v : {&h->x, &h->r, &h->z, &h->p, &h->q}) v->alloc(n, h->tr);
        h->parts.alloc(6 * (size_t)kReduceBlocks, h->tr);
        h->rparts.alloc(4 * (size_t)kReduceBlocks, h->tr);
        h->scal.alloc(8, h->tr);
        h->pcg.alloc(2, h->tr);
        VAG_HIP(hipMemsetAsync(h->pcg.p, 0, 2 * sizeof(PcgState), h->stream));
        h->u_node.alloc(nn, h->tr);
        h->u_cell.alloc(nc, h->tr);
        h->u_frac.alloc(std::max<int64_t>(nf, 1), h->tr);
        if (!h->general) {
            h->F_cell.alloc(8 * (size_t)nc, h->tr);
            h->F_cell_frac.alloc(2 * (size_t)std::max<int64_t>(nf, 1), h->tr);
            h->F_frac.alloc(4 * (size_t)std::max<int64_t>(nf, 1), h->tr);
        }
        h->phi_cell.alloc(nc, h->tr);
        h->phi_frac.alloc(std::max<int64_t>(nf, 1), h->tr);
        h->phi_node.alloc(nn, h->tr);
        const int64_t nrow = nc + nf + nn;
        const int64_t nslice = (nrow + kSliceRows - 1) / kSliceRows;
        h->slice_width.alloc(nslice, h->tr);
        h->slice_nnz.alloc(nslice, h->tr);
        h->tmeta.alloc((size_t)nslice * kSliceRows, h->tr);
        h->slice_ptr.alloc(nslice + 1, h->tr);
        h->xsplit.alloc(18, h->tr);
        h->tdiag.alloc(nrow, h->tr);
        // one more entry: the constant control volume (concentration 1) that
        // well injection terms of the upwind operator read
        h->cbuf0.alloc(nrow + 1, h->tr);
        h->cbuf1.alloc(nrow + 1, h->tr);
        h->dt4.alloc(4, h->tr);
        h->tscan.alloc((size_t)nslice / 1024 + 2, h->tr);
        h->h_cnt = static_cast<unsigned long long *>(pinned_get(vag_handle::kCntWords * sizeof(unsigned long long)));
        h->h_pcg = static_cast<PcgState *>(pinned_get(sizeof(PcgState)));
        h->h_scal = static_cast<double *>(pinned_get(16 * sizeof(double)));
        for (auto &e : h->ev) VAG_HIP(hipEventCreate(&e));
        inputs.finish();
        if (h->general) return;
        // system positions of the eliminated groups' node pairs
        h->grp_pos.alloc(std::max<int64_t>(S.grp_poff.back(), 1), h->tr);
        VAG_HIP(hipMemsetAsync(h->bad.p, 0x7f, sizeof(int), h->stream));
        launch_grp_pos(h->stream, asm_args(h), S.ngroup, h->grp_poff.p, h->grp_pos.p);
        // slots of the cell-matrix columns in the node rows
        h->node_pos.alloc(64 * (size_t)nc, h->tr);  // 8 slots per node_cell entry
        launch_node_pos(h->stream, asm_args(h), h->node_pos.p);
        int bad = 0;
        VAG_HIP(hipMemcpyAsync(&bad, h->bad.p, sizeof(int), hipMemcpyDeviceToHost, h->stream));
        VAG_HIP(hipStreamSynchronize(h->stream));
        if (bad != 0x7f7f7f7f) throw Error(VAG_ERR_ARG, "internal: a group's node pair is missing from the pattern");
    });
    if (st != VAG_OK) {
        g_create_error = h->err;
        delete h;
        return st;
    }
    *out = h;
    return VAG_OK;
}

vag_status vag_update(vag_handle *h, const vag_rock *rock, const vag_fractures *fr, const double *p_bar,
                      const double *c_bar, vag_mem mem) {
    if (!h) return VAG_ERR_ARG;
    return guard(h, [&] {
        const size_t nn = h->S.nn, nc = h->S.nc, nf = h->S.nf;
        if (rock) {
            if (rock->perm) upload(h, h->perm, rock->perm, 6 * nc, mem);
            if (rock->porosity) upload(h, h->poro, rock->porosity, nc, mem);
            if (rock->mu > 0) h->mu = rock->mu;
        }
        if (fr && nf) {
            if (fr->width) upload(h, h->fwidth, fr->width, nf, mem);
            if (fr->perm) upload(h, h->fperm, fr->perm, nf, mem);
            if (fr->porosity) upload(h, h->fporo, fr->porosity, nf, mem);
        }
        if (p_bar) upload(h, h->p_bar, p_bar, nn, mem);
        if (c_bar) upload(h, h->c_bar, c_bar, nn, mem);
        h->solved = false;
        h->have_flux = false;
    });
}

vag_status vag_set_fluxes(vag_handle *h, const double *F_cell, const double *F_cell_frac, const double *F_frac,
                          vag_mem mem) {
    if (!h) return VAG_ERR_ARG;
    return guard(h, [&] {
        const Symbolic &S = h->S;
        hipStream_t s = h->stream;
        if (!F_cell || (S.nf && (!F_cell_frac || !F_frac))) throw Error(VAG_ERR_ARG, "null flux array");
        VAG_HIP(hipMemcpyAsync(h->flux_cell(), F_cell, (size_t)h->n_flux_cell() * sizeof(double), kind_in(mem), s));
        if (S.nf) {
            VAG_HIP(hipMemcpyAsync(h->flux_cell_frac(), F_cell_frac, 2 * (size_t)S.nf * sizeof(double), kind_in(mem),
                                   s));
            VAG_HIP(hipMemcpyAsync(h->flux_frac(), F_frac, (size_t)h->n_flux_frac() * sizeof(double), kind_in(mem),
                                   s));
        }
        // cell volumes and face areas come with the local matrices
        VAG_HIP(hipMemsetAsync(h->bad.p, 0x7f, sizeof(int), s));
        if (h->general) {
            const GenMesh g = h->gmesh();
            launch_gen_local(s, g, h->xyz.p, h->perm.p, 1.0 / h->mu, h->gloc.p, h->ga.p, h->gr.p, h->AKK.p,
                             h->vol.p, h->bad.p);
            launch_gen_frac_local(s, g, h->xyz.p, h->fwidth.p, h->fperm.p, 1.0 / h->mu, h->gloc.p, h->area.p);
            porous_volumes(h, s);
        } else {
            launch_local(s, S.nc, h->xyz.p, h->hex8.p, h->perm.p, h->mu, h->fmask.p, h->cell_frac.p,
                         h->frac_cell.p, h->aK.p, h->rK.p, h->AKK.p, h->vol.p, h->fside.p, h->bad.p);
            launch_frac_local(s, S.nf, h->xyz.p, h->frac_nodes.p, h->fwidth.p, h->fperm.p, h->mu, h->A5.p,
                              h->area.p);
            porous_volumes(h, s);
        }
        if (h->nw) {  // given fluxes come without well rates until vag_set_well_rates
            launch_fill(s, h->nw, 0.0, h->wrate.p);
            launch_fill(s, S.nf, 0.0, h->wsrc.p);
            launch_fill(s, S.nf, 0.0, h->wout.p);
        }
        VAG_HIP(hipStreamSynchronize(s));
        h->solved = false;
        h->have_flux = true;
        h->have_c = false;
    });
}

vag_status vag_set_wells(vag_handle *h, int64_t n, const int32_t *face, const double *wi, const double *p_w,
                         const double *q, const double *c_inj, vag_mem mem) {
    if (!h || n < 0) return VAG_ERR_ARG;
    return guard(h, [&] {
        const Symbolic &S = h->S;
        hipStream_t s = h->stream;
        if (n > 0 && (!face || !wi || !p_w || !q || !c_inj)) throw Error(VAG_ERR_ARG, "null well array");
        if (n > INT32_MAX) throw Error(VAG_ERR_ARG, "too many wells");
        const std::vector<int32_t> f = host_copy(face, (size_t)n, mem, s);
        const std::vector<double> a = host_copy(wi, (size_t)n, mem, s), b = host_copy(p_w, (size_t)n, mem, s),
                                  c = host_copy(q, (size_t)n, mem, s), d = host_copy(c_inj, (size_t)n, mem, s);
        std::vector<uint8_t> seen((size_t)std::max(S.nf, 1), 0);
        for (int64_t k = 0; k < n; ++k) {
            if (f[k] < 0 || f[k] >= S.nf)
                throw Error(VAG_ERR_ARG, "well " + std::to_string(k) + ": fracture face out of range");
            if (seen[f[k]]++) throw Error(VAG_ERR_ARG, "fracture face " + std::to_string(f[k]) + " perforated twice");
            if (!(a[k] >= 0) || !std::isfinite(a[k]) || !std::isfinite(b[k]) || !std::isfinite(c[k]) ||
                !std::isfinite(d[k]))
                throw Error(VAG_ERR_ARG, "well " + std::to_string(k) + ": WI must be >= 0 and all values finite");
        }
        h->nw = (int32_t)n;
        if (n) {
            upload_vec(h, h->wface, f);
            upload_vec(h, h->wwi, a);
            upload_vec(h, h->wpw, b);
            upload_vec(h, h->wq, c);
            upload_vec(h, h->wcinj, d);
            h->wrate.alloc((size_t)n, h->tr);
            h->wgiven.alloc((size_t)n, h->tr);
            h->wsrc.alloc((size_t)S.nf, h->tr);
            h->wout.alloc((size_t)S.nf, h->tr);
            launch_fill(s, n, 0.0, h->wrate.p);
            launch_fill(s, S.nf, 0.0, h->wsrc.p);
            launch_fill(s, S.nf, 0.0, h->wout.p);
            VAG_HIP(hipStreamSynchronize(s));
        }
        h->solved = false;
        h->have_flux = false;
    });
}

vag_status vag_get_well_rates(vag_handle *h, double *Q, vag_mem mem) {
    if (!h || (!Q && h->nw)) return VAG_ERR_ARG;
    return guard(h, [&] {
        if (!h->have_flux) throw Error(VAG_ERR_STATE, "no pressure solve (or fluxes) yet");
        download(h, Q, h->wrate, (size_t)h->nw, mem);
        VAG_HIP(hipStreamSynchronize(h->stream));
    });
}

vag_status vag_set_well_rates(vag_handle *h, const double *Q, vag_mem mem) {
    if (!h || (!Q && h->nw)) return VAG_ERR_ARG;
    return guard(h, [&] {
        if (!h->have_flux) throw Error(VAG_ERR_STATE, "vag_set_well_rates follows vag_set_fluxes");
        if (!h->nw) return;
        const Symbolic &S = h->S;
        hipStream_t s = h->stream;
        VAG_HIP(hipMemcpyAsync(h->wgiven.p, Q, (size_t)h->nw * sizeof(double), kind_in(mem), s));
        launch_fill(s, S.nf, 0.0, h->wsrc.p);
        launch_fill(s, S.nf, 0.0, h->wout.p);
        launch_well_rates(s, h->nw, h->wface.p, h->wwi.p, h->wpw.p, h->wq.p, h->wcinj.p, h->u_frac.p, h->wgiven.p,
                          h->wrate.p, h->wsrc.p, h->wout.p);
        VAG_HIP(hipStreamSynchronize(s));
        h->have_c = false;
    });
}

double vag_peaceman_wi(double dx, double dz, double d_f, double lambda_f, double r_w) {
    if (!(dx > 0 && dz > 0 && d_f > 0 && lambda_f > 0 && r_w > 0)) return 0.0;
    // the face expanded to a dx x d_f x dz box: its VAG cell coefficient is
    // lambda_f C, its corners sit at distance D from the axis
    const double pi = 3.14159265358979323846;
    const double C = 4.0 / 3.0 * (dx * dz / d_f + dx * d_f / dz + dz * d_f / dx);
    const double D = 0.5 * std::sqrt(dx * dx + d_f * d_f);
    const double lr = std::log(D / r_w) - 2.0 * pi * dz / C;  // ln(r0 / r_w)
    return lr > 0 ? 2.0 * pi * dz * lambda_f / lr : 0.0;
}

vag_status vag_set_stream(vag_handle *h, void *hip_stream) {
    if (!h) return VAG_ERR_ARG;
    return guard(h, [&] {
        // the old stream may still use the buffers: let it drain first
        VAG_HIP(hipStreamSynchronize(h->stream));
        h->stream = reinterpret_cast<hipStream_t>(hip_stream);
        h->tr.stream = h->stream;
    });
}

vag_status vag_set_options(vag_handle *h, const vag_options *opt) {
    if (!h || !opt) return VAG_ERR_ARG;
    return guard(h, [&] {
        check_options(*opt);
        if ((opt->eliminate_frac_faces != 0) != (h->opt.eliminate_frac_faces != 0))
            throw Error(VAG_ERR_ARG, "eliminate_frac_faces is fixed when the handle is created");
        h->opt = *opt;
    });
}

vag_status vag_solve_pressure(vag_handle *h, vag_solve_info *info) {
    if (!h) return VAG_ERR_ARG;
    bool converged = true;
    vag_status st = guard(h, [&] {
        const Symbolic &S = h->S;
        hipStream_t s = h->stream;
        const int32_t n = S.nunk;
        Phases ph("vag.assembly");
        VAG_HIP(hipEventRecord(h->ev[0], s));
        // 1. local matrices and fracture matrices (their coefficients checked on the way)
        VAG_HIP(hipMemsetAsync(h->bad.p, 0x7f, sizeof(int), s));
        VAG_HIP(hipMemsetAsync(h->coef_bad.p, 0x7f, 2 * sizeof(int), s));
        launch_check_coef(s, S.nc, h->perm.p, S.nf, h->fwidth.p, h->fperm.p, h->coef_bad.p);
        {
            int cb[2] = {0, 0};
            VAG_HIP(hipMemcpyAsync(cb, h->coef_bad.p, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
            VAG_HIP(hipStreamSynchronize(s));
            if (cb[0] != 0x7f7f7f7f)
                throw Error(VAG_ERR_ARG,
                            "cell " + std::to_string(cb[0]) + ": permeability tensor is not symmetric positive definite");
            if (cb[1] != 0x7f7f7f7f)
                throw Error(VAG_ERR_ARG,
                            "fracture face " + std::to_string(cb[1]) + ": width and permeability must be positive");
        }
        if (h->general) {
            // 2. the Schur blocks gathered into the system, Dirichlet columns to b
            const GenMesh g = h->gmesh();
            launch_gen_local(s, g, h->xyz.p, h->perm.p, 1.0 / h->mu, h->gloc.p, h->ga.p, h->gr.p, h->AKK.p,
                             h->vol.p, h->bad.p);
            launch_gen_frac_local(s, g, h->xyz.p, h->fwidth.p, h->fperm.p, 1.0 / h->mu, h->gloc.p, h->area.p);
            launch_gen_assemble(s, S.sell_ptr.back(), h->g_con_ptr.p, h->g_con.p, h->gloc.p, h->A.p);
            launch_gen_rhs(s, S.nunk, h->g_bcon_ptr.p, h->g_bcon.p, h->g_bcon_node.p, h->gloc.p, h->p_bar.p,
                           h->b.p);
        } else {
            launch_local(s, S.nc, h->xyz.p, h->hex8.p, h->perm.p, h->mu, h->fmask.p, h->cell_frac.p,
                         h->frac_cell.p, h->aK.p, h->rK.p, h->AKK.p, h->vol.p, h->fside.p, h->bad.p);
            launch_frac_local(s, S.nf, h->xyz.p, h->frac_nodes.p, h->fwidth.p, h->fperm.p, h->mu, h->A5.p,
                              h->area.p);
            // 2. cell elimination: one thread per row gathers its cells' Schur blocks
            launch_fill(s, (int64_t)h->A.n, 0.0, h->A.p);  // padding stays 0
            launch_fill(s, S.nx, 0.0, h->b.p);
            if (S.ngroup) launch_fill(s, S.grp_off.back(), 0.0, h->Gb.p);
            launch_assemble(s, asm_args(h), S.nunk - S.nfree, S.grp_ptr.empty() ? 0 : S.grp_ptr.back());
        }
        if (h->nw)
            launch_well_assemble(s, h->nw, h->wface.p, h->wwi.p, h->wpw.p, h->wq.p,
                                 WellAsm{S.nunk, h->frac_unk.p, h->diag_pos.p, h->face_grp.p, h->face_loc.p,
                                         h->grp_ptr.p, h->grp_nptr.p, h->grp_off.p, h->A.p, h->Gb.p, h->b.p});
        // fracture-face groups onto the nodes, colour by colour
        for (int c = 0; c < S.ngcolor; ++c)
            launch_group_elim(s, S.gcolor_ptr[c], S.gcolor_ptr[c + 1] - S.gcolor_ptr[c], S.grp_max_g, S.grp_max_m,
                              h->grp_ptr.p, h->grp_face.p, h->grp_nptr.p, h->grp_node.p, h->grp_off.p,
                              h->grp_poff.p, h->grp_pos.p, h->frac_unk.p, h->Gb.p, h->A.p, h->b.p, h->bad.p);
        launch_diag_inv(s, n, h->diag_pos.p, h->A.p, h->dinv.p);
        VAG_HIP(hipEventRecord(h->ev[1], s));
        ph.next("vag.preconditioner_setup");
        if (h->opt.precond == VAG_PC_AMG) {
            h->amg.setup(s, h->tr, h->Asell(), (int64_t)h->A.n, amg_options(h->opt));
            h->amg.stream_mode = h->opt.stream_loads;
            if (h->opt.precision == VAG_MIXED) h->amg.make_fp32(s, h->tr, nullptr);
        } else if (h->opt.precond == VAG_PC_BJILU0) {
            const int B = h->opt.ilu_block_rows > 0 ? h->opt.ilu_block_rows : kIluDefaultBlock;
            if (!h->ilu.ready(B)) {
                host_pattern(h);
                h->ilu.build(s, h->tr, S, B);
            }
            if (!h->ilu_bad.p) h->ilu_bad.alloc(1, h->tr);
            VAG_HIP(hipMemsetAsync(h->ilu_bad.p, 0, sizeof(int), s));
            h->ilu.factor(s, h->A.p, h->ilu_bad.p);
        }
        VAG_HIP(hipEventRecord(h->ev[2], s));
        ph.next("vag.krylov");
        // 3. Krylov
        if (h->opt.precision == VAG_MIXED_IR)
            run_mixed(h);
        else if (h->opt.krylov == VAG_GMRES)
            run_gmres(h);
        else if (h->opt.krylov == VAG_BICGSTAB)
            run_bicgstab(h);
        else
            run_pcg(h);
        VAG_HIP(hipEventRecord(h->ev[3], s));
        ph.next("vag.fluxes");
        const PcgState pst = *h->h_pcg;
        converged = pst.converged != 0;
        // 4. recovery and fluxes
        launch_group_back(s, S.ngroup, h->grp_ptr.p, h->grp_face.p, h->grp_nptr.p, h->grp_node.p, h->grp_off.p,
                          h->frac_unk.p, h->Gb.p, h->b.p, h->x.p);
        launch_node_pressure(s, S.nn, h->node_unk.p, h->x.p, h->p_bar.p, h->u_node.p);
        if (S.nf) launch_node_pressure(s, S.nf, h->frac_unk.p, h->x.p, h->p_bar.p, h->u_frac.p);  // all mapped
        if (h->nw) {
            launch_fill(s, S.nf, 0.0, h->wsrc.p);
            launch_fill(s, S.nf, 0.0, h->wout.p);
            launch_well_rates(s, h->nw, h->wface.p, h->wwi.p, h->wpw.p, h->wq.p, h->wcinj.p, h->u_frac.p, nullptr,
                              h->wrate.p, h->wsrc.p, h->wout.p);
        }
        if (h->general) {
            const GenMesh g = h->gmesh();
            launch_fill(s, 2 * (int64_t)S.nf, 0.0, h->flux_cell_frac());  // a missing second cell keeps 0
            launch_gen_flux(s, g, h->gloc.p, h->ga.p, h->gr.p, h->AKK.p, h->u_node.p, h->u_frac.p, h->u_cell.p,
                            h->Fall.p);
            porous_volumes(h, s);
        } else {
            launch_fill(s, 2 * (int64_t)std::max(S.nf, 1), 0.0, h->F_cell_frac.p);
            launch_cell_flux(s, S.nc, h->hex8.p, h->fmask.p, h->cell_frac.p, h->frac_cell.p, h->aK.p, h->rK.p,
                             h->AKK.p, h->fside.p, h->u_node.p, h->u_frac.p, h->u_cell.p, h->F_cell.p,
                             h->F_cell_frac.p);
            launch_frac_flux(s, S.nf, h->frac_nodes.p, h->A5.p, h->u_node.p, h->u_frac.p, h->F_frac.p);
            porous_volumes(h, s);
        }
        VAG_HIP(hipEventRecord(h->ev[4], s));
        ph.next("vag.residual");
        // true residual ||b - A x|| / ||b||
        launch_residual_norm(s, h->Asell(), h->x.p, h->b.p, h->r.p, h->rparts.p, h->scal.p);
        VAG_HIP(hipMemcpyAsync(h->h_scal, h->scal.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        int bad = 0, ilu_bad = 0;
        VAG_HIP(hipMemcpyAsync(&bad, h->bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
        if (h->opt.precond == VAG_PC_BJILU0)
            VAG_HIP(hipMemcpyAsync(&ilu_bad, h->ilu_bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
        VAG_HIP(hipStreamSynchronize(s));
        if (bad == INT_MIN) throw Error(VAG_ERR_ARG, "internal: an assembled entry is missing from the pattern");
        if (bad < 0)
            throw Error(VAG_ERR_ARG, "fracture-face group " + std::to_string(-1 - bad) +
                                         " has a face block that is not positive definite");
        if (bad != 0x7f7f7f7f)
            throw Error(VAG_ERR_MESH, "cell " + std::to_string(bad) + " has a non-positive sub-tetrahedron");
        if (ilu_bad)
            throw Error(VAG_ERR_UNSUPPORTED, "ILU(0) pivot of system row " + std::to_string(ilu_bad - 1) +
                                                 " (natural order) is zero or not finite");
        if (info) {
            std::memset(info, 0, sizeof *info);
            info->iterations = pst.iter;
            info->outer_iterations = h->last_outer;
            info->rel_residual = h->h_scal[1] > 0 ? std::sqrt(h->h_scal[0] / h->h_scal[1]) : 0.0;
            info->n_unknowns = n;
            info->nnz = S.nnz;
            info->amg_levels = h->opt.precond == VAG_PC_AMG ? h->amg.nlev : 0;
            info->amg_operator_complexity = h->opt.precond == VAG_PC_AMG ? h->amg.op_complexity : 1.0;
            info->ms_assembly = elapsed(h->ev[0], h->ev[1]);
            info->ms_setup = elapsed(h->ev[1], h->ev[2]);
            info->ms_solve = elapsed(h->ev[2], h->ev[3]);
            info->ms_fluxes = elapsed(h->ev[3], h->ev[4]);
        }
        h->solved = true;
        h->have_flux = true;
        h->have_c = false;
    });
    if (st == VAG_OK && !converged) {
        h->err = "Krylov solve stopped at max_iter before reaching rtol";
        return VAG_WARN_NOT_CONVERGED;
    }
    return st;
}

namespace {
// vag_transport up to its steps: CFL time step, the upwind operator, the
// initial state (ev[5] .. ev[6] on the handle's stream)
TransportPlan transport_prepare(vag_handle *h, int64_t n_steps, double t_final, const double *c0_cell,
                                const double *c0_frac, const double *c0_node, vag_mem mem) {
    if (!h->have_flux) throw Error(VAG_ERR_STATE, "vag_transport needs a pressure solve (or vag_set_fluxes) first");
    if (n_steps < 0 || t_final < 0) throw Error(VAG_ERR_ARG, "negative step count or final time");
    const Symbolic &S = h->S;
    hipStream_t s = h->stream;
    const int64_t nrow = (int64_t)S.nc + S.nf + S.nn;
    const int32_t nslice = (int32_t)((nrow + kSliceRows - 1) / kSliceRows);
    VAG_HIP(hipEventRecord(h->ev[5], s));
    if (h->general) {
        launch_gen_cfl(s, h->ginc(), h->Fall.p, h->well_out(), h->phi_cell.p, h->phi_frac.p, h->phi_node.p,
                       h->opt.cfl, h->rparts.p, h->dt4.p);
        launch_gen_upwind_count(s, h->ginc(), h->Fall.p, h->well_src(), h->slice_width.p, h->tmeta.p,
                                h->slice_nnz.p);
    } else {
        launch_cfl(s, S.nc, S.nf, S.nn, h->hex8.p, h->fmask.p, h->cell_frac.p, h->frac_cell.p, h->dirichlet.p,
                   h->node_cell_ptr.p, h->node_cell.p, h->node_frac_ptr.p, h->node_frac.p, h->F_cell.p,
                   h->F_cell_frac.p, h->F_frac.p, h->well_out(), h->phi_cell.p, h->phi_frac.p, h->phi_node.p,
                   h->opt.cfl, h->rparts.p, h->dt4.p);
        launch_upwind_count(s, S.nc, S.nf, S.nn, h->fmask.p, h->cell_frac.p, h->frac_cell.p, h->dirichlet.p,
                            h->node_cell_ptr.p, h->node_cell.p, h->node_frac_ptr.p, h->node_frac.p, h->F_cell.p,
                            h->F_cell_frac.p, h->F_frac.p, h->well_src(), h->slice_width.p, h->tmeta.p,
                            h->slice_nnz.p);
    }
    launch_scan64(s, nslice, h->slice_nnz.p, h->slice_ptr.p, h->tscan.p);  // slice offsets; the total at nslice
    // segment A: the slices of cells and fracture faces, B: of nodes
    launch_xcd_split(s, nslice, (int32_t)((S.nc + (int64_t)S.nf + kSliceRows - 1) / kSliceRows), h->slice_ptr.p,
                     h->xsplit.p);
    int64_t total = 0;
    VAG_HIP(hipMemcpyAsync(&total, h->slice_ptr.p + nslice, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    VAG_HIP(hipMemcpyAsync(h->h_xsplit(), h->xsplit.p, 18 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    VAG_HIP(hipMemcpyAsync(h->h_scal, h->dt4.p, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    VAG_HIP(hipStreamSynchronize(s));
    for (int x = 0; x < 18; ++x) h->xlo[x] = h->h_xsplit()[x];
    h->h_cnt[0] = (unsigned long long)total;  // entries without padding
    const double dt = h->h_scal[3];
    double dtb[3] = {h->h_scal[0], h->h_scal[1], h->h_scal[2]};
    if (!(dt < INFINITY)) throw Error(VAG_ERR_ARG, "no control volume has an outflow: CFL bound is infinite");
    if ((size_t)total > h->tcol.n) {
        h->tcol.alloc((size_t)total + (size_t)total / 8, h->tr);
        h->tcol16.alloc((size_t)total + (size_t)total / 8, h->tr);
        h->tval.alloc((size_t)total + (size_t)total / 8, h->tr);
    }
    ensure(h->tbase, (size_t)std::max<int64_t>(nslice, 1), h->tr);
    if (h->general)
        launch_gen_upwind_fill(s, h->ginc(), h->Fall.p, h->well_src(), h->well_out(), h->phi_cell.p,
                               h->phi_frac.p, h->phi_node.p, h->dt4.p, h->slice_ptr.p, h->tmeta.p, h->tcol.p,
                               h->tval.p, h->tdiag.p);
    else
        launch_upwind_fill(s, S.nc, S.nf, S.nn, h->hex8.p, h->fmask.p, h->cell_frac.p, h->frac_cell.p,
                           h->frac_nodes.p, h->dirichlet.p, h->node_cell_ptr.p, h->node_cell.p,
                           h->node_frac_ptr.p, h->node_frac.p, h->F_cell.p, h->F_cell_frac.p, h->F_frac.p,
                           h->well_src(), h->well_out(), h->phi_cell.p, h->phi_frac.p, h->phi_node.p, h->dt4.p,
                           h->slice_ptr.p, h->tmeta.p, h->tcol.p, h->tval.p, h->tdiag.p);
    launch_upwind_pack(s, h->upwind(), h->tcol16.p, h->tbase.p);
    h->have_op = true;
    // initial state
    if (c0_cell || c0_frac || c0_node) {
        if (!c0_cell || !c0_node || (S.nf && !c0_frac))
            throw Error(VAG_ERR_ARG, "give all of c0_cell, c0_frac, c0_node or none");
        h->cur = 0;
        VAG_HIP(hipMemcpyAsync(h->cbuf0.p, c0_cell, S.nc * sizeof(double), kind_in(mem), s));
        if (S.nf)
            VAG_HIP(hipMemcpyAsync(h->cbuf0.p + S.nc, c0_frac, S.nf * sizeof(double), kind_in(mem), s));
        VAG_HIP(hipMemcpyAsync(h->cbuf0.p + S.nc + S.nf, c0_node, S.nn * sizeof(double), kind_in(mem), s));
        if (mem == VAG_MEM_HOST) VAG_HIP(hipStreamSynchronize(s));
    } else if (!h->have_c) {
        h->cur = 0;
        launch_fill(s, nrow, 0.0, h->cbuf0.p);
    }
    launch_set_dirichlet(s, S.nn, S.nc + S.nf, h->dirichlet.p, h->c_bar.p, h->c_cur());
    launch_fill(s, 1, 1.0, h->cbuf0.p + nrow);  // the constant control volume
    launch_fill(s, 1, 1.0, h->cbuf1.p + nrow);
    h->have_c = true;
    TransportPlan P;
    P.N = n_steps;
    P.dt = P.last_dt = dt;
    P.total = total;
    for (int i = 0; i < 3; ++i) P.dtb[i] = dtb[i];
    if (t_final > 0) {
        P.N = (int64_t)std::ceil(t_final / dt);
        if (P.N < 1) P.N = 1;
        P.last_dt = t_final - (double)(P.N - 1) * dt;
        P.theta_last = P.last_dt / dt;
    }
    VAG_HIP(hipEventRecord(h->ev[6], s));
    return P;
}

void transport_report(vag_handle *h, const TransportPlan &P, vag_transport_info *info) {
    if (!info) return;
    const Symbolic &S = h->S;
    std::memset(info, 0, sizeof *info);
    info->n_steps = P.N;
    info->dt = P.dt;
    info->last_dt = P.last_dt;
    for (int i = 0; i < 3; ++i) info->dt_bounds[i] = P.dtb[i];
    info->ms_setup = elapsed(h->ev[5], h->ev[6]);
    info->ms_steps = elapsed(h->ev[6], h->ev[7]);
    info->n_rows = (int64_t)S.nc + S.nf + S.nn;
    info->t_nnz = h->h_cnt[0];
    info->t_stored = P.total;
}
}  // namespace

vag_status vag_transport(vag_handle *h, int64_t n_steps, double t_final, const double *c0_cell,
                         const double *c0_frac, const double *c0_node, vag_mem mem, vag_transport_info *info) {
    if (!h) return VAG_ERR_ARG;
    return guard(h, [&] {
        Phases ph("vag.transport_setup");
        const TransportPlan P = transport_prepare(h, n_steps, t_final, c0_cell, c0_frac, c0_node, mem);
        ph.next("vag.transport_steps");
        hipStream_t s = h->stream;
        for (int64_t k = 0; k < P.N; ++k) {
            const double th = (k == P.N - 1) ? P.theta_last : 1.0;
            launch_transport_step(s, h->upwind(), h->c_cur(), h->c_next(), th, (k & 1) != 0);
            h->cur ^= 1;
        }
        VAG_HIP(hipEventRecord(h->ev[7], s));
        VAG_HIP(hipEventSynchronize(h->ev[7]));
        transport_report(h, P, info);
    });
}

// Served jobs: the steps of a job's transport run in launches shared with
// other jobs (launch_transport_batch), driven by the server.
vag_status vag_serving_transport_begin(vag_handle *h, int64_t n_steps, double t_final, int64_t *N) {
    if (!h || !N) return VAG_ERR_ARG;
    return guard(h, [&] {
        h->plan = std::make_unique<TransportPlan>(transport_prepare(h, n_steps, t_final, nullptr, nullptr, nullptr,
                                                                    VAG_MEM_HOST));
        *N = h->plan->N;
    });
}
void vag_serving_transport_job(vag_handle *h, int64_t k, TransportJob *J) {
    const TransportPlan &P = *h->plan;
    J->T = h->upwind();
    J->c_in = h->c_cur();
    J->c_out = h->c_next();
    J->theta = (k == P.N - 1) ? P.theta_last : 1.0;
    J->backward = (k & 1) != 0;
    h->cur ^= 1;
}
hipEvent_t vag_serving_event(vag_handle *h, int i) { return h->ev[i]; }
vag_status vag_serving_transport_end(vag_handle *h, vag_transport_info *info) {
    if (!h || !h->plan) return VAG_ERR_ARG;
    return guard(h, [&] {
        VAG_HIP(hipEventSynchronize(h->ev[7]));
        transport_report(h, *h->plan, info);
        h->plan.reset();
    });
}

vag_status vag_transport_noalloc(vag_handle *h, int64_t n_steps, double t_final, const double *c0_cell,
                                 const double *c0_frac, const double *c0_node, double *c_cell, double *c_frac,
                                 double *c_node, vag_transport_info *info) {
    if (!h) return VAG_ERR_ARG;
    return guard(h, [&] {
        if (h->general)
            throw Error(VAG_ERR_UNSUPPORTED, "vag_transport_noalloc takes hex8 meshes; use vag_transport");
        if (!h->have_flux)
            throw Error(VAG_ERR_STATE, "vag_transport_noalloc needs a pressure solve (or vag_set_fluxes) first");
        if (n_steps < 0 || t_final < 0) throw Error(VAG_ERR_ARG, "negative step count or final time");
        const Symbolic &S = h->S;
        hipStream_t s = h->stream;
        const int64_t nrow = (int64_t)S.nc + S.nf + S.nn;
        // the CFL reduction's partials (3 per block of its grid) and dt_out
        size_t cap = 0;
        double *scr = noalloc_scratch(&cap);
        const size_t need = 3 * (size_t)kReduceBlocks + 4;
        if (need > cap)
            throw Error(VAG_ERR_ARG, "transport scratch of " + std::to_string(need) + " doubles exceeds the " +
                                         std::to_string(cap) + " of the static array");
        double *parts = scr, *dt4 = scr + 3 * (size_t)kReduceBlocks;
        const bool sync_dt = t_final > 0 || info;
        VAG_HIP(hipEventRecord(h->ev[5], s));
        launch_cfl(s, S.nc, S.nf, S.nn, h->hex8.p, h->fmask.p, h->cell_frac.p, h->frac_cell.p, h->dirichlet.p,
                   h->node_cell_ptr.p, h->node_cell.p, h->node_frac_ptr.p, h->node_frac.p, h->F_cell.p,
                   h->F_cell_frac.p, h->F_frac.p, h->well_out(), h->phi_cell.p, h->phi_frac.p, h->phi_node.p,
                   h->opt.cfl, parts, dt4);
        if (c0_cell || c0_frac || c0_node) {
            if (!c0_cell || !c0_node || (S.nf && !c0_frac))
                throw Error(VAG_ERR_ARG, "give all of c0_cell, c0_frac, c0_node or none");
            h->cur = 0;
            VAG_HIP(hipMemcpyAsync(h->cbuf0.p, c0_cell, S.nc * sizeof(double), hipMemcpyDeviceToDevice, s));
            if (S.nf)
                VAG_HIP(hipMemcpyAsync(h->cbuf0.p + S.nc, c0_frac, S.nf * sizeof(double), hipMemcpyDeviceToDevice,
                                       s));
            VAG_HIP(hipMemcpyAsync(h->cbuf0.p + S.nc + S.nf, c0_node, S.nn * sizeof(double),
                                   hipMemcpyDeviceToDevice, s));
        } else if (!h->have_c) {
            h->cur = 0;
            launch_fill(s, nrow, 0.0, h->cbuf0.p);
        }
        launch_set_dirichlet(s, S.nn, S.nc + S.nf, h->dirichlet.p, h->c_bar.p, h->c_cur());
        h->have_c = true;
        double dt = 0.0, dtb[3] = {0.0, 0.0, 0.0};
        if (sync_dt) {
            VAG_HIP(hipMemcpyAsync(h->h_scal, dt4, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
            VAG_HIP(hipStreamSynchronize(s));
            dt = h->h_scal[3];
            for (int i = 0; i < 3; ++i) dtb[i] = h->h_scal[i];
            if (!(dt < INFINITY)) throw Error(VAG_ERR_ARG, "no control volume has an outflow: CFL bound is infinite");
        }
        int64_t N = n_steps;
        double theta_last = 1.0, last_dt = dt;
        if (t_final > 0) {
            N = (int64_t)std::ceil(t_final / dt);
            if (N < 1) N = 1;
            last_dt = t_final - (double)(N - 1) * dt;
            theta_last = last_dt / dt;
        }
        VAG_HIP(hipEventRecord(h->ev[6], s));
        for (int64_t k = 0; k < N; ++k) {
            const double th = (k == N - 1) ? theta_last : 1.0;
            launch_transport_gather(s, S.nc, S.nf, S.nn, h->hex8.p, h->fmask.p, h->cell_frac.p, h->frac_cell.p,
                                    h->frac_nodes.p, h->dirichlet.p, h->node_cell_ptr.p, h->node_cell.p,
                                    h->node_frac_ptr.p, h->node_frac.p, h->F_cell.p, h->F_cell_frac.p, h->F_frac.p,
                                    h->well_src(), h->well_out(), h->phi_cell.p, h->phi_frac.p, h->phi_node.p, dt4,
                                    th, h->c_cur(), h->c_next());
            h->cur ^= 1;
        }
        const double *c = h->c_cur();
        if (c_cell) VAG_HIP(hipMemcpyAsync(c_cell, c, S.nc * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (c_frac && S.nf)
            VAG_HIP(hipMemcpyAsync(c_frac, c + S.nc, S.nf * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (c_node)
            VAG_HIP(hipMemcpyAsync(c_node, c + S.nc + S.nf, S.nn * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (info) {
            VAG_HIP(hipEventRecord(h->ev[7], s));
            VAG_HIP(hipEventSynchronize(h->ev[7]));
            std::memset(info, 0, sizeof *info);
            info->n_steps = N;
            info->dt = dt;
            info->last_dt = last_dt;
            for (int i = 0; i < 3; ++i) info->dt_bounds[i] = dtb[i];
            info->ms_setup = elapsed(h->ev[5], h->ev[6]);
            info->ms_steps = elapsed(h->ev[6], h->ev[7]);
            info->n_rows = nrow;
        }
    });
}

vag_status vag_get_pressure(vag_handle *h, double *u_node, double *u_cell, double *u_frac, vag_mem mem) {
    if (!h) return VAG_ERR_ARG;
    return guard(h, [&] {
        if (!h->solved) throw Error(VAG_ERR_STATE, "no pressure solve yet");
        download(h, u_node, h->u_node, h->S.nn, mem);
        download(h, u_cell, h->u_cell, h->S.nc, mem);
        download(h, u_frac, h->u_frac, h->S.nf, mem);
        VAG_HIP(hipStreamSynchronize(h->stream));
    });
}

vag_status vag_get_fluxes(vag_handle *h, double *F_cell, double *F_cell_frac, double *F_frac, vag_mem mem) {
    if (!h) return VAG_ERR_ARG;
    return guard(h, [&] {
        if (!h->have_flux) throw Error(VAG_ERR_STATE, "no pressure solve yet");
        auto get = [&](double *dst, const double *src, int64_t n) {
            if (dst && n > 0) VAG_HIP(hipMemcpyAsync(dst, src, (size_t)n * sizeof(double), kind_out(mem), h->stream));
        };
        get(F_cell, h->flux_cell(), h->n_flux_cell());
        get(F_cell_frac, h->flux_cell_frac(), 2 * (int64_t)h->S.nf);
        get(F_frac, h->flux_frac(), h->n_flux_frac());
        VAG_HIP(hipStreamSynchronize(h->stream));
    });
}

vag_status vag_flux_layout(const vag_handle *h, int64_t *n_cell_flux, int64_t *n_frac_flux) {
    if (!h) return VAG_ERR_ARG;
    if (n_cell_flux) *n_cell_flux = h->n_flux_cell();
    if (n_frac_flux) *n_frac_flux = h->n_flux_frac();
    return VAG_OK;
}

vag_status vag_get_porous_volumes(vag_handle *h, double *phi_cell, double *phi_frac, double *phi_node,
                                  vag_mem mem) {
    if (!h) return VAG_ERR_ARG;
    return guard(h, [&] {
        if (!h->have_flux) throw Error(VAG_ERR_STATE, "no pressure solve yet");
        download(h, phi_cell, h->phi_cell, h->S.nc, mem);
        download(h, phi_frac, h->phi_frac, h->S.nf, mem);
        download(h, phi_node, h->phi_node, h->S.nn, mem);
        VAG_HIP(hipStreamSynchronize(h->stream));
    });
}

vag_status vag_get_concentration(vag_handle *h, double *c_cell, double *c_frac, double *c_node, vag_mem mem) {
    if (!h) return VAG_ERR_ARG;
    return guard(h, [&] {
        if (!h->have_c) throw Error(VAG_ERR_STATE, "no transport yet");
        const Symbolic &S = h->S;
        hipMemcpyKind k = kind_out(mem);
        if (c_cell) VAG_HIP(hipMemcpyAsync(c_cell, h->c_cur(), S.nc * sizeof(double), k, h->stream));
        if (c_frac && S.nf) VAG_HIP(hipMemcpyAsync(c_frac, h->c_cur() + S.nc, S.nf * sizeof(double), k, h->stream));
        if (c_node) VAG_HIP(hipMemcpyAsync(c_node, h->c_cur() + S.nc + S.nf, S.nn * sizeof(double), k, h->stream));
        VAG_HIP(hipStreamSynchronize(h->stream));
    });
}

vag_status vag_system_size(vag_handle *h, int64_t *n, int64_t *nnz) {
    if (!h || !n || !nnz) return VAG_ERR_ARG;
    *n = h->S.nunk;
    *nnz = h->S.nnz;
    return VAG_OK;
}

vag_status vag_get_system(vag_handle *h, int64_t *row_ptr, int64_t *col, double *val, double *b, vag_mem mem) {
    if (!h) return VAG_ERR_ARG;
    return guard(h, [&] {
        if (!h->solved) throw Error(VAG_ERR_STATE, "no pressure solve yet");
        host_pattern(h);
        const Symbolic &S = h->S;
        const int32_t n = S.nunk;
        std::vector<double> sv(h->A.n), bv(std::max(n, 1));
        VAG_HIP(hipMemcpyAsync(sv.data(), h->A.p, sv.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        VAG_HIP(hipMemcpyAsync(bv.data(), h->b.p, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        VAG_HIP(hipStreamSynchronize(h->stream));
        // back to the natural order (free nodes by node index, then kept faces
        // by face index); entry k of stored row r sits at sell_ptr[r/64] + 64 k + r%64
        std::vector<int64_t> rp(n + 1, 0), cl(S.nnz);
        std::vector<double> cv(S.nnz), bo(std::max(n, 1));
        for (int32_t o = 0; o < n; ++o) {
            const int32_t r = S.sys_new[o];
            rp[o + 1] = rp[o] + (S.row_ptr[r + 1] - S.row_ptr[r]);
        }
        std::vector<std::pair<int32_t, double>> row;
        for (int32_t o = 0; o < n; ++o) {
            const int32_t r = S.sys_new[o];
            row.clear();
            for (int32_t k = 0; k < S.row_ptr[r + 1] - S.row_ptr[r]; ++k)
                row.emplace_back(S.sys_old[S.col[S.row_ptr[r] + k]],
                                 sv[S.sell_ptr[r >> 6] + 64 * (int64_t)k + (r & 63)]);
            std::sort(row.begin(), row.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
            for (size_t k = 0; k < row.size(); ++k) {
                cl[rp[o] + k] = row[k].first;
                cv[rp[o] + k] = row[k].second;
            }
            bo[o] = bv[r];
        }
        hipMemcpyKind k = mem == VAG_MEM_DEVICE ? hipMemcpyHostToDevice : hipMemcpyHostToHost;
        if (row_ptr) VAG_HIP(hipMemcpyAsync(row_ptr, rp.data(), rp.size() * sizeof(int64_t), k, h->stream));
        if (col) VAG_HIP(hipMemcpyAsync(col, cl.data(), cl.size() * sizeof(int64_t), k, h->stream));
        if (val) VAG_HIP(hipMemcpyAsync(val, cv.data(), cv.size() * sizeof(double), k, h->stream));
        if (b) VAG_HIP(hipMemcpyAsync(b, bo.data(), (size_t)n * sizeof(double), k, h->stream));
        VAG_HIP(hipStreamSynchronize(h->stream));
    });
}

vag_status vag_benchmark_kernel(vag_handle *h, int kernel, int reps, double *ms) {
    if (!h || !ms || reps <= 0) return VAG_ERR_ARG;
    return guard(h, [&] {
        if (!h->solved) throw Error(VAG_ERR_STATE, "no pressure solve yet");
        const Symbolic &S = h->S;
        hipStream_t s = h->stream;
        const int64_t nrow = (int64_t)S.nc + S.nf + S.nn;
        if (kernel == VAG_KERNEL_TRANSPORT_STEP && (!h->have_c || !h->have_op))
            throw Error(VAG_ERR_STATE, "the transport step needs a transport call first");
        int rep = 0;
        auto once = [&] {
            ++rep;
            switch (kernel) {
                case VAG_KERNEL_SPMV:  // the Krylov loop's SpMV (with its dot-product partials)
                    if (h->opt.precision == VAG_MIXED_IR && h->amg.have32)
                        launch_pcg_spmv<float, float>(s, h->amg.L[0]->A32, h->x32.p, h->q32.p,
                                                      PcgParts{h->parts.p, pcg_grid(S.nunk)}, h->pcg.p + 1);
                    else
                        launch_pcg_spmv<double, double>(s, h->Asell(), h->x.p, h->q.p,
                                                        PcgParts{h->parts.p, pcg_grid(S.nunk)}, h->pcg.p + 1);
                    break;
                case VAG_KERNEL_TRANSPORT_STEP:  // reads the current state, writes the spare buffer;
                    // the sweep direction alternates as in vag_transport
                    launch_transport_step(s, h->upwind(), h->c_cur(), h->c_next(), 1.0, (rep & 1) == 0);
                    break;
                case VAG_KERNEL_LOCAL:
                    if (h->general)
                        launch_gen_local(s, h->gmesh(), h->xyz.p, h->perm.p, 1.0 / h->mu, h->gloc.p, h->ga.p,
                                         h->gr.p, h->AKK.p, h->vol.p, h->bad.p);
                    else
                        launch_local(s, S.nc, h->xyz.p, h->hex8.p, h->perm.p, h->mu, h->fmask.p, h->cell_frac.p,
                                     h->frac_cell.p, h->aK.p, h->rK.p, h->AKK.p, h->vol.p, h->fside.p, h->bad.p);
                    break;
                case VAG_KERNEL_PRECOND:
                    if (h->opt.precision == VAG_MIXED_IR && h->amg.have32)
                        h->amg.apply32(s, h->r32.p, h->z32.p, nullptr);
                    else
                        precond_apply(h, h->r.p, h->z.p, nullptr);
                    break;
                default:
                    throw Error(VAG_ERR_ARG, "unknown kernel id");
            }
        };
        once();  // warm
        VAG_HIP(hipEventRecord(h->ev[5], s));
        for (int k = 0; k < reps; ++k) once();
        VAG_HIP(hipEventRecord(h->ev[6], s));
        VAG_HIP(hipEventSynchronize(h->ev[6]));
        *ms = elapsed(h->ev[5], h->ev[6]) / reps;
    });
}

vag_status vag_apply_preconditioner(vag_handle *h, const double *r, double *z, vag_mem mem) {
    if (!h || !r || !z) return VAG_ERR_ARG;
    return guard(h, [&] {
        if (!h->solved) throw Error(VAG_ERR_STATE, "no pressure solve yet");
        if (h->opt.precision == VAG_MIXED_IR)
            throw Error(VAG_ERR_UNSUPPORTED, "VAG_MIXED_IR applies its preconditioner to FP32 vectors inside the inner solve");
        const Symbolic &S = h->S;
        const int32_t n = S.nunk;
        hipStream_t s = h->stream;
        if (n == 0) return;
        // natural order <-> device order on the host (a test and debugging entry)
        const std::vector<double> rn = host_copy(r, (size_t)n, mem, s);
        std::vector<double> rd((size_t)n), zd((size_t)n), zn((size_t)n);
        for (int32_t o = 0; o < n; ++o) rd[S.sys_new[o]] = rn[o];
        VAG_HIP(hipMemcpyAsync(h->r.p, rd.data(), (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
        precond_apply(h, h->r.p, h->z.p, h->pcg.p + 1);
        VAG_HIP(hipMemcpyAsync(zd.data(), h->z.p, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s));
        VAG_HIP(hipStreamSynchronize(s));
        for (int32_t o = 0; o < n; ++o) zn[o] = zd[S.sys_new[o]];
        VAG_HIP(hipMemcpyAsync(z, zn.data(), (size_t)n * sizeof(double),
                               mem == VAG_MEM_DEVICE ? hipMemcpyHostToDevice : hipMemcpyHostToHost, s));
        VAG_HIP(hipStreamSynchronize(s));
    });
}

vag_status vag_amg_levels(vag_handle *h, int *nlev, int64_t *rows, int64_t *nnz, int64_t *stored, int max_levels) {
    if (!h || !nlev) return VAG_ERR_ARG;
    return guard(h, [&] {
        *nlev = h->opt.precond == VAG_PC_AMG && h->solved ? h->amg.nlev : 0;
        std::vector<unsigned long long> cnt(std::max(*nlev, 1), 0);
        if (*nlev > 1 && nnz) {
            VAG_HIP(hipMemcpyAsync(cnt.data(), h->amg.level_nnz.p, *nlev * sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost, h->stream));
            VAG_HIP(hipStreamSynchronize(h->stream));
        }
        for (int l = 0; l < *nlev && l < max_levels; ++l) {
            if (rows) rows[l] = h->amg.L[l]->n;
            if (stored) stored[l] = h->amg.L[l]->stored;
            if (nnz) nnz[l] = l == 0 ? h->S.nnz : (int64_t)cnt[l];
        }
    });
}

vag_status vag_amg_level_csr(vag_handle *h, int level, int64_t *sizes, int64_t *a_ptr, int64_t *a_col,
                             double *a_val, int64_t *p_ptr, int64_t *p_col, double *p_val, int32_t *coarse_index) {
    if (!h || !sizes) return VAG_ERR_ARG;
    return guard(h, [&] {
        if (!h->solved || h->opt.precond != VAG_PC_AMG) throw Error(VAG_ERR_STATE, "no AMG hierarchy yet");
        Amg &amg = h->amg;
        if (level < 0 || level >= amg.nlev) throw Error(VAG_ERR_ARG, "level out of range");
        hipStream_t s = h->stream;
        const Symbolic &S = h->S;
        AmgLevel &lv = *amg.L[level];
        const int32_t n = lv.n;
        const bool last = level == amg.nlev - 1;
        const int32_t nc = last ? 0 : amg.L[level + 1]->n;
        // level 0 rows and columns go back to the natural order
        auto nat = [&](int32_t r) { return level == 0 ? S.sys_old[r] : r; };
        auto dev = [&](int32_t o) { return level == 0 ? S.sys_new[o] : o; };
        const int64_t ns = (n + 63) / 64;
        std::vector<int64_t> ptr((size_t)ns + 1);
        VAG_HIP(hipMemcpyAsync(ptr.data(), lv.A.ptr, ptr.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        VAG_HIP(hipStreamSynchronize(s));
        std::vector<int32_t> col((size_t)ptr[ns]);
        std::vector<double> val((size_t)ptr[ns]);
        VAG_HIP(hipMemcpyAsync(col.data(), lv.A.col, col.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        VAG_HIP(hipMemcpyAsync(val.data(), lv.A.val, val.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        // interpolation in CSR (device row order)
        std::vector<int32_t> pp, pc, agg, rp, rc;
        std::vector<double> pv;
        if (!last) {
            if (amg.classical()) {
                pp.resize((size_t)n + 1);
                VAG_HIP(hipMemcpyAsync(pp.data(), lv.pptr.p, pp.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
                VAG_HIP(hipStreamSynchronize(s));
                pc.resize((size_t)pp[n]);
                pv.resize((size_t)pp[n]);
                VAG_HIP(hipMemcpyAsync(pc.data(), lv.pcol.p, pc.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
                VAG_HIP(hipMemcpyAsync(pv.data(), lv.pval.p, pv.size() * sizeof(double), hipMemcpyDeviceToHost, s));
                rp.resize((size_t)nc + 1);
                VAG_HIP(hipMemcpyAsync(rp.data(), lv.rptr.p, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
                VAG_HIP(hipStreamSynchronize(s));
                rc.resize((size_t)rp[nc]);
                VAG_HIP(hipMemcpyAsync(rc.data(), lv.rcol.p, rc.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            } else {
                agg.resize((size_t)n);
                VAG_HIP(hipMemcpyAsync(agg.data(), lv.agg.p, agg.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            }
        }
        VAG_HIP(hipStreamSynchronize(s));
        // A: every stored entry except slice padding (the row itself with value 0)
        std::vector<int64_t> arp((size_t)n + 1, 0);
        for (int32_t o = 0; o < n; ++o) {
            const int32_t r = dev(o);
            const int64_t w = (ptr[r / 64 + 1] - ptr[r / 64]) / 64;
            int64_t c = 0;
            for (int64_t j = 0; j < w; ++j) {
                const int64_t q = ptr[r / 64] + j * 64 + r % 64;
                c += !(col[q] == r && val[q] == 0.0);
            }
            arp[o + 1] = arp[o] + c;
        }
        int64_t pnnz = 0;
        if (!last) pnnz = amg.classical() ? (int64_t)pc.size() : n;
        sizes[0] = n;
        sizes[1] = arp[n];
        sizes[2] = nc;
        sizes[3] = pnnz;
        if (a_ptr) std::copy(arp.begin(), arp.end(), a_ptr);
        if (a_col || a_val)
            for (int32_t o = 0; o < n; ++o) {
                const int32_t r = dev(o);
                const int64_t w = (ptr[r / 64 + 1] - ptr[r / 64]) / 64;
                std::vector<std::pair<int32_t, double>> e;
                for (int64_t j = 0; j < w; ++j) {
                    const int64_t q = ptr[r / 64] + j * 64 + r % 64;
                    if (!(col[q] == r && val[q] == 0.0)) e.emplace_back(nat(col[q]), val[q]);
                }
                std::sort(e.begin(), e.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
                for (size_t k = 0; k < e.size(); ++k) {
                    if (a_col) a_col[arp[o] + (int64_t)k] = e[k].first;
                    if (a_val) a_val[arp[o] + (int64_t)k] = e[k].second;
                }
            }
        if (!last && (p_ptr || p_col || p_val)) {
            int64_t q = 0;
            for (int32_t o = 0; o < n; ++o) {
                const int32_t r = dev(o);
                if (p_ptr) p_ptr[o] = q;
                if (amg.classical()) {
                    for (int32_t t = pp[r]; t < pp[r + 1]; ++t, ++q) {
                        if (p_col) p_col[q] = pc[t];
                        if (p_val) p_val[q] = pv[t];
                    }
                } else {
                    if (p_col) p_col[q] = agg[r];
                    if (p_val) p_val[q] = 1.0;
                    ++q;
                }
            }
            if (p_ptr) p_ptr[n] = q;
        }
        if (coarse_index) {
            std::fill(coarse_index, coarse_index + n, -1);
            // the first entry of row c of R = P^T is the coarse point itself
            if (!last && amg.classical())
                for (int32_t c = 0; c < nc; ++c) coarse_index[nat(rc[rp[c]])] = c;
        }
    });
}

size_t vag_footprint_bytes(const vag_handle *h) { return h ? h->tr.bytes : 0; }

size_t vag_estimate_footprint(int64_t nn, int64_t nc, int64_t nf, const vag_options *opt) {
    vag_options o;
    if (opt) o = *opt; else vag_default_options(&o);
    if (nn <= 0 || nc <= 0 || nf < 0) return 0;
    const double Nn = (double)nn, Nc = (double)nc, Nf = (double)nf, Nx = Nn + Nf;
    // system entries: at most 27 per node row plus the couplings of the
    // fracture faces (face rows, their columns and the group fill); sliced
    // ELL padding
    const double nnz = 27.0 * Nn + 64.0 * Nf;
    const double S = 1.4 * nnz + 4096.0;
    double b = 0.0;
    b += 24 * Nn + 97 * Nc + 72 * Nf + 14 * Nn + 12.0 * S / 64;    // topology, adjacency
    b += 4 * S + 4 * (64 * Nc + 58 * Nf) + 8 * Nc;                 // pattern, slot maps
    b += 3000.0 * Nf;                                               // fracture-face groups
    b += 56 * Nc + 24 * Nf + 16 * Nn;                               // rock, fracture, boundary data
    b += 376 * Nc + 304 * Nf + 8 * S + 16 * Nx;                     // local matrices, system
    b += 40 * Nx + 64.0 * 1024;                                     // Krylov vectors and partials
    b += 88 * Nc + 56 * Nf + 16 * Nn;                               // pressures, fluxes, porous volumes
    if (o.alpha_rule == 1) b += 8 * Nn;                             // largest permeability per node
    const double nrow = Nn + Nc + Nf, tst = 2.0 * (8 * Nc + 6 * Nf) + 64.0 * 16;
    b += 24 * nrow + 12 * tst + 12 * nrow / 64;                     // transport
    if (o.precond == VAG_PC_AMG) {
        double amg = 104 * Nx + 17 * S + 0.15 * (12 * S + 104 * Nx);
        if (o.precision == VAG_MIXED) amg += 4.6 * S + 50 * Nx;
        if (o.precision == VAG_MIXED_IR) amg += 4.6 * S + 74 * Nx;
        if (o.amg_kind == 1)  // denser levels, P, R, A P and the product tables of one chunk of rows
            amg += 1.5 * amg + 12 * 48 * Nx + 12 * 1024 * std::min(Nx, (double)kClChunk);
        // the dense inverse of the coarsest level (FP64, and FP32 for the mixed
        // modes) and its elimination workspace: at most coarse_size rows
        const double cs = o.amg_coarse_size > 0 ? o.amg_coarse_size : 1000.0;
        const double d = std::min(Nx, std::min(cs, 1024.0));
        b += 1.125 * amg + 12.0 * d * d + 1024.0 * d + 0.5 * 1024 * 1024;
    }
    if (o.precond == VAG_PC_BJILU0) b += 14 * nnz + 28 * Nx;        // factor entries, rows, schedules
    if (o.krylov == VAG_GMRES) {  // flexible GMRES: m + 1 basis vectors, m preconditioned ones, two work vectors
        const double m = o.gmres_restart > 0 ? o.gmres_restart : 100;
        b += (2 * m + 3) * Nx * (o.precision == VAG_MIXED_IR ? 4.0 : 8.0) + 8 * (m + 1) * Nx / 256;
    }
    return (size_t)(1.15 * b) + ((size_t)1 << 20);
}

size_t vag_estimate_footprint_mesh(const vag_mesh *mesh, int64_t n_frac, const vag_options *opt) {
    if (!mesh || n_frac < 0) return 0;
    const int64_t nn = mesh->n_nodes, nc = mesh->n_cells;
    size_t b = vag_estimate_footprint(nn, nc, n_frac, opt);
    if (mesh->hex8 || !b) return b;
    // A general mesh adds, per cell of m = nv + f unknowns (nv nodes, f
    // fracture faces), m^2 local values, their derivatives and their
    // positions in the system (the gather lists of the assembly), and per
    // cell node its flux and incidence entries.  nv is bounded by the cell's
    // face-node count over 3 (a node of a polyhedron lies on three faces at
    // least) and by 8; with f <= 6 and at most 2 n_frac fracture sides,
    // sum m^2 <= sum nv^2 + (2 * 8 + 6) * 2 n_frac.
    const int64_t nF = mesh->n_faces;
    if (!mesh->cell_face_ptr || !mesh->cell_faces || !mesh->face_node_ptr || nF <= 0) return 0;
    double m2 = 0.0, ncn = 0.0;
    if (mesh->cell_face_ptr[0] != 0) return 0;
    for (int64_t K = 0; K < nc; ++K) {
        if (mesh->cell_face_ptr[K + 1] < mesh->cell_face_ptr[K]) return 0;
        int64_t fn = 0;
        for (int64_t q = mesh->cell_face_ptr[K]; q < mesh->cell_face_ptr[K + 1]; ++q) {
            const int32_t f = mesh->cell_faces[q];
            if (f < 0 || f >= nF) return 0;
            const int64_t d = mesh->face_node_ptr[f + 1] - mesh->face_node_ptr[f];
            if (d < 0) return 0;
            fn += d;
        }
        const double nv = (double)std::min<int64_t>(8, (fn + 2) / 3);
        m2 += nv * nv;
        ncn += nv;
    }
    m2 += 44.0 * (double)n_frac;
    b += (size_t)(1.15 * (24.0 * m2 + 48.0 * ncn + 32.0 * (double)nc + 16.0 * (double)nF));
    return b;
}

const char *vag_last_error(const vag_handle *h) { return h ? h->err.c_str() : g_create_error.c_str(); }

vag_status vag_trim_memory(void) {
    try {
        VAG_HIP(hipDeviceSynchronize());
        dev_trim();
        return VAG_OK;
    } catch (const Error &e) {
        return e.status;
    }
}

void vag_destroy(vag_handle *h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    delete h;
}

}  // extern "C"
