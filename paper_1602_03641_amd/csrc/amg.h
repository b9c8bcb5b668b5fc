// Host orchestration of the aggregation AMG hierarchy (kernels in amg.hip).
#pragma once

#include <memory>
#include <vector>

#include "vag_internal.h"

namespace vag {

// levels of at most this many rows run their V-cycle kernels with several
// lanes per row
constexpr int32_t kSmallRows = 131072;

// kernel launchers (amg.hip)
void amg_launch_diag(hipStream_t s, Sell<double> A, double *diag, double *dinv);
// roots of the coarsening (flag); scol: a stored-size scratch array;
// undecided: rounds * kCntSlots * kCntStride zeroed counters; hcnt: pinned
// host memory of kCntSlots * kCntStride ints
constexpr int kCntSlots = 16, kCntStride = 32, kMisRounds = 48;
void amg_launch_mis(hipStream_t s, Sell<double> A, const double *diag, double theta, int rounds, int hops,
                    uint32_t *T, uint32_t *T1, int *undecided, int32_t *flag, int *hcnt, int32_t *scol);
void amg_launch_scan(hipStream_t s, int32_t n, const int32_t *in, int32_t *out, int32_t *tmp);
void amg_launch_aggregate(hipStream_t s, Sell<double> A, const double *diag, double theta, const int32_t *root,
                          const int32_t *rid, int32_t *agg1, int32_t *agg, int32_t *lonely);
void amg_launch_lonely(hipStream_t s, int32_t n, const int32_t *lonely, const int32_t *lid, const int32_t *nroot,
                       int32_t *agg);
void amg_launch_members(hipStream_t s, int32_t n, int32_t nc, const int32_t *agg, int32_t *cnt, int32_t *ptr,
                        int32_t *cursor, int32_t *tmp, int32_t *rows, int32_t *scan_tmp);
// row i of A P into the first apn[i] slots of (apJ, apv); nspill zeroed by the caller
void amg_launch_collapse(hipStream_t s, Sell<double> A, const int32_t *agg, int32_t *Jcol, int32_t *apJ,
                         double *apv, int32_t *apn, int32_t *spill, int *nspill);
void amg_launch_galerkin(hipStream_t s, Sell<double> A, const int32_t *Jcol, const double *apv, const int32_t *apn,
                         const int32_t *mptr, const int32_t *mrows, int32_t nc, int mode, int32_t *big,
                         int32_t *rowlen, const int64_t *cptr, int32_t *ccol, double *cval, int *overflow);
// slice widths and pointers from row lengths; *nnz = the number of entries
// (cnt: one int per slice, scratch)
void amg_launch_slices(hipStream_t s, int32_t n, const int32_t *rowlen, int32_t *width, int32_t *cnt, int64_t *ptr,
                       unsigned long long *nnz);
void amg_launch_slice_tail(hipStream_t s, int32_t n, const int64_t *ptr, int32_t *col, double *val);
// D = A^-1 (dense, row-major); work holds 128 * A.n doubles
void amg_launch_dense_inverse(hipStream_t s, Sell<double> A, double *D, double *work);
template <class V, class X>
void amg_launch_pre(hipStream_t s, Sell<V> A, const X *dinv, const X *b, X *x, X *r, const PcgState *st);
// bc = R r; with xc also xc = D_c^-1 bc
template <class X>
void amg_launch_restrict(hipStream_t s, int32_t nc, const int32_t *mptr, const int32_t *mrows, const X *r, X *bc,
                         const X *dinv_c, X *xc, const PcgState *st);
// r = b - A x
template <class V, class X>
void amg_launch_resid(hipStream_t s, Sell<V> A, const X *b, const X *x, X *r, const PcgState *st);
// y = x + P e, then out = y + M^-1 (b - A y); with rz, partials of b . out
// (and with zq, of qv . out)
template <class V, class X>
void amg_launch_post(hipStream_t s, Sell<V> A, const X *dinv, const X *b, const X *x, const int32_t *agg,
                     const X *e, X *y, X *out, double *rz, const PcgState *st, double *zq = nullptr,
                     const X *qv = nullptr);
// K-cycle kernels (see amg.hip); parts: 5 * kc_grid(n) doubles
int kc_grid(int32_t n);
template <class V, class X>
void amg_launch_kc_av(hipStream_t s, Sell<V> A, const X *c, const X *b, X *v, double *parts, const PcgState *st);
template <class X>
void amg_launch_kc_rt(hipStream_t s, int32_t n, const X *b, const X *v, const X *dinv, const double *parts, X *rt,
                      X *xa, const PcgState *st);
template <class V, class X>
void amg_launch_kc_aw(hipStream_t s, Sell<V> A, const X *d, const X *v, const X *rt, X *w, double *parts,
                      const PcgState *st);
template <class X>
void amg_launch_kc_combine(hipStream_t s, int32_t n, const X *c, const X *d, const double *parts, X *e,
                           const PcgState *st);
// the same with x = D^-1 b and y formed on the fly (one kernel)
template <class V, class X>
void amg_launch_post_fused(hipStream_t s, Sell<V> A, const X *dinv, const X *b, const int32_t *agg, const X *e,
                           X *out, const PcgState *st);
template <class X>
void amg_launch_dense(hipStream_t s, int32_t n, const X *Ainv, const X *b, X *x, const PcgState *st);
template <class V, class X>
void amg_launch_sweep(hipStream_t s, Sell<V> A, const X *dinv, const X *b, const X *x, X *out, const PcgState *st);
// levels of at most kSmallRows rows: out = y + D^-1 (b - A y) with y = x + P e
// in one kernel (out must not alias x)
template <class V, class X>
void amg_launch_post_x(hipStream_t s, Sell<V> A, const X *dinv, const X *b, const X *x, const int32_t *agg,
                       const X *e, X *out, const PcgState *st);
void launch_to_float(hipStream_t s, int64_t n, const double *a, float *b);
// FP32 off-diagonal values and an FP64 diagonal that keeps each row sum
void launch_to_float_rowsum(hipStream_t s, Sell<double> A, float *v32, double *dg);
void launch_to_double(hipStream_t s, int64_t n, const float *a, double *b);

// classical AMG (amg_classical.hip): product tables hold at most kClCapMax
// slots per row; rows are processed in chunks of kClChunk
constexpr int32_t kClCapMax = 16384;
constexpr int32_t kClChunk = 65536;
void cl_launch_strength(hipStream_t s, Sell<double> A, double theta, double *m, uint8_t *sf, uint64_t *key,
                        int8_t *state);
// one PMIS round (tmp: n bytes); *cnt += blocks that still hold undecided points
void cl_launch_pmis_round(hipStream_t s, Sell<double> A, const uint8_t *sf, const uint64_t *key, int8_t *st,
                          int8_t *tmp, int *cnt);
void cl_launch_pmis_close(hipStream_t s, int32_t n, int8_t *st);
void cl_launch_interp_count(hipStream_t s, Sell<double> A, const uint8_t *sf, const int8_t *st, int32_t *plen,
                            int32_t *cflag);
void cl_launch_interp_fill(hipStream_t s, Sell<double> A, const uint8_t *sf, const int8_t *st, const int32_t *cidx,
                           const int32_t *pptr, int32_t *pcol, double *pval, int32_t *cfine);
// rptr null: row lengths into rlen; else the rows
void cl_launch_transpose(hipStream_t s, Sell<double> A, int32_t nc, const int32_t *cfine, const int8_t *st,
                         const int32_t *pptr, const int32_t *pcol, const double *pval, int32_t *rlen,
                         const int32_t *rptr, int32_t *rcol, double *rval);
void cl_launch_ap_cap(hipStream_t s, Sell<double> A, const int32_t *pptr, int32_t *cap);
void cl_launch_rap_cap(hipStream_t s, int32_t nc, const int32_t *rptr, const int32_t *rcol, const int32_t *apptr,
                       int32_t *cap);
void cl_launch_chunk_sums(hipStream_t s, int32_t n, const int32_t *cap, int64_t *sums);
// rows [r0, r1) of X Y (X: AX in sliced ELL, or CSR xptr/xcol/xval); tables at
// hoff[i - r0]; count (rowlen) or fill (CSR optr, or sliced ELL when sell_out)
void cl_launch_product(hipStream_t s, int32_t r0, int32_t r1, const Sell<double> *AX, const int32_t *xptr,
                       const int32_t *xcol, const double *xval, const int32_t *yptr, const int32_t *ycol,
                       const double *yval, const int32_t *cap, const int32_t *hoff, int32_t *hkey, double *hval,
                       bool fill, int32_t *rowlen, const int64_t *optr, bool sell_out, int32_t *ocol, double *oval,
                       int *overflow);
void cl_launch_widen(hipStream_t s, int32_t n, const int32_t *in, int64_t *out);
template <class X>
void cl_launch_restrict(hipStream_t s, int32_t nc, const int32_t *rptr, const int32_t *rcol, const double *rval,
                        const X *r, X *bc, const X *dinv_c, X *xc, const PcgState *st);
template <class X>
void cl_launch_prolong(hipStream_t s, int32_t n, const int32_t *pptr, const int32_t *pcol, const double *pval,
                       const X *x, const X *e, X *y, const PcgState *st);

// grow-only device buffer (keeps its allocation across solves)
template <class T>
void ensure(DBuf<T> &b, size_t n, Tracker &t) {
    if (b.n < n) b.alloc(n + n / 8 + 64, t);
}

struct AmgLevel {
    int32_t n = 0;
    int64_t stored = 0;             // SELL entries incl. padding
    DBuf<int64_t> ptr;              // owned storage (coarse levels)
    DBuf<int32_t> col;
    DBuf<double> val;
    Sell<double> A;                 // view (level 0: the handle's matrix)
    DBuf<double> diag, dinv;
    DBuf<int32_t> agg, mptr, mrows; // aggregation to the next level
    DBuf<int32_t> pptr, pcol, rptr, rcol;  // classical: interpolation P and R = P^T (CSR)
    DBuf<double> pval, rval;
    DBuf<double> b, xa, xb, r;      // cycle vectors
    DBuf<float> val32, dinv32, b32, xa32, xb32, r32;
    DBuf<double> dg32;  // FP64 diagonal of the FP32 copy (row sums kept)
    DBuf<double> kc_c, kc_v, kc_rt, kc_d, kc_w, kc_parts;  // K-cycle work of this level
    Sell<float> A32;
};

struct AmgOptions {
    double theta = 0.02;
    int coarse_size = 1000;
    int max_levels = 12;
    int mis_rounds = 32;
    int dense_max = 1024;
    int coarse_sweeps = 4;  // sweeps of the coarsest level when it is not inverted
    int sweeps = 1;         // sweeps before and after the correction on levels >= 1
    int hops = 2;           // roots: distance-2 (2) or distance-1 (1) independent set
    int kcycle = 0;         // coarse levels 1..kcycle take the K-cycle (when not the coarsest)
    int kind = 0;           // 0: aggregation, 1: classical (PMIS, direct interpolation)
    double strong_theta = 0.25;  // classical strength threshold
};

class Amg {
  public:
    std::vector<std::unique_ptr<AmgLevel>> L;
    int nlev = 0;
    bool dense = false;
    bool have32 = false;
    double op_complexity = 1.0;
    int stream_mode = 0;  // non-temporal matrix loads of the FP32 copies (vag_options.stream_loads)
    DBuf<double> Ainv, gj_work;
    DBuf<float> Ainv32;
    DBuf<unsigned long long> level_nnz;  // entries (without padding) of each coarse level

    // Builds the hierarchy for A0 (n0 rows); host-synchronises a few times per level.
    void setup(hipStream_t s, Tracker &tr, Sell<double> A0, int64_t stored0, const AmgOptions &o);
    // Single-precision copy of every level (values, smoother, coarse inverse).
    void make_fp32(hipStream_t s, Tracker &tr, const int32_t *A0col);
    // z = M^-1 r, one V-cycle (FP64 or FP32); st may be null.  With x_ready
    // the caller has already written D^-1 r into L[0]->xa (the first
    // smoothing iterate); with rz, the last sweep also writes the block
    // partials of r . z there.
    // With zq (and qv), the last sweep also writes the partials of qv . z.
    // K-cycle levels make the preconditioner nonlinear (flexible CG).
    void apply(hipStream_t s, const double *r, double *z, const PcgState *st, bool x_ready = false,
               double *rz = nullptr, double *zq = nullptr, const double *qv = nullptr);
    void apply32(hipStream_t s, const float *r, float *z, const PcgState *st);
    // FP32 matrices, FP64 vectors
    void apply_mixed(hipStream_t s, const double *r, double *z, const PcgState *st, bool x_ready = false,
                     double *rz = nullptr, double *zq = nullptr, const double *qv = nullptr);
    // true when applying the hierarchy runs K-cycles (a nonlinear preconditioner)
    bool nonlinear() const { return o_.kcycle > 0 && nlev >= 3; }
    bool classical() const { return o_.kind == 1; }
    // levels at or below this many rows prolongate and smooth in one kernel
    static constexpr int32_t kFusedPostRows = kSmallRows;

  private:
    DBuf<uint32_t> T_, T1_;
    DBuf<int32_t> flag_, rid_, agg1_, lonely_, lid_, cnt_, cursor_, rowlen_, width_, big_, mtmp_, stmp_, jcol_, apn_, spill_, scnt_;
    DBuf<double> apv_;
    DBuf<int32_t> apj_;
    DBuf<int> counters_, mis_cnt_;
    int32_t *h_ = nullptr;  // pinned host scratch, 1024 ints
    AmgOptions o_;
    double *zq_ = nullptr;        // flexible-CG partials of the current application
    const double *qv_ = nullptr;
    // classical hierarchy: scratch of the setup
    DBuf<double> cm_, chval_, capval_;
    DBuf<uint8_t> csf_;
    DBuf<uint64_t> ckey_;
    DBuf<int8_t> cst_, cst2_;
    DBuf<int32_t> cplen_, cflag_, ccidx_, ccfine_, crlen_, ccap_, choff_, chkey_, captr_, capcol_;
    DBuf<int64_t> captr64_, csums_;
    void setup_classical(hipStream_t s, Tracker &tr, int64_t stored0);
    // vectors, K-cycle work and the coarsest inverse once level l is the coarsest
    void finish_setup(hipStream_t s, Tracker &tr, int l, int64_t stored_total, int64_t stored0);
    // sparse product X Y in chunks (count: rowlen; fill: into optr/ocol/oval); false on table overflow
    bool product(hipStream_t s, Tracker &tr, int32_t n, const Sell<double> *AX, const int32_t *xptr,
                 const int32_t *xcol, const double *xval, const int32_t *yptr, const int32_t *ycol,
                 const double *yval, bool fill, int32_t *rowlen, const int64_t *optr, bool sell_out, int32_t *ocol,
                 double *oval);
    template <class V, class X>
    void cycle(hipStream_t s, int l, const X *b, X *out, const PcgState *st, bool x_ready, double *rz);
    template <class V, class X>
    void cycle_classical(hipStream_t s, int l, const X *b, X *out, const PcgState *st, bool x_ready);
    // coarse-grid correction of level m: a V-cycle, or a K-cycle (two flexible CG steps)
    template <class V, class X>
    void coarse(hipStream_t s, int m, const X *b, X *e, const PcgState *st, bool x_ready);

  public:
    ~Amg();
};

}  // namespace vag
