// Setup and application of the aggregation AMG hierarchy (see amg.hip).
#include "amg.h"

#include <algorithm>

namespace vag {

Amg::~Amg() {
    pinned_put(h_, 1024 * sizeof(int32_t));
}

void Amg::setup(hipStream_t s, Tracker &tr, Sell<double> A0, int64_t stored0, const AmgOptions &o) {
    o_ = o;
    if (o.kind == 1) o_.kcycle = 0;  // the classical hierarchy runs V-cycles
    if (!h_) h_ = static_cast<int32_t *>(pinned_get(1024 * sizeof(int32_t)));
    const int32_t n0 = A0.n;
    if (o.kind == 1) {
        if (L.empty()) L.emplace_back(new AmgLevel());
        L[0]->n = n0;
        L[0]->A = A0;
        L[0]->stored = stored0;
        have32 = false;
        dense = false;
        setup_classical(s, tr, stored0);
        return;
    }
    // the coarsening keys hold a row's priority in 30 bits
    if (n0 >= (1 << 30)) throw Error(VAG_ERR_UNSUPPORTED, "AMG: more than 2^30 - 1 rows");
    ensure(T_, n0, tr);
    ensure(T1_, n0, tr);
    for (auto *b : {&flag_, &rid_, &agg1_, &lonely_, &lid_, &cnt_, &cursor_, &rowlen_}) ensure(*b, (size_t)n0 + 1, tr);
    ensure(width_, (size_t)n0 / 64 + 2, tr);
    ensure(big_, (size_t)n0 + 1, tr);
    ensure(mtmp_, (size_t)n0 + 1, tr);
    ensure(apn_, (size_t)n0, tr);
    ensure(spill_, (size_t)n0, tr);
    ensure(stmp_, 2 * ((size_t)n0 / 1024 + 4), tr);
    ensure(jcol_, (size_t)stored0, tr);
    ensure(apv_, (size_t)stored0, tr);
    ensure(counters_, 64, tr);
    ensure(mis_cnt_, (size_t)kMisRounds * kCntSlots * kCntStride, tr);
    ensure(scnt_, (size_t)n0 / 64 + 2, tr);
    ensure(level_nnz, (size_t)std::max(o.max_levels, 1), tr);
    VAG_HIP(hipMemsetAsync(level_nnz.p, 0, level_nnz.n * sizeof(unsigned long long), s));
    if (L.empty()) L.emplace_back(new AmgLevel());
    L[0]->n = n0;
    L[0]->A = A0;
    L[0]->stored = stored0;
    have32 = false;
    dense = false;
    int64_t stored_total = stored0;
    int l = 0;
    for (;; ++l) {
        AmgLevel &lv = *L[l];
        const int32_t n = lv.n;
        ensure(lv.diag, n, tr);
        ensure(lv.dinv, n, tr);
        amg_launch_diag(s, lv.A, lv.diag.p, lv.dinv.p);
        if (n <= o.coarse_size || l + 1 >= o.max_levels) break;
        // aggregation
        VAG_HIP(hipMemsetAsync(counters_.p, 0, 64 * sizeof(int), s));
        VAG_HIP(hipMemsetAsync(mis_cnt_.p, 0, mis_cnt_.n * sizeof(int), s));
        ensure(jcol_, (size_t)lv.stored, tr);  // the strong columns until the collapse reuses it
        amg_launch_mis(s, lv.A, lv.diag.p, o.theta, std::min(o.mis_rounds, kMisRounds), o.hops, T_.p, T1_.p, mis_cnt_.p,
                       flag_.p, h_ + 64, jcol_.p);
        amg_launch_scan(s, n, flag_.p, rid_.p, stmp_.p);
        ensure(lv.agg, n, tr);
        amg_launch_aggregate(s, lv.A, lv.diag.p, o.theta, flag_.p, rid_.p, agg1_.p, lv.agg.p, lonely_.p);
        amg_launch_scan(s, n, lonely_.p, lid_.p, stmp_.p);
        amg_launch_lonely(s, n, lonely_.p, lid_.p, rid_.p + n, lv.agg.p);
        VAG_HIP(hipMemcpyAsync(h_, rid_.p + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        VAG_HIP(hipMemcpyAsync(h_ + 1, lid_.p + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        VAG_HIP(hipStreamSynchronize(s));
        const int32_t nc = h_[0] + h_[1];
        if (nc <= 0 || nc > (int64_t)n * 9 / 10) break;  // coarsening stalled: this level is the coarsest
        // aggregate members and the Galerkin product
        ensure(lv.mptr, (size_t)nc + 1, tr);
        ensure(lv.mrows, n, tr);
        VAG_HIP(hipMemsetAsync(cnt_.p, 0, ((size_t)nc + 1) * sizeof(int32_t), s));
        VAG_HIP(hipMemsetAsync(cursor_.p, 0, ((size_t)nc + 1) * sizeof(int32_t), s));
        amg_launch_members(s, n, nc, lv.agg.p, cnt_.p, lv.mptr.p, cursor_.p, mtmp_.p, lv.mrows.p, stmp_.p);
        ensure(jcol_, (size_t)lv.stored, tr);
        ensure(apv_, (size_t)lv.stored, tr);
        ensure(apj_, (size_t)lv.stored, tr);
        amg_launch_collapse(s, lv.A, lv.agg.p, jcol_.p, apj_.p, apv_.p, apn_.p, spill_.p, counters_.p + 62);
        if ((int)L.size() <= l + 1) L.emplace_back(new AmgLevel());
        AmgLevel &cv = *L[l + 1];
        const int32_t ns = (nc + 63) / 64;
        ensure(cv.ptr, (size_t)ns + 1, tr);
        amg_launch_galerkin(s, lv.A, apj_.p, apv_.p, apn_.p, lv.mptr.p, lv.mrows.p, nc, 0, big_.p, rowlen_.p, nullptr,
                            nullptr, nullptr, counters_.p + 63);
        amg_launch_slices(s, nc, rowlen_.p, width_.p, scnt_.p, cv.ptr.p, level_nnz.p + l + 1);
        int64_t hv[2];
        VAG_HIP(hipMemcpyAsync(&hv[0], cv.ptr.p + ns, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        VAG_HIP(hipMemcpyAsync(h_ + 2, counters_.p + 63, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        VAG_HIP(hipStreamSynchronize(s));
        if (h_[2] != 0) break;  // a coarse row has too many candidates: stop coarsening here
        const int64_t stored = hv[0];
        ensure(cv.col, (size_t)stored, tr);
        ensure(cv.val, (size_t)stored, tr);
        amg_launch_galerkin(s, lv.A, apj_.p, apv_.p, apn_.p, lv.mptr.p, lv.mrows.p, nc, 1, big_.p, rowlen_.p, cv.ptr.p,
                            cv.col.p, cv.val.p, counters_.p + 63);
        amg_launch_slice_tail(s, nc, cv.ptr.p, cv.col.p, cv.val.p);
        cv.n = nc;
        cv.stored = stored;
        cv.A = Sell<double>{nc, cv.ptr.p, cv.col.p, cv.val.p};
        stored_total += stored;
        // vectors of the coarse level
        for (auto *v : {&cv.b, &cv.xa, &cv.xb, &cv.r}) ensure(*v, nc, tr);
    }
    finish_setup(s, tr, l, stored_total, stored0);
}

void Amg::finish_setup(hipStream_t s, Tracker &tr, int l, int64_t stored_total, int64_t stored0) {
    const int32_t n0 = L[0]->n;
    nlev = l + 1;
    op_complexity = (double)stored_total / (double)std::max<int64_t>(stored0, 1);
    AmgLevel &cl = *L[l];
    if (l == 0) {
        for (auto *v : {&cl.xa, &cl.r}) ensure(*v, cl.n, tr);
    } else {
        for (auto *v : {&L[0]->xa, &L[0]->r}) ensure(*v, n0, tr);
    }
    // K-cycle work on levels 1 .. kcycle that are not the coarsest
    for (int m = 1; m < nlev - 1 && m <= o_.kcycle; ++m) {
        AmgLevel &kv = *L[m];
        for (auto *v : {&kv.kc_c, &kv.kc_v, &kv.kc_rt, &kv.kc_d, &kv.kc_w}) ensure(*v, kv.n, tr);
        ensure(kv.kc_parts, (size_t)5 * kc_grid(kv.n), tr);
    }
    if (cl.n <= o_.dense_max && cl.n > 0) {
        ensure(Ainv, (size_t)cl.n * cl.n, tr);
        ensure(gj_work, (size_t)128 * cl.n, tr);
        amg_launch_dense_inverse(s, cl.A, Ainv.p, gj_work.p);
        dense = true;
    }
}

bool Amg::product(hipStream_t s, Tracker &tr, int32_t n, const Sell<double> *AX, const int32_t *xptr,
                  const int32_t *xcol, const double *xval, const int32_t *yptr, const int32_t *ycol,
                  const double *yval, bool fill, int32_t *rowlen, const int64_t *optr, bool sell_out, int32_t *ocol,
                  double *oval) {
    // table sizes are in ccap_; each chunk of rows gets its tables side by side
    const int32_t nch = (n + kClChunk - 1) / kClChunk;
    if (nch == 0) return true;
    ensure(csums_, (size_t)nch, tr);
    cl_launch_chunk_sums(s, n, ccap_.p, csums_.p);
    std::vector<int64_t> sums((size_t)nch);
    VAG_HIP(hipMemcpyAsync(sums.data(), csums_.p, (size_t)nch * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    VAG_HIP(hipMemsetAsync(counters_.p + 61, 0, sizeof(int), s));
    VAG_HIP(hipStreamSynchronize(s));
    const int64_t mx = *std::max_element(sums.begin(), sums.end());
    ensure(chkey_, (size_t)mx, tr);
    ensure(chval_, (size_t)mx, tr);
    ensure(choff_, (size_t)kClChunk + 1, tr);
    for (int32_t q = 0; q < nch; ++q) {
        const int32_t r0 = q * kClChunk, r1 = std::min(n, r0 + kClChunk);
        amg_launch_scan(s, r1 - r0, ccap_.p + r0, choff_.p, stmp_.p);
        cl_launch_product(s, r0, r1, AX, xptr, xcol, xval, yptr, ycol, yval, ccap_.p, choff_.p, chkey_.p, chval_.p,
                          fill, rowlen, optr, sell_out, ocol, oval, counters_.p + 61);
    }
    VAG_HIP(hipMemcpyAsync(h_ + 8, counters_.p + 61, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    VAG_HIP(hipStreamSynchronize(s));
    return h_[8] == 0;
}

// Classical hierarchy: strength, PMIS splitting, direct interpolation, R = P^T
// and the Galerkin product R (A P), level by level (see amg_classical.hip).
void Amg::setup_classical(hipStream_t s, Tracker &tr, int64_t stored0) {
    const int32_t n0 = L[0]->n;
    ensure(counters_, 64, tr);
    ensure(mis_cnt_, (size_t)kMisRounds, tr);
    ensure(stmp_, 2 * ((size_t)std::max(n0, kClChunk) / 1024 + 4), tr);
    ensure(width_, (size_t)n0 / 64 + 2, tr);
    ensure(scnt_, (size_t)n0 / 64 + 2, tr);
    ensure(level_nnz, (size_t)std::max(o_.max_levels, 1), tr);
    VAG_HIP(hipMemsetAsync(level_nnz.p, 0, level_nnz.n * sizeof(unsigned long long), s));
    int64_t stored_total = stored0;
    int l = 0;
    auto read32 = [&](const int32_t *d, int k) {
        VAG_HIP(hipMemcpyAsync(h_ + k, d, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    };
    for (;; ++l) {
        AmgLevel &lv = *L[l];
        const int32_t n = lv.n;
        ensure(lv.diag, n, tr);
        ensure(lv.dinv, n, tr);
        amg_launch_diag(s, lv.A, lv.diag.p, lv.dinv.p);
        if (n <= o_.coarse_size || l + 1 >= o_.max_levels) break;
        // strength and PMIS
        ensure(cm_, n, tr);
        ensure(csf_, (size_t)lv.stored, tr);
        ensure(ckey_, n, tr);
        ensure(cst_, n, tr);
        ensure(cst2_, n, tr);
        cl_launch_strength(s, lv.A, o_.strong_theta, cm_.p, csf_.p, ckey_.p, cst_.p);
        VAG_HIP(hipMemsetAsync(mis_cnt_.p, 0, (size_t)kMisRounds * sizeof(int), s));
        bool done = false;
        for (int r = 0; r < kMisRounds && !done;) {
            const int r1 = std::min(r + 4, kMisRounds);
            for (; r < r1; ++r) cl_launch_pmis_round(s, lv.A, csf_.p, ckey_.p, cst_.p, cst2_.p, mis_cnt_.p + r);
            read32(mis_cnt_.p + r - 1, 0);
            VAG_HIP(hipStreamSynchronize(s));
            done = h_[0] == 0;
        }
        if (!done) cl_launch_pmis_close(s, n, cst_.p);
        // interpolation
        ensure(cplen_, (size_t)n + 1, tr);
        ensure(cflag_, (size_t)n + 1, tr);
        ensure(ccidx_, (size_t)n + 1, tr);
        ensure(lv.pptr, (size_t)n + 1, tr);
        cl_launch_interp_count(s, lv.A, csf_.p, cst_.p, cplen_.p, cflag_.p);
        amg_launch_scan(s, n, cflag_.p, ccidx_.p, stmp_.p);
        amg_launch_scan(s, n, cplen_.p, lv.pptr.p, stmp_.p);
        read32(ccidx_.p + n, 0);
        read32(lv.pptr.p + n, 1);
        VAG_HIP(hipStreamSynchronize(s));
        const int32_t nc = h_[0], pnnz = h_[1];
        if (nc <= 0 || nc > (int64_t)n * 9 / 10) break;  // coarsening stalled: this level is the coarsest
        ensure(lv.pcol, (size_t)pnnz, tr);
        ensure(lv.pval, (size_t)pnnz, tr);
        ensure(ccfine_, (size_t)nc, tr);
        cl_launch_interp_fill(s, lv.A, csf_.p, cst_.p, ccidx_.p, lv.pptr.p, lv.pcol.p, lv.pval.p, ccfine_.p);
        // R = P^T
        ensure(crlen_, (size_t)std::max(n, nc) + 1, tr);
        ensure(lv.rptr, (size_t)nc + 1, tr);
        cl_launch_transpose(s, lv.A, nc, ccfine_.p, cst_.p, lv.pptr.p, lv.pcol.p, lv.pval.p, crlen_.p, nullptr,
                            nullptr, nullptr);
        amg_launch_scan(s, nc, crlen_.p, lv.rptr.p, stmp_.p);
        read32(lv.rptr.p + nc, 0);
        VAG_HIP(hipStreamSynchronize(s));
        const int32_t rnnz = h_[0];
        ensure(lv.rcol, (size_t)rnnz, tr);
        ensure(lv.rval, (size_t)rnnz, tr);
        cl_launch_transpose(s, lv.A, nc, ccfine_.p, cst_.p, lv.pptr.p, lv.pcol.p, lv.pval.p, nullptr, lv.rptr.p,
                            lv.rcol.p, lv.rval.p);
        // A P (CSR)
        ensure(ccap_, (size_t)std::max(n, nc) + 1, tr);
        cl_launch_ap_cap(s, lv.A, lv.pptr.p, ccap_.p);
        if (!product(s, tr, n, &lv.A, nullptr, nullptr, nullptr, lv.pptr.p, lv.pcol.p, lv.pval.p, false, cplen_.p,
                     nullptr, false, nullptr, nullptr))
            break;  // a row of A P is too wide for its table: stop coarsening here
        cl_launch_chunk_sums(s, n, cplen_.p, csums_.p);
        {
            const int32_t nch = (n + kClChunk - 1) / kClChunk;
            std::vector<int64_t> sums((size_t)nch);
            VAG_HIP(hipMemcpyAsync(sums.data(), csums_.p, (size_t)nch * sizeof(int64_t), hipMemcpyDeviceToHost, s));
            VAG_HIP(hipStreamSynchronize(s));
            int64_t tot = 0;
            for (auto v : sums) tot += v;
            if (tot >= INT32_MAX) break;  // A P would need 64-bit row pointers: stop coarsening here
        }
        ensure(captr_, (size_t)n + 1, tr);
        ensure(captr64_, (size_t)n + 1, tr);
        amg_launch_scan(s, n, cplen_.p, captr_.p, stmp_.p);
        read32(captr_.p + n, 0);
        VAG_HIP(hipStreamSynchronize(s));
        const int32_t apnnz = h_[0];
        cl_launch_widen(s, n, captr_.p, captr64_.p);
        ensure(capcol_, (size_t)std::max(apnnz, 1), tr);
        ensure(capval_, (size_t)std::max(apnnz, 1), tr);
        product(s, tr, n, &lv.A, nullptr, nullptr, nullptr, lv.pptr.p, lv.pcol.p, lv.pval.p, true, nullptr,
                captr64_.p, false, capcol_.p, capval_.p);
        // R (A P): the coarse level in sliced ELL
        if ((int)L.size() <= l + 1) L.emplace_back(new AmgLevel());
        AmgLevel &cv = *L[l + 1];
        const int32_t ns = (nc + 63) / 64;
        ensure(cv.ptr, (size_t)ns + 1, tr);
        cl_launch_rap_cap(s, nc, lv.rptr.p, lv.rcol.p, captr_.p, ccap_.p);
        if (!product(s, tr, nc, nullptr, lv.rptr.p, lv.rcol.p, lv.rval.p, captr_.p, capcol_.p, capval_.p, false,
                     crlen_.p, nullptr, true, nullptr, nullptr))
            break;
        amg_launch_slices(s, nc, crlen_.p, width_.p, scnt_.p, cv.ptr.p, level_nnz.p + l + 1);
        int64_t stored = 0;
        VAG_HIP(hipMemcpyAsync(&stored, cv.ptr.p + ns, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        VAG_HIP(hipStreamSynchronize(s));
        if (stored >= INT32_MAX) break;
        ensure(cv.col, (size_t)stored, tr);
        ensure(cv.val, (size_t)stored, tr);
        product(s, tr, nc, nullptr, lv.rptr.p, lv.rcol.p, lv.rval.p, captr_.p, capcol_.p, capval_.p, true, nullptr,
                cv.ptr.p, true, cv.col.p, cv.val.p);
        amg_launch_slice_tail(s, nc, cv.ptr.p, cv.col.p, cv.val.p);
        cv.n = nc;
        cv.stored = stored;
        cv.A = Sell<double>{nc, cv.ptr.p, cv.col.p, cv.val.p};
        stored_total += stored;
        for (auto *v : {&cv.b, &cv.xa, &cv.xb, &cv.r}) ensure(*v, nc, tr);
    }
    finish_setup(s, tr, l, stored_total, stored0);
}

void Amg::make_fp32(hipStream_t s, Tracker &tr, const int32_t *) {
    for (int l = 0; l < nlev; ++l) {
        AmgLevel &lv = *L[l];
        ensure(lv.val32, (size_t)lv.stored, tr);
        ensure(lv.dg32, lv.n, tr);
        launch_to_float_rowsum(s, lv.A, lv.val32.p, lv.dg32.p);
        ensure(lv.dinv32, lv.n, tr);
        launch_to_float(s, lv.n, lv.dinv.p, lv.dinv32.p);
        for (auto *v : {&lv.b32, &lv.xa32, &lv.xb32, &lv.r32}) ensure(*v, lv.n, tr);
        lv.A32 = Sell<float>{lv.n, lv.A.ptr, lv.A.col, lv.val32.p, lv.dg32.p, lv.A.col16, lv.A.cbase};
        lv.A32.nt = stream_matrix(lv.stored, sizeof(float), stream_mode);
    }
    if (dense) {
        const int32_t nc = L[nlev - 1]->n;
        ensure(Ainv32, (size_t)nc * nc, tr);
        launch_to_float(s, (int64_t)nc * nc, Ainv.p, Ainv32.p);
    }
    have32 = true;
}

// V-cycle on level l: out = M_l^-1 b.  x_ready: xa already holds D^-1 b (the
// first smoothing iterate), written by the kernel that produced b.
template <class V, class X>
void Amg::cycle(hipStream_t s, int l, const X *b, X *out, const PcgState *st, bool x_ready, double *rz) {
    if (o_.kind == 1 && l < nlev - 1) {
        if (rz) throw Error(VAG_ERR_ARG, "internal: the classical hierarchy does not fuse r.z");
        cycle_classical<V, X>(s, l, b, out, st, x_ready);
        return;
    }
    AmgLevel &lv = *L[l];
    Sell<V> A;
    const X *dinv;
    X *xa, *r;
    if constexpr (sizeof(V) == 4) A = lv.A32; else A = lv.A;
    if constexpr (sizeof(X) == 4) {
        dinv = lv.dinv32.p;
        xa = lv.xa32.p;
        r = lv.r32.p;
    } else {
        dinv = lv.dinv.p;
        xa = lv.xa.p;
        r = lv.r.p;
    }
    if (l == nlev - 1) {
        if (dense) {
            const X *Ai;
            if constexpr (sizeof(X) == 4) Ai = Ainv32.p; else Ai = Ainv.p;
            amg_launch_dense<X>(s, lv.n, Ai, b, out, st);
        } else {
            // a few l1-Jacobi sweeps from zero, ping-ponging between xa and out
            if (!x_ready) amg_launch_pre<V, X>(s, A, dinv, b, xa, r, st);
            X *src = xa, *dst = out;
            for (int k = 1; k < o_.coarse_sweeps; ++k) {
                amg_launch_sweep<V, X>(s, A, dinv, b, src, dst, st);
                std::swap(src, dst);
            }
            if (src != out) amg_launch_sweep<V, X>(s, A, dinv, b, src, out, st);
        }
        return;
    }
    AmgLevel &cv = *L[l + 1];
    X *bc, *ec, *xc;
    const X *dinv_c;
    if constexpr (sizeof(X) == 4) {
        bc = cv.b32.p;
        ec = cv.xb32.p;
        xc = cv.xa32.p;
        dinv_c = cv.dinv32.p;
    } else {
        bc = cv.b.p;
        ec = cv.xb.p;
        xc = cv.xa.p;
        dinv_c = cv.dinv.p;
    }
    const bool coarse_x = !(l + 1 == nlev - 1 && dense);  // the dense solve needs no iterate
    // sweeps on this level: one on the finest, o_.sweeps on the coarser ones
    // (the same number before and after the coarse correction: symmetric)
    const int nu = l == 0 ? 1 : std::max(1, o_.sweeps);
    if (nu == 1) {
        if (x_ready)
            amg_launch_resid<V, X>(s, A, b, xa, r, st);
        else
            amg_launch_pre<V, X>(s, A, dinv, b, xa, r, st);
        amg_launch_restrict<X>(s, cv.n, lv.mptr.p, lv.mrows.p, r, bc, coarse_x ? dinv_c : nullptr,
                               coarse_x ? xc : nullptr, st);
        coarse<V, X>(s, l + 1, bc, ec, st, coarse_x);
        if (lv.n <= kFusedPostRows && !rz) {
            amg_launch_post_fused<V, X>(s, A, dinv, b, lv.agg.p, ec, out, st);
        } else {
            double *zq = nullptr;
            const X *qv = nullptr;
            if constexpr (sizeof(X) == 8) {
                zq = rz ? zq_ : nullptr;
                qv = zq ? qv_ : nullptr;
            }
            amg_launch_post<V, X>(s, A, dinv, b, xa, lv.agg.p, ec, r, out, rz, st, zq, qv);  // r reused for y
        }
        return;
    }
    // nu pre-sweeps ping-ponging between xa and r, residual into the other
    X *xs = xa, *tmp = r;
    if (!x_ready) amg_launch_pre<V, X>(s, A, dinv, b, xa, r, st);  // xa = D^-1 b (r: discarded)
    for (int k = 1; k < nu; ++k) {
        amg_launch_sweep<V, X>(s, A, dinv, b, xs, tmp, st);
        std::swap(xs, tmp);
    }
    amg_launch_resid<V, X>(s, A, b, xs, tmp, st);
    amg_launch_restrict<X>(s, cv.n, lv.mptr.p, lv.mrows.p, tmp, bc, coarse_x ? dinv_c : nullptr,
                           coarse_x ? xc : nullptr, st);
    coarse<V, X>(s, l + 1, bc, ec, st, coarse_x);
    // the first post-sweep from y = x + P e (small levels: one kernel into tmp;
    // otherwise y into tmp and the sweep into xs), then nu - 1 more sweeps,
    // the last one into out (levels >= 1 only: no r.z partials)
    X *src = xs, *dst = tmp;
    if (lv.n <= kSmallRows) {
        amg_launch_post_x<V, X>(s, A, dinv, b, xs, lv.agg.p, ec, tmp, st);
        std::swap(src, dst);
    } else {
        amg_launch_post<V, X>(s, A, dinv, b, xs, lv.agg.p, ec, tmp, xs, nullptr, st);
    }
    for (int k = 1; k < nu; ++k) {
        amg_launch_sweep<V, X>(s, A, dinv, b, src, k == nu - 1 ? out : dst, st);
        std::swap(src, dst);
    }
}

// V-cycle on level l of the classical hierarchy: nu l1-Jacobi sweeps, the
// residual restricted by R, the coarse correction prolongated by P, nu sweeps.
template <class V, class X>
void Amg::cycle_classical(hipStream_t s, int l, const X *b, X *out, const PcgState *st, bool x_ready) {
    AmgLevel &lv = *L[l];
    AmgLevel &cv = *L[l + 1];
    Sell<V> A;
    const X *dinv, *dinv_c;
    X *xa, *r, *bc, *ec, *xc;
    if constexpr (sizeof(V) == 4) A = lv.A32; else A = lv.A;
    if constexpr (sizeof(X) == 4) {
        dinv = lv.dinv32.p;
        xa = lv.xa32.p;
        r = lv.r32.p;
        bc = cv.b32.p;
        ec = cv.xb32.p;
        xc = cv.xa32.p;
        dinv_c = cv.dinv32.p;
    } else {
        dinv = lv.dinv.p;
        xa = lv.xa.p;
        r = lv.r.p;
        bc = cv.b.p;
        ec = cv.xb.p;
        xc = cv.xa.p;
        dinv_c = cv.dinv.p;
    }
    const bool coarse_x = !(l + 1 == nlev - 1 && dense);
    const int nu = l == 0 ? 1 : std::max(1, o_.sweeps);
    // pre-smoothing: x = D^-1 b, then nu - 1 sweeps ping-ponging between xa and r
    if (!x_ready) amg_launch_pre<V, X>(s, A, dinv, b, xa, r, st);  // also r = b - A x
    X *x = xa, *t = r;
    for (int k = 1; k < nu; ++k) {
        amg_launch_sweep<V, X>(s, A, dinv, b, x, t, st);
        std::swap(x, t);
    }
    if (x_ready || nu > 1) amg_launch_resid<V, X>(s, A, b, x, t, st);
    cl_launch_restrict<X>(s, cv.n, lv.rptr.p, lv.rcol.p, lv.rval.p, t, bc, coarse_x ? dinv_c : nullptr,
                          coarse_x ? xc : nullptr, st);
    cycle<V, X>(s, l + 1, bc, ec, st, coarse_x, nullptr);
    // y = x + P e into t, then nu sweeps, the last one into out
    cl_launch_prolong<X>(s, lv.n, lv.pptr.p, lv.pcol.p, lv.pval.p, x, ec, t, st);
    X *src = t, *dst = x;
    for (int k = 1; k < nu; ++k) {
        amg_launch_sweep<V, X>(s, A, dinv, b, src, dst, st);
        std::swap(src, dst);
    }
    amg_launch_sweep<V, X>(s, A, dinv, b, src, out, st);
}

template <class V, class X>
void Amg::coarse(hipStream_t s, int m, const X *b, X *e, const PcgState *st, bool x_ready) {
    if constexpr (sizeof(X) == 8) {
        if (m <= o_.kcycle && m < nlev - 1 && x_ready) {
            // two flexible CG steps on A_m e = b, each preconditioned by a V-cycle from level m
            AmgLevel &lv = *L[m];
            Sell<V> A;
            if constexpr (sizeof(V) == 4) A = lv.A32; else A = lv.A;
            cycle<V, X>(s, m, b, lv.kc_c.p, st, true, nullptr);                  // c = B b (xa = D^-1 b given)
            amg_launch_kc_av<V, X>(s, A, lv.kc_c.p, b, lv.kc_v.p, lv.kc_parts.p, st);
            amg_launch_kc_rt<X>(s, lv.n, b, lv.kc_v.p, lv.dinv.p, lv.kc_parts.p, lv.kc_rt.p, lv.xa.p, st);
            cycle<V, X>(s, m, lv.kc_rt.p, lv.kc_d.p, st, true, nullptr);          // d = B rt
            amg_launch_kc_aw<V, X>(s, A, lv.kc_d.p, lv.kc_v.p, lv.kc_rt.p, lv.kc_w.p, lv.kc_parts.p, st);
            amg_launch_kc_combine<X>(s, lv.n, lv.kc_c.p, lv.kc_d.p, lv.kc_parts.p, e, st);
            return;
        }
    }
    cycle<V, X>(s, m, b, e, st, x_ready, nullptr);
}

void Amg::apply(hipStream_t s, const double *r, double *z, const PcgState *st, bool x_ready, double *rz, double *zq,
                const double *qv) {
    zq_ = zq;
    qv_ = qv;
    cycle<double, double>(s, 0, r, z, st, x_ready, rz);
    zq_ = nullptr;
    qv_ = nullptr;
}

void Amg::apply32(hipStream_t s, const float *r, float *z, const PcgState *st) {
    cycle<float, float>(s, 0, r, z, st, false, nullptr);
}

void Amg::apply_mixed(hipStream_t s, const double *r, double *z, const PcgState *st, bool x_ready, double *rz,
                      double *zq, const double *qv) {
    zq_ = zq;
    qv_ = qv;
    cycle<float, double>(s, 0, r, z, st, x_ready, rz);
    zq_ = nullptr;
    qv_ = nullptr;
}

}  // namespace vag
