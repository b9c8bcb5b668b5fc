// Setup and application of the aggregation AMG hierarchy (see amg.hip).
#include "amg.h"

#include <algorithm>

namespace vag {

Amg::~Amg() {
    pinned_put(h_, 1024 * sizeof(int32_t));
}

void Amg::setup(hipStream_t s, Tracker &tr, Sell<double> A0, int64_t stored0, const AmgOptions &o) {
    o_ = o;
    if (!h_) h_ = static_cast<int32_t *>(pinned_get(1024 * sizeof(int32_t)));
    const int32_t n0 = A0.n;
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
    nlev = l + 1;
    op_complexity = (double)stored_total / (double)std::max<int64_t>(stored0, 1);
    AmgLevel &cl = *L[l];
    if (l == 0) {
        for (auto *v : {&cl.xa, &cl.r}) ensure(*v, cl.n, tr);
    } else {
        for (auto *v : {&L[0]->xa, &L[0]->r}) ensure(*v, n0, tr);
    }
    // K-cycle work on levels 1 .. kcycle that are not the coarsest
    for (int m = 1; m < nlev - 1 && m <= o.kcycle; ++m) {
        AmgLevel &kv = *L[m];
        for (auto *v : {&kv.kc_c, &kv.kc_v, &kv.kc_rt, &kv.kc_d, &kv.kc_w}) ensure(*v, kv.n, tr);
        ensure(kv.kc_parts, (size_t)5 * kc_grid(kv.n), tr);
    }
    if (cl.n <= o.dense_max && cl.n > 0) {
        ensure(Ainv, (size_t)cl.n * cl.n, tr);
        ensure(gj_work, (size_t)128 * cl.n, tr);
        amg_launch_dense_inverse(s, cl.A, Ainv.p, gj_work.p);
        dense = true;
    }
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
        lv.A32 = Sell<float>{lv.n, lv.A.ptr, lv.A.col, lv.val32.p, lv.dg32.p};
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
