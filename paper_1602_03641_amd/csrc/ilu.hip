// Block-Jacobi ILU(0): host symbolic phase, factorization and triangular
// solves (§5.3's block Jacobi ILU(0) preconditioner; blocks and elimination
// order are stated in ilu.h).
//
// One wavefront per block.  Inside a block the rows are visited by levels of
// the dependency graph (a row's level is one more than the highest level of
// the rows it depends on), so the rows of one level are independent: the
// factorization and the forward solve follow the lower-triangle graph, the
// backward solve the upper one.  The solve keeps the block's vector in LDS.
#include <algorithm>
#include <atomic>
#include <exception>
#include <thread>

#include "host_parallel.h"
#include "ilu.h"

namespace vag {

namespace {

constexpr int kIluThreads = 64;

template <class T>
void put(hipStream_t s, Tracker &tr, DBuf<T> &d, const std::vector<T> &v) {
    d.alloc(std::max<size_t>(v.size(), 1), tr);
    if (!v.empty()) VAG_HIP(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Levels of one block (natural rows [r0, r1)): forward uses the entries left
// of the diagonal, backward those right of it.  Fills the block's slice of
// rows (r0-based) and its level pointers (absolute offsets into rows).
void block_levels(const std::vector<int32_t> &fptr, const std::vector<uint16_t> &fcol,
                  const std::vector<int32_t> &fdiag, int32_t r0, int32_t r1, bool forward, std::vector<int32_t> &lev,
                  std::vector<int32_t> &rows, std::vector<int32_t> &lptr) {
    const int32_t m = r1 - r0;
    int32_t top = 0;
    if (forward) {
        for (int32_t i = 0; i < m; ++i) {
            const int32_t o = r0 + i;
            int32_t l = 0;
            for (int32_t p = fptr[o]; p < fdiag[o]; ++p) l = std::max(l, lev[r0 + fcol[p]] + 1);
            lev[o] = l;
            top = std::max(top, l);
        }
    } else {
        for (int32_t i = m - 1; i >= 0; --i) {
            const int32_t o = r0 + i;
            int32_t l = 0;
            for (int32_t p = fdiag[o] + 1; p < fptr[o + 1]; ++p) l = std::max(l, lev[r0 + fcol[p]] + 1);
            lev[o] = l;
            top = std::max(top, l);
        }
    }
    // counting sort of the block's rows by level (ascending row inside a level)
    std::vector<int32_t> cnt(top + 2, 0);
    for (int32_t i = 0; i < m; ++i) ++cnt[lev[r0 + i] + 1];
    for (int32_t l = 0; l <= top; ++l) cnt[l + 1] += cnt[l];
    for (int32_t l = 0; l <= top; ++l) lptr.push_back(r0 + cnt[l]);
    for (int32_t i = 0; i < m; ++i) rows[r0 + cnt[lev[r0 + i]]++] = r0 + i;
}

}  // namespace

void Ilu::build(hipStream_t s, Tracker &tr, const Symbolic &S, int B) {
    const int32_t n = S.nunk;
    if (B < 1 || B > kIluMaxBlock) throw Error(VAG_ERR_ARG, "ilu_block_rows out of range");
    const int32_t nblk = (n + B - 1) / B;
    // in-block entries of each natural row, by local column
    std::vector<int32_t> cnt(n), fptr((size_t)n + 1, 0);
    parallel_chunks(n, [&](int, int64_t o0, int64_t o1) {
        for (int64_t o = o0; o < o1; ++o) {
            const int32_t r = S.sys_new[o], b0 = (int32_t)(o / B) * B;
            int32_t c = 0;
            for (int32_t q = S.row_ptr[r]; q < S.row_ptr[r + 1]; ++q) {
                const int32_t co = S.sys_old[S.col[q]];
                c += co >= b0 && co < b0 + B;
            }
            cnt[o] = c;
        }
    }, 4096);
    for (int32_t o = 0; o < n; ++o) fptr[o + 1] = fptr[o] + cnt[o];
    const int64_t nent = fptr[n];
    std::vector<uint16_t> fcol(nent);
    std::vector<int32_t> fsrc(nent), fdiag(n), rdev(n);
    std::atomic<bool> nodiag{false};
    parallel_chunks(n, [&](int, int64_t o0, int64_t o1) {
        std::vector<std::pair<int32_t, int32_t>> e;
        for (int64_t o = o0; o < o1; ++o) {
            const int32_t r = S.sys_new[o], b0 = (int32_t)(o / B) * B;
            const int64_t base = S.sell_ptr[r / kSliceRows] + r % kSliceRows;
            e.clear();
            for (int32_t q = S.row_ptr[r]; q < S.row_ptr[r + 1]; ++q) {
                const int32_t co = S.sys_old[S.col[q]];
                if (co >= b0 && co < b0 + B)
                    e.emplace_back(co - b0, (int32_t)(base + (int64_t)(q - S.row_ptr[r]) * kSliceRows));
            }
            std::sort(e.begin(), e.end());
            int32_t d = -1;
            for (size_t k = 0; k < e.size(); ++k) {
                fcol[fptr[o] + k] = (uint16_t)e[k].first;
                fsrc[fptr[o] + k] = e[k].second;
                if (e[k].first == o - b0) d = fptr[o] + (int32_t)k;
            }
            if (d < 0) nodiag.store(true);
            fdiag[o] = d;
            rdev[o] = r;
        }
    }, 4096);
    if (nodiag.load()) throw Error(VAG_ERR_ARG, "internal: a system row has no diagonal entry");
    // level schedules, block by block
    std::vector<int32_t> lev(n), rows_f(n), rows_b(n);
    std::vector<std::vector<int32_t>> lf(nblk), lb(nblk);
    parallel_chunks(nblk, [&](int, int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b) {
            const int32_t r0 = (int32_t)b * B, r1 = std::min<int32_t>(n, r0 + B);
            block_levels(fptr, fcol, fdiag, r0, r1, true, lev, rows_f, lf[b]);
            block_levels(fptr, fcol, fdiag, r0, r1, false, lev, rows_b, lb[b]);
        }
    }, 8);
    std::vector<int32_t> lvb_f(nblk + 1, 0), lvb_b(nblk + 1, 0), lptr_f, lptr_b;
    for (int32_t b = 0; b < nblk; ++b) {
        lvb_f[b + 1] = lvb_f[b] + (int32_t)lf[b].size();
        lvb_b[b + 1] = lvb_b[b] + (int32_t)lb[b].size();
        lptr_f.insert(lptr_f.end(), lf[b].begin(), lf[b].end());
        lptr_b.insert(lptr_b.end(), lb[b].begin(), lb[b].end());
    }
    lptr_f.push_back(n);
    lptr_b.push_back(n);
    std::vector<int4> slot_f(n), slot_b(n);
    for (int32_t t = 0; t < n; ++t) {
        const int32_t of = rows_f[t], ob = rows_b[t];
        slot_f[t] = make_int4(of - (of / B) * B, fptr[of], fdiag[of], 0);
        slot_b[t] = make_int4(ob - (ob / B) * B, fdiag[ob], fptr[ob + 1], 0);
    }
    nlev_ = std::max(lvb_f[nblk], lvb_b[nblk]);
    put(s, tr, fptr_, fptr);
    put(s, tr, fcol_, fcol);
    put(s, tr, fsrc_, fsrc);
    put(s, tr, fdiag_, fdiag);
    put(s, tr, rdev_, rdev);
    put(s, tr, lvb_f_, lvb_f);
    put(s, tr, lptr_f_, lptr_f);
    put(s, tr, rows_f_, rows_f);
    put(s, tr, lvb_b_, lvb_b);
    put(s, tr, lptr_b_, lptr_b);
    put(s, tr, rows_b_, rows_b);
    put(s, tr, slot_f_, slot_f);
    put(s, tr, slot_b_, slot_b);
    fval_.alloc(std::max<int64_t>(nent, 1), tr);
    VAG_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
    nent_ = nent;
    B_ = B;
    a_ = IluArgs{n,          B,         nblk,      fptr_.p,   fcol_.p,   fsrc_.p,   fdiag_.p,  rdev_.p,
                 lvb_f_.p,   lptr_f_.p, rows_f_.p, lvb_b_.p,  lptr_b_.p, rows_b_.p, slot_f_.p, slot_b_.p,
                 fval_.p};
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kIluThreads) void ilu_factor_kernel(IluArgs g, const double *__restrict__ A,
                                                                 int *bad) {
    const int32_t b = blockIdx.x, r0 = b * g.B, r1 = min(g.n, r0 + g.B);
    const int tid = threadIdx.x;
    for (int32_t e = g.fptr[r0] + tid; e < g.fptr[r1]; e += kIluThreads) g.fval[e] = A[g.fsrc[e]];
    __syncthreads();
    for (int32_t l = g.lvb_f[b]; l < g.lvb_f[b + 1]; ++l) {
        for (int32_t t = g.lptr_f[l] + tid; t < g.lptr_f[l + 1]; t += kIluThreads) {
            const int32_t o = g.rows_f[t], p1 = g.fptr[o + 1], pd = g.fdiag[o];
            // subtract multiples of the final rows k < o, in increasing k,
            // at the positions row o stores
            for (int32_t p = g.fptr[o]; p < pd; ++p) {
                const int32_t k = r0 + g.fcol[p], dk = g.fdiag[k], k1 = g.fptr[k + 1];
                const double lik = g.fval[p] / g.fval[dk];
                g.fval[p] = lik;
                int32_t pp = p + 1;
                for (int32_t q = dk + 1; q < k1 && pp < p1; ++q) {
                    const uint16_t j = g.fcol[q];
                    while (pp < p1 && g.fcol[pp] < j) ++pp;
                    if (pp < p1 && g.fcol[pp] == j) g.fval[pp] -= lik * g.fval[q];
                }
            }
            const double d = g.fval[pd];
            if (!(d != 0.0) || !__builtin_isfinite(d)) *bad = 1 + o;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kIluThreads) void ilu_solve_kernel(IluArgs g, const double *__restrict__ r,
                                                                double *__restrict__ z, const PcgState *st) {
    if (st && st->done) return;
    extern __shared__ double y[];
    const int32_t b = blockIdx.x, r0 = b * g.B, r1 = min(g.n, r0 + g.B);
    const int tid = threadIdx.x;
    const double *__restrict__ v = g.fval;
    const uint16_t *__restrict__ col = g.fcol;
    // the block's right-hand side into LDS, all loads in flight at once
    for (int32_t i = tid; i < r1 - r0; i += kIluThreads) y[i] = r[g.rdev[r0 + i]];
    __syncthreads();
    // L y = r (unit diagonal), in place
    for (int32_t l = g.lvb_f[b]; l < g.lvb_f[b + 1]; ++l) {
        for (int32_t t = g.lptr_f[l] + tid; t < g.lptr_f[l + 1]; t += kIluThreads) {
            const int4 m = g.slot_f[t];
            double s = y[m.x];
            for (int32_t p = m.y; p < m.z; ++p) s -= v[p] * y[col[p]];
            y[m.x] = s;
        }
        __syncthreads();
    }
    // U z = y, in place
    for (int32_t l = g.lvb_b[b]; l < g.lvb_b[b + 1]; ++l) {
        for (int32_t t = g.lptr_b[l] + tid; t < g.lptr_b[l + 1]; t += kIluThreads) {
            const int4 m = g.slot_b[t];
            double s = y[m.x];
            for (int32_t p = m.y + 1; p < m.z; ++p) s -= v[p] * y[col[p]];
            y[m.x] = s / v[m.y];
        }
        __syncthreads();
    }
    for (int32_t i = tid; i < r1 - r0; i += kIluThreads) z[g.rdev[r0 + i]] = y[i];
}

void Ilu::factor(hipStream_t s, const double *A, int *bad) {
    if (a_.nblk == 0) return;
    hipLaunchKernelGGL(ilu_factor_kernel, dim3(a_.nblk), dim3(kIluThreads), 0, s, a_, A, bad);
    VAG_HIP(hipGetLastError());
}

void Ilu::apply(hipStream_t s, const double *r, double *z, const PcgState *st) const {
    if (a_.nblk == 0) return;
    const size_t lds = (size_t)std::min(a_.B, a_.n) * sizeof(double);
    hipLaunchKernelGGL(ilu_solve_kernel, dim3(a_.nblk), dim3(kIluThreads), lds, s, a_, r, z, st);
    VAG_HIP(hipGetLastError());
}

}  // namespace vag
