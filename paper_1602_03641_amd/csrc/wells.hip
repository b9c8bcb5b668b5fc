// Peaceman wells perforating fracture faces (§5.5): the flow from well k into
// its face is Q_k = WI_k (p_w,k - u_sigma) + q_k.  In the face's conservation
// equation this puts WI on the diagonal and WI p_w + q on the right; in the
// transport it takes fluid out at the face's concentration (Q < 0) or brings
// it in at c_inj (Q > 0).  Each face is perforated at most once (checked on
// the host), so one thread per well writes without conflicts.
#include "vag_internal.h"

namespace vag {

namespace {
constexpr int kWT = 128;
}

// before the group elimination: kept faces add to the system row, eliminated
// ones to their group block (diagonal of the face's row) and to b
__global__ __launch_bounds__(kWT) void well_assemble_kernel(int32_t nw, const int32_t *__restrict__ wface,
                                                            const double *__restrict__ wi,
                                                            const double *__restrict__ pw,
                                                            const double *__restrict__ q, WellAsm g) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nw) return;
    const int32_t sg = wface[k];
    const int32_t u = g.frac_unk[sg];
    g.b[u] += wi[k] * pw[k] + q[k];
    if (u < g.nunk) {
        g.A[g.diag_pos[u]] += wi[k];
    } else {
        const int32_t G = g.face_grp[sg], loc = g.face_loc[sg];
        const int64_t W = (g.grp_ptr[G + 1] - g.grp_ptr[G]) + (g.grp_nptr[G + 1] - g.grp_nptr[G]);
        g.Gb[g.grp_off[G] + (int64_t)loc * W + loc] += wi[k];
    }
}

// Q_k from the face pressures, or given (Q != null: copied); per face the
// injected tracer rate c_inj Q^+ and the produced volume rate Q^- (the
// caller zeroes both face arrays first)
__global__ __launch_bounds__(kWT) void well_rates_kernel(int32_t nw, const int32_t *__restrict__ wface,
                                                         const double *__restrict__ wi, const double *__restrict__ pw,
                                                         const double *__restrict__ q,
                                                         const double *__restrict__ cinj,
                                                         const double *__restrict__ u_frac,
                                                         const double *__restrict__ given, double *__restrict__ rate,
                                                         double *__restrict__ fsrc, double *__restrict__ fout) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nw) return;
    const int32_t sg = wface[k];
    const double Q = given ? given[k] : wi[k] * (pw[k] - u_frac[sg]) + q[k];
    rate[k] = Q;
    fsrc[sg] = Q > 0.0 ? cinj[k] * Q : 0.0;
    fout[sg] = Q < 0.0 ? -Q : 0.0;
}

void launch_well_assemble(hipStream_t s, int32_t nw, const int32_t *wface, const double *wi, const double *pw,
                          const double *q, const WellAsm &g) {
    if (nw <= 0) return;
    hipLaunchKernelGGL(well_assemble_kernel, dim3((nw + kWT - 1) / kWT), dim3(kWT), 0, s, nw, wface, wi, pw, q, g);
    VAG_HIP(hipGetLastError());
}

void launch_well_rates(hipStream_t s, int32_t nw, const int32_t *wface, const double *wi, const double *pw,
                       const double *q, const double *cinj, const double *u_frac, const double *given, double *rate,
                       double *fsrc, double *fout) {
    if (nw <= 0) return;
    hipLaunchKernelGGL(well_rates_kernel, dim3((nw + kWT - 1) / kWT), dim3(kWT), 0, s, nw, wface, wi, pw, q, cinj,
                       u_frac, given, rate, fsrc, fout);
    VAG_HIP(hipGetLastError());
}

}  // namespace vag
