// Global scalars of the evaluation, assembled in FP64:
//   E = U_NEP + U_ES (Eqs. 2-4), U_ES = U_r + U_k + U_s (+ background) in mode 1 or
//   U_k in mode 2 (Eq. 5), the direct Coulomb sum for an isolated system; W = static
//   real + reciprocal + many-body partial-force
//   virial (+ background); P = sum_i q~'_i r_i (Eq. 26).
#include "plan.h"

namespace qnep {

__global__ void k_finalize(int mode, int iso, double alpha, double vol, double qtot, const float *__restrict__ theta,
                           int64_t off_s, const double *__restrict__ scalars, const int *__restrict__ kcount,
                           double nk_default, double *__restrict__ energy, double *__restrict__ virial,
                           double *__restrict__ pol, double *__restrict__ terms) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double s = theta[off_s];
    double Ur = 0, Us = 0, Ubg = 0;
    double W[9];
    for (int k = 0; k < 9; ++k) W[k] = scalars[S_WK + k] + scalars[S_WNEP + k];
    if (iso) {  // direct Coulomb sum: no self or background term
        Ur = scalars[S_UREAL];
        for (int k = 0; k < 9; ++k) W[k] += scalars[S_WREAL + k];
    } else if (mode == 1) {
        Ur = scalars[S_UREAL];
        Us = -KE * alpha / sqrt(PI_D) * scalars[S_QSQ];
        const double Qs = qtot / s;
        Ubg = -KE * PI_D * Qs * Qs / (2.0 * vol * alpha * alpha);
        for (int k = 0; k < 9; ++k) W[k] += scalars[S_WREAL + k];
        W[0] += Ubg;
        W[4] += Ubg;
        W[8] += Ubg;
    }
    const double Uk = scalars[S_UK];
    if (energy) *energy = scalars[S_UNEP] + Ur + Uk + Us + Ubg;
    if (virial)
        for (int k = 0; k < 9; ++k) virial[k] = W[k];
    if (pol)
        for (int a = 0; a < 3; ++a) pol[a] = scalars[S_POL + a];
    if (terms) {
        terms[0] = scalars[S_UNEP];
        terms[1] = Ur;
        terms[2] = Uk;
        terms[3] = Us;
        terms[4] = Ubg;
        terms[5] = scalars[S_SUMQ];
        terms[6] = scalars[S_PHIBAR];
        terms[7] = kcount ? 2.0 * (double)(*kcount) : nk_default;
    }
}

hipError_t launch_finalize(const Plan &p) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, p.stream, p.mode, p.iso, p.alpha, p.vol, p.qtot, p.theta,
                       p.off_s, p.scalars, (p.method == 0 && !p.iso) ? p.kcount : (const int *)nullptr,
                       p.method == 1 ? (double)(p.mesh_pts - 1) : 0.0, p.out.energy, p.out.virial,
                       p.out.polarization, p.out.energy_terms);
    return hipGetLastError();
}

// N = 0: every requested output is zero
__global__ void k_zero_scalars(double *__restrict__ energy, double *__restrict__ virial, double *__restrict__ pol,
                               double *__restrict__ terms) {
    const int t = threadIdx.x;
    if (energy && t == 0) *energy = 0.0;
    if (virial && t < 9) virial[t] = 0.0;
    if (pol && t < 3) pol[t] = 0.0;
    if (terms && t < 8) terms[t] = 0.0;
}

hipError_t launch_zero_outputs(const Plan &p) {
    hipLaunchKernelGGL(k_zero_scalars, dim3(1), dim3(64), 0, p.stream, p.out.energy, p.out.virial,
                       p.out.polarization, p.out.energy_terms);
    return hipGetLastError();
}

}  // namespace qnep
