// Molecular dynamics in the microcanonical ensemble with the qNEP forces: velocity
// Verlet steps on the device, each with one full evaluation, and the time series of
// the polarization current P_dot = sum_i Z_i v_i (Sec. 2.4 Eq. 30) that the paper
// integrates for the polarization and correlates for infrared spectra and the ionic
// conductivity.  Units: positions Angstrom, velocities Angstrom/fs, masses amu,
// forces eV/Angstrom, energies eV.
#include "plan.h"

namespace qnep {

// 1 eV/(Angstrom amu) in Angstrom/fs^2, and 1 amu Angstrom^2/fs^2 in eV (CODATA 2018:
// e = 1.602176634e-19 C, u = 1.66053906660e-27 kg)
constexpr double MD_ACC = 1.602176634e-19 / 1.66053906660e-27 * 1e-10;
constexpr double MD_EKIN = 1.66053906660e-27 / 1.602176634e-19 * 1e10;

struct MdMasses {
    float inv[MAX_T];  // dt / (2 m_t) * MD_ACC: velocity change per unit force in half a step
    float m[MAX_T];    // m_t * MD_EKIN / 2: kinetic energy per unit v^2
};

// v += dt/2 F/m, then r += dt v
__global__ void k_md_kick_drift(int N, float dt, MdMasses ms, const int32_t *__restrict__ type,
                                const float *__restrict__ F, float *__restrict__ pos, float *__restrict__ vel) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int t = min(max(type[i], 0), MAX_T - 1);
    const float h = ms.inv[t];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const size_t k = (size_t)a * N + i;
        const float v = fmaf(h, F[k], vel[k]);
        vel[k] = v;
        pos[k] = fmaf(dt, v, pos[k]);
    }
}

// v += dt/2 F/m with the new forces; FP64 partials of the kinetic energy and of
// P_dot = sum_i Z_i v_i
__global__ __launch_bounds__(256) void k_md_kick_stats(int N, MdMasses ms, const int32_t *__restrict__ type,
                                                       const float *__restrict__ F, const float *__restrict__ Z,
                                                       float *__restrict__ vel, double *__restrict__ partials) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double red[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < N) {
        const int t = min(max(type[i], 0), MAX_T - 1);
        float v[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const size_t k = (size_t)a * N + i;
            v[a] = fmaf(ms.inv[t], F[k], vel[k]);
            vel[k] = v[a];
        }
        red[0] = (double)ms.m[t] * ((double)v[0] * v[0] + (double)v[1] * v[1] + (double)v[2] * v[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a)
            red[1 + a] = (double)Z[(size_t)(3 * a) * N + i] * v[0] + (double)Z[(size_t)(3 * a + 1) * N + i] * v[1] +
                         (double)Z[(size_t)(3 * a + 2) * N + i] * v[2];
    }
    block_partials<4>(red, partials);
}

// one row of the series: E_pot, E_kin, P_dot (3), P (3)
__global__ void k_md_record(const double *__restrict__ energy, const double *__restrict__ sums,
                            const double *__restrict__ pol, double *__restrict__ row) {
    if (threadIdx.x != 0) return;
    row[0] = energy[0];
    row[1] = sums[0];
    for (int a = 0; a < 3; ++a) {
        row[2 + a] = sums[1 + a];
        row[5 + a] = pol[a];
    }
}

static MdMasses md_masses(const double *masses, int T, double dt) {
    MdMasses ms{};
    for (int t = 0; t < MAX_T; ++t) {
        const double m = t < T ? masses[t] : 1.0;
        ms.inv[t] = (float)(0.5 * dt * MD_ACC / m);
        ms.m[t] = (float)(0.5 * m * MD_EKIN);
    }
    return ms;
}

hipError_t md_kick_drift(const Plan &p, const double *masses, double dt, float *pos, float *vel, const float *F) {
    const MdMasses ms = md_masses(masses, p.T, dt);
    hipLaunchKernelGGL(k_md_kick_drift, dim3((p.N + 255) / 256), dim3(256), 0, p.stream, p.N, (float)dt, ms, p.type,
                       F, pos, vel);
    return hipGetLastError();
}

hipError_t md_kick_record(const Plan &p, const double *masses, double dt, float *vel, const float *F,
                          const float *Z, const double *energy, const double *pol, double *sums, double *row) {
    const MdMasses ms = md_masses(masses, p.T, dt);
    const int G = (p.N + 255) / 256;
    hipLaunchKernelGGL(k_md_kick_stats, dim3(G), dim3(256), 0, p.stream, p.N, ms, p.type, F, Z, vel, p.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = reduce_partials_to(p, G, 4, sums);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_md_record, dim3(1), dim3(64), 0, p.stream, energy, sums, pol, row);
    return hipGetLastError();
}

}  // namespace qnep
