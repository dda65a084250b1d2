// Per-species network with an energy and a charge output (Sec. 2.1 Eq. 1, Sec. 2.2):
//   h = tanh(W0 D - b0),  U_i = w1E . h - b1E,  q_i = w1q . h - b1q,
// plus dU_i/dD = W0^T[(1 - h^2) w1E] and dq_i/dD = W0^T[(1 - h^2) w1q],
// and the charge correction of Eq. 33 (q'_i = q_i + delta).
#include "plan.h"

namespace qnep {

// FP32 vector-ALU form: one thread per atom, all species' weights in LDS.
template <int NDES>
__global__ __launch_bounds__(256) void k_mlp_fp32(int N, int T, int H, const int *__restrict__ ts,
                                                  const float *__restrict__ D, const float *__restrict__ theta,
                                                  int64_t off_nn, int64_t per_species, int64_t off_b1E,
                                                  float *__restrict__ U, float *__restrict__ qraw,
                                                  float *__restrict__ gU, float *__restrict__ gq,
                                                  double *__restrict__ partials) {
    extern __shared__ float wts[];  // T * per_species
    const int total = (int)(T * per_species);
    for (int k = threadIdx.x; k < total; k += blockDim.x) wts[k] = theta[off_nn + k];
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double red[2] = {0.0, 0.0};
    if (i < N) {
        const int t = ts[i];
        const float *W0 = wts + (size_t)t * per_species;
        const float *b0 = W0 + H * NDES;
        const float *w1E = b0 + H;
        const float *w1q = w1E + H;
        const float b1q = w1q[H];
        float d[NDES], gE[NDES], gQ[NDES];
#pragma unroll
        for (int v = 0; v < NDES; ++v) {
            d[v] = D[(size_t)v * N + i];
            gE[v] = 0.f;
            gQ[v] = 0.f;
        }
        float u = -theta[off_b1E], q = -b1q;
        for (int mu = 0; mu < H; ++mu) {
            const float *row = W0 + mu * NDES;
            float z = -b0[mu];
#pragma unroll
            for (int v = 0; v < NDES; ++v) z = fmaf(row[v], d[v], z);
            float h = tanhf(z);
            u = fmaf(w1E[mu], h, u);
            q = fmaf(w1q[mu], h, q);
            float dh = 1.0f - h * h;
            float a = w1E[mu] * dh, b = w1q[mu] * dh;
#pragma unroll
            for (int v = 0; v < NDES; ++v) {
                gE[v] = fmaf(a, row[v], gE[v]);
                gQ[v] = fmaf(b, row[v], gQ[v]);
            }
        }
        U[i] = u;
        qraw[i] = q;
#pragma unroll
        for (int v = 0; v < NDES; ++v) {
            gU[(size_t)v * N + i] = gE[v];
            gq[(size_t)v * N + i] = gQ[v];
        }
        red[0] = u;
        red[1] = q;
    }
    block_partials<2>(red, partials);
}

hipError_t launch_mlp_bf16(const Plan &p);

hipError_t launch_mlp(const Plan &p) {
    if (p.mlp_prec == QNEP_MLP_BF16 || p.mlp_prec == QNEP_MLP_BF16X3) return launch_mlp_bf16(p);
    const int G = (p.N + 255) / 256;
    const size_t lds = sizeof(float) * (size_t)(p.T * p.per_species);
    if (p.ndes == 25)
        hipLaunchKernelGGL(k_mlp_fp32<25>, dim3(G), dim3(256), lds, p.stream, p.N, p.T, p.H, p.ts, p.D, p.theta,
                           p.off_nn, p.per_species, p.off_b1E, p.U, p.qraw, p.gU, p.gq, p.partials);
    else if (p.ndes == 37)
        hipLaunchKernelGGL(k_mlp_fp32<37>, dim3(G), dim3(256), lds, p.stream, p.N, p.T, p.H, p.ts, p.D, p.theta,
                           p.off_nn, p.per_species, p.off_b1E, p.U, p.qraw, p.gU, p.gq, p.partials);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_partials(p, G, 2, S_UNEP, false);  // S_UNEP, S_SUMQ
}

// delta = (Q/s - sum_j q_j)/N so that q'_i = q_i + delta and sum q~' = Q (Eq. 33 as read)
__global__ void k_charge_shift(int N, double qtot, const float *__restrict__ theta, int64_t off_s,
                               double *__restrict__ scalars) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = theta[off_s];
        scalars[S_DELTA] = (qtot / s - scalars[S_SUMQ]) / (double)N;
    }
}

hipError_t launch_charges(const Plan &p) {
    hipLaunchKernelGGL(k_charge_shift, dim3(1), dim3(64), 0, p.stream, p.N, p.qtot, p.theta, p.off_s, p.scalars);
    return hipGetLastError();
}

}  // namespace qnep
