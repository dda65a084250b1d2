// One generation of the separable natural evolution strategy the paper trains with
// (Sec. 2.5; Schaul, Glasmachers and Schmidhuber 2011): sample the population
// z_k = mu + sigma s_k from caller-supplied standard-normal draws s_k, evaluate every
// member with the batched loss, rank the members, and move the search distribution
// along the natural gradient with the published rank utilities,
//   u_r = max(0, ln(C/2 + 1) - ln r) / sum_j max(0, ln(C/2 + 1) - ln j) - 1/C,
//   mu <- mu + eta_mu sigma sum_k u_k s_k,  sigma <- sigma exp(eta_sigma/2 sum_k u_k (s_k^2 - 1)).
#include <cmath>

#include "plan.h"

namespace qnep {

__global__ void k_snes_sample(int64_t d, int C, const float *__restrict__ mu, const float *__restrict__ sigma,
                              const float *__restrict__ noise, float *__restrict__ thetas) {
    const int64_t total = d * C;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % d;
        thetas[idx] = fmaf(sigma[i], noise[idx], mu[i]);
    }
}

constexpr int SNES_MAX_C = 1024;

// every work-group ranks the C losses itself (C is small) and then updates its slice of
// the d parameters; the sums over members run in index order in FP64
__global__ __launch_bounds__(256) void k_snes_update(int64_t d, int C, const double *__restrict__ loss,
                                                     const float *__restrict__ noise, double eta_mu,
                                                     double eta_sigma, float *__restrict__ mu,
                                                     float *__restrict__ sigma) {
    __shared__ double util[SNES_MAX_C];  // utility of member k
    __shared__ double raw_sum;
    const double top = log(0.5 * C + 1.0);
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int r = 1; r <= C; ++r) s += fmax(0.0, top - log((double)r));
        raw_sum = s;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < C; k += blockDim.x) {
        const double lk = loss[k];
        int rank = 0;  // members with a lower loss, or an equal loss and a lower index
        for (int j = 0; j < C; ++j) {
            const double lj = loss[j];
            rank += (lj < lk || (lj == lk && j < k)) ? 1 : 0;
        }
        util[k] = fmax(0.0, top - log((double)(rank + 1))) / raw_sum - 1.0 / C;
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d; i += (int64_t)gridDim.x * blockDim.x) {
        double gm = 0.0, gs = 0.0;
        for (int k = 0; k < C; ++k) {
            const double s = noise[(int64_t)k * d + i];
            gm = fma(util[k], s, gm);
            gs = fma(util[k], s * s - 1.0, gs);
        }
        const double sg = sigma[i];
        mu[i] = (float)(mu[i] + eta_mu * sg * gm);
        sigma[i] = (float)(sg * exp(0.5 * eta_sigma * gs));
    }
}

hipError_t snes_sample(int64_t d, int C, const float *mu, const float *sigma, const float *noise, float *thetas,
                       hipStream_t st) {
    const int64_t total = d * C;
    const int G = (int)std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_snes_sample, dim3(G), dim3(256), 0, st, d, C, mu, sigma, noise, thetas);
    return hipGetLastError();
}

hipError_t snes_update(int64_t d, int C, const double *loss, const float *noise, double eta_mu, double eta_sigma,
                       float *mu, float *sigma, hipStream_t st) {
    if (C < 1 || C > SNES_MAX_C) return hipErrorInvalidValue;
    const int G = (int)std::min<int64_t>((d + 255) / 256, 1024);
    hipLaunchKernelGGL(k_snes_update, dim3(G), dim3(256), 0, st, d, C, loss, noise, eta_mu, eta_sigma, mu, sigma);
    return hipGetLastError();
}

}  // namespace qnep
