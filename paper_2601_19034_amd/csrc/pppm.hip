// PPPM reciprocal part (Sec. 2.6):
//   charge assignment with the order-5 B-spline W (Eq. 35), forward FFT to S(k),
//   optimized influence function G_opt = G [prod sinc^5]^2 / [prod poly(z)]^2 (Eq. 36,
//   with the denominator squared and the z^6 coefficient -17/189, the value of the
//   P = 5 alias sum), energy k_e sum G_opt |S|^2 (Eq. 34) and virial k_e sum G_opt |S|^2 B
//   (B as in Eq. 21), ik differentiation for the static force (Eq. 37) and the
//   potential mesh for the dynamic-charge force (Eq. 38), gathered with the same W.
// Two packed complex inverse transforms give (E_x + i E_y) and (E_z + i phi).
#include "plan.h"

namespace qnep {

// order-5 weights of the mesh points m0 - 2 .. m0 + 2 for dx = u - m0 in [-1/2, 1/2]
__host__ __device__ inline void bspline5(float x, float *w) {
    const float x2 = x * x;
    const float a = 1.0f - 2.0f * x, b = 1.0f + 2.0f * x;
    w[0] = (a * a) * (a * a) * (1.0f / 384.0f);
    w[1] = (19.0f - 44.0f * x + 24.0f * x2 + 16.0f * x2 * x - 16.0f * x2 * x2) * (1.0f / 96.0f);
    w[2] = (115.0f - 120.0f * x2 + 48.0f * x2 * x2) * (1.0f / 192.0f);
    w[3] = (19.0f + 44.0f * x + 24.0f * x2 - 16.0f * x2 * x - 16.0f * x2 * x2) * (1.0f / 96.0f);
    w[4] = (b * b) * (b * b) * (1.0f / 384.0f);
}

struct MeshGeom {
    int n[3];
};

__device__ inline void mesh_stencil(float x, float y, float z, const Cell &c, const MeshGeom &g, int *m0,
                                    float (*w)[5]) {
    double s[3];
    s[0] = (double)x * c.hinv[0] + (double)y * c.hinv[3] + (double)z * c.hinv[6];
    s[1] = (double)x * c.hinv[1] + (double)y * c.hinv[4] + (double)z * c.hinv[7];
    s[2] = (double)x * c.hinv[2] + (double)y * c.hinv[5] + (double)z * c.hinv[8];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double sa = s[a] - floor(s[a]);
        double u = sa * g.n[a];
        double m = floor(u + 0.5);
        m0[a] = (int)m;
        bspline5((float)(u - m), w[a]);
    }
}

__device__ inline int wrap_index(int j, int n) {
    j %= n;
    return j < 0 ? j + n : j;
}

__global__ __launch_bounds__(256) void k_spread(int N, const float4 *__restrict__ xyzt, Cell c, MeshGeom g,
                                                const float *__restrict__ qraw, const double *__restrict__ scalars,
                                                float *__restrict__ rho) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float q = qraw[i] + (float)scalars[S_DELTA];
    int m0[3];
    float w[3][5];
    const float4 pa = xyzt[i];
    mesh_stencil(pa.x, pa.y, pa.z, c, g, m0, w);
    int j0[5], j1[5], j2[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        j0[t] = wrap_index(m0[0] + t - 2, g.n[0]);
        j1[t] = wrap_index(m0[1] + t - 2, g.n[1]);
        j2[t] = wrap_index(m0[2] + t - 2, g.n[2]);
    }
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        const float qa = q * w[0][a];
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            const float qab = qa * w[1][b];
            const size_t row = ((size_t)j0[a] * g.n[1] + j1[b]) * g.n[2];
#pragma unroll
            for (int e = 0; e < 5; ++e) atomicAdd(&rho[row + j2[e]], qab * w[2][e]);
        }
    }
}

__global__ void k_real_to_complex(int64_t M, const float *__restrict__ rho, float2 *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) out[i] = make_float2(rho[i], 0.0f);
}

__device__ inline float alias_poly5(float z) {
    const float z2 = z * z;
    return 1.0f + z2 * (-5.0f / 3.0f + z2 * (7.0f / 9.0f + z2 * (-17.0f / 189.0f + z2 * (2.0f / 2835.0f))));
}

__device__ inline float sinc_pi(float x) {  // sin(pi x)/(pi x)
    if (x == 0.0f) return 1.0f;
    return sinpif(x) / (3.14159265358979f * x);
}

// Pointwise in k: energy and virial partials, then the two packed spectra
//   A <- i X (k~_z + 1)  (inverse: E_z + i phi'),  B <- i X k~_x - X k~_y  (inverse: E_x + i E_y)
// with X = S G_opt and k~ the derivative wave vector (zero index at a Nyquist plane).
__global__ __launch_bounds__(256) void k_influence(MeshGeom g, Cell c, float alpha, double vol,
                                                   float2 *__restrict__ A, float2 *__restrict__ Bm,
                                                   double *__restrict__ partials) {
    const int64_t M = (int64_t)g.n[0] * g.n[1] * g.n[2];
    double red[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < M;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int j2 = (int)(idx % g.n[2]);
        const int j1 = (int)((idx / g.n[2]) % g.n[1]);
        const int j0 = (int)(idx / ((int64_t)g.n[2] * g.n[1]));
        int nv[3] = {2 * j0 < g.n[0] ? j0 : j0 - g.n[0], 2 * j1 < g.n[1] ? j1 : j1 - g.n[1],
                     2 * j2 < g.n[2] ? j2 : j2 - g.n[2]};
        const float2 S = A[idx];
        if (nv[0] == 0 && nv[1] == 0 && nv[2] == 0) {
            A[idx] = make_float2(0.f, 0.f);
            Bm[idx] = make_float2(0.f, 0.f);
            continue;
        }
        int nt[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) nt[a] = ((g.n[a] & 1) == 0 && 2 * nv[a] == -g.n[a]) ? 0 : nv[a];
        float k[3], kt[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            k[b] = (float)(2.0 * PI_D * (c.hinv[3 * b] * nv[0] + c.hinv[3 * b + 1] * nv[1] + c.hinv[3 * b + 2] * nv[2]));
            kt[b] = (float)(2.0 * PI_D * (c.hinv[3 * b] * nt[0] + c.hinv[3 * b + 1] * nt[1] + c.hinv[3 * b + 2] * nt[2]));
        }
        const float k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        const float G = (float)(2.0 * PI_D / vol) * __expf(-k2 / (4.0f * alpha * alpha)) / k2;
        float num = 1.0f, den = 1.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float x = (float)nv[a] / (float)g.n[a];
            const float sc = sinc_pi(x);
            const float sc2 = sc * sc;
            num *= sc2 * sc2 * sc;
            den *= alias_poly5(sinpif(x));
        }
        const float Gopt = G * (num * num) / (den * den);
        const float e = (float)KE * Gopt * (S.x * S.x + S.y * S.y);
        const float cB = 2.0f / (4.0f * alpha * alpha) + 2.0f / k2;
        red[0] += e;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) red[1 + 3 * a + b] += e * ((a == b ? 1.0f : 0.0f) - cB * k[a] * k[b]);
        const float2 X = make_float2(S.x * Gopt, S.y * Gopt);
        const float2 iX = make_float2(-X.y, X.x);
        A[idx] = make_float2(iX.x * (kt[2] + 1.0f), iX.y * (kt[2] + 1.0f));
        Bm[idx] = make_float2(iX.x * kt[0] - X.x * kt[1], iX.y * kt[0] - X.y * kt[1]);
    }
    block_partials<10>(red, partials);
}

// phi^k_i += 2 k_e sum_s W phi'_s,  F^k_i += -2 k_e q'_i sum_s W E_s
__global__ __launch_bounds__(256) void k_gather(int N, const float4 *__restrict__ xyzt, Cell c, MeshGeom g,
                                                const float *__restrict__ qraw, const double *__restrict__ scalars,
                                                const float2 *__restrict__ A, const float2 *__restrict__ Bm,
                                                float *__restrict__ phi, float *__restrict__ Fst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int m0[3];
    float w[3][5];
    const float4 pa = xyzt[i];
    mesh_stencil(pa.x, pa.y, pa.z, c, g, m0, w);
    int j0[5], j1[5], j2[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        j0[t] = wrap_index(m0[0] + t - 2, g.n[0]);
        j1[t] = wrap_index(m0[1] + t - 2, g.n[1]);
        j2[t] = wrap_index(m0[2] + t - 2, g.n[2]);
    }
    float ph = 0.f, ex = 0.f, ey = 0.f, ez = 0.f;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            const float wab = w[0][a] * w[1][b];
            const size_t row = ((size_t)j0[a] * g.n[1] + j1[b]) * g.n[2];
#pragma unroll
            for (int e = 0; e < 5; ++e) {
                const float ww = wab * w[2][e];
                const float2 va = A[row + j2[e]], vb = Bm[row + j2[e]];
                ez = fmaf(ww, va.x, ez);
                ph = fmaf(ww, va.y, ph);
                ex = fmaf(ww, vb.x, ex);
                ey = fmaf(ww, vb.y, ey);
            }
        }
    }
    const float q = qraw[i] + (float)scalars[S_DELTA];
    const float k2 = 2.0f * (float)KE;
    phi[i] += k2 * ph;
    Fst[i] += -k2 * q * ex;
    Fst[(size_t)N + i] += -k2 * q * ey;
    Fst[(size_t)2 * N + i] += -k2 * q * ez;
}

hipError_t launch_pppm(const Plan &p) {
    MeshGeom g{{p.mesh[0], p.mesh[1], p.mesh[2]}};
    const int64_t M = p.mesh_pts;
    const int G = (p.N + 255) / 256;
    hipError_t e = fill_zero(p.rho, sizeof(float) * (size_t)M, p.stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_spread, dim3(G), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell, g, p.qraw, p.scalars,
                       p.rho);
    const int GM = (int)((M + 255) / 256);
    hipLaunchKernelGGL(k_real_to_complex, dim3(GM), dim3(256), 0, p.stream, M, p.rho, p.meshA);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    stage_mark(p, ST_SPREAD, 3);
    e = fft3d(p.meshA, nullptr, p.mesh, -1, p.stream);
    if (e != hipSuccess) return e;
    stage_mark(p, ST_FFT_FWD, 3);
    const int GI = GM < 2048 ? GM : 2048;
    hipLaunchKernelGGL(k_influence, dim3(GI), dim3(256), 0, p.stream, g, p.cell, (float)p.alpha, p.vol, p.meshA,
                       p.meshB, p.partials);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = reduce_partials(p, GI, 10, S_UK, false);  // S_UK, S_WK[9]
    if (e != hipSuccess) return e;
    stage_mark(p, ST_INFLUENCE, 2);
    e = fft3d(p.meshA, nullptr, p.mesh, +1, p.stream);
    if (e != hipSuccess) return e;
    e = fft3d(p.meshB, nullptr, p.mesh, +1, p.stream);
    if (e != hipSuccess) return e;
    stage_mark(p, ST_FFT_INV, 6);
    hipLaunchKernelGGL(k_gather, dim3(G), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell, g, p.qraw,
                       p.scalars, p.meshA, p.meshB, p.phi, p.Fst);
    stage_mark(p, ST_GATHER);
    return hipGetLastError();
}

}  // namespace qnep
