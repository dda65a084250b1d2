// Device building blocks of the in-house FFT: complex helpers, the radix-4 DFT, and
// the length-256 line transform done as 16 x 16 in registers (four-step: a 16-point
// DFT over m of x[t + 16 m], twiddles w_256^{t k1}, an exchange through LDS so that
// thread k1 gathers the values of all t, and a second 16-point DFT, leaving
// X[k1 + 16 k2] in thread k1 at register k2 -- the load pattern).
#pragma once
#include <hip/hip_runtime.h>

namespace qnep {

__device__ inline float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
template <int SG>
__device__ inline float2 mul_i(float2 a) {  // (SG i) a
    return make_float2(-(float)SG * a.y, (float)SG * a.x);
}

template <int SG>
__device__ inline void dft4(float2 a0, float2 a1, float2 a2, float2 a3, float2 (&o)[4]) {
    const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = mul_i<SG>(csub(a1, a3));
    o[0] = cadd(t0, t2);
    o[1] = cadd(t1, t3);
    o[2] = csub(t0, t2);
    o[3] = csub(t1, t3);
}
constexpr int F256_LS = 16 * 17 + 1;  // LDS stride of one line (padded rows of 17)

template <int SG>
__device__ inline float2 w16(int e) {  // e^{SG 2 pi i e / 16}, e < 16
    constexpr float c[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                             0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                             -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
                             0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
    return make_float2(c[e], (float)SG * c[(e + 12) & 15]);  // sin(x) = cos(x - pi/2)
}

template <int SG>
__device__ inline void dft16(float2 (&a)[16]) {
    float2 y[4][4];  // y[n1][k1] = sum_n2 a[n1 + 4 n2] w4^{n2 k1}
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) dft4<SG>(a[n1], a[n1 + 4], a[n1 + 8], a[n1 + 12], y[n1]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        float2 z[4], o[4];
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) z[n1] = (n1 * k1 == 0) ? y[n1][k1] : cmul(y[n1][k1], w16<SG>(n1 * k1));
        dft4<SG>(z[0], z[1], z[2], z[3], o);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = o[k2];
    }
}

// Line transform of length 256 held by 16 threads: thread t holds x[t + 16 m] in a[m]
// and ends with X[t + 16 k2] in a[k2].  tw[m] = e^{SG 2 pi i m / 256} in LDS, ready at
// the first barrier inside; row = the line's LDS exchange area (F256_LS float2).  Every
// thread of the work-group must call it (two __syncthreads).
template <int SG>
__device__ inline void line256(float2 (&a)[16], int t, const float2 *tw, float2 *row) {
    dft16<SG>(a);
    __syncthreads();  // twiddle table ready
#pragma unroll
    for (int k1 = 1; k1 < 16; ++k1) a[k1] = cmul(a[k1], tw[t * k1]);
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) row[k1 * 17 + t] = a[k1];
    __syncthreads();
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) a[n1] = row[t * 17 + n1];
    dft16<SG>(a);
}

}  // namespace qnep
