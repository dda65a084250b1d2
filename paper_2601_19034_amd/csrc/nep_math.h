// Radial basis and angular harmonics of the NEP descriptors (FP32).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace qnep {

// sin and cos of x = (pi/2) u for u in [0, 1] by their Taylor series through x^13 and
// x^14 (truncation below 1e-9 on [0, pi/2])
__device__ inline void sincos_half_pi(float u, float &sn, float &cs) {
    const float x = 1.5707963267948966f * u, x2 = x * x;
    float ps = fmaf(-x2, 1.0f / 156.0f, 1.0f);
    ps = fmaf(-x2 * (1.0f / 110.0f), ps, 1.0f);
    ps = fmaf(-x2 * (1.0f / 72.0f), ps, 1.0f);
    ps = fmaf(-x2 * (1.0f / 42.0f), ps, 1.0f);
    ps = fmaf(-x2 * (1.0f / 20.0f), ps, 1.0f);
    ps = fmaf(-x2 * (1.0f / 6.0f), ps, 1.0f);
    sn = x * ps;
    float pc = fmaf(-x2, 1.0f / 182.0f, 1.0f);
    pc = fmaf(-x2 * (1.0f / 132.0f), pc, 1.0f);
    pc = fmaf(-x2 * (1.0f / 90.0f), pc, 1.0f);
    pc = fmaf(-x2 * (1.0f / 56.0f), pc, 1.0f);
    pc = fmaf(-x2 * (1.0f / 30.0f), pc, 1.0f);
    pc = fmaf(-x2 * (1.0f / 12.0f), pc, 1.0f);
    cs = fmaf(-x2 * 0.5f, pc, 1.0f);
}

// f_k(r) = (T_k(x) + 1)/2 * f_c(r), x = 2 (r/rc - 1)^2 - 1, f_c = (1 + cos(pi r/rc))/2,
// k = 0..NB-1, and df_k/dr, with T_k' = k U_{k-1}.
template <int NB>
__device__ inline void cheb_basis(float r, float rc, float *f, float *df) {
    const float irc = __builtin_amdgcn_rcpf(rc);  // v_rcp_f32, 1 ulp
    const float pr = 3.14159265358979f * irc;
    // f_c = cos^2(theta), theta = pi r / (2 rc): no cancellation near the cutoff
    float sh, ch;
    sincos_half_pi(r * irc, sh, ch);
    float fc = ch * ch, dfc = -pr * sh * ch;
    float t = r * irc - 1.0f;
    float x = 2.0f * t * t - 1.0f, dx = 4.0f * t * irc;
    float Tm2 = 1.0f, Tm1 = x;       // T_0, T_1
    float Um2 = 1.0f, Um1 = 2.0f * x; // U_0, U_1
    f[0] = fc;
    df[0] = dfc;
    if (NB > 1) {
        f[1] = 0.5f * (x + 1.0f) * fc;
        df[1] = 0.5f * dx * fc + 0.5f * (x + 1.0f) * dfc;
    }
#pragma unroll
    for (int k = 2; k < NB; ++k) {
        float Tk = 2.0f * x * Tm1 - Tm2;
        float dT = (float)k * Um1;  // k U_{k-1}
        f[k] = 0.5f * (Tk + 1.0f) * fc;
        df[k] = 0.5f * dT * dx * fc + 0.5f * (Tk + 1.0f) * dfc;
        float Uk = 2.0f * x * Um1 - Um2;
        Tm2 = Tm1;
        Tm1 = Tk;
        Um2 = Um1;
        Um1 = Uk;
    }
}

// Real spherical harmonics of l = 1..4 (24 values, l-major, m = -l..l), scaled so
// that sum_m Y_lm(u) Y_lm(v) = P_l(u.v) for unit vectors u, v.
__host__ __device__ inline void harmonics(float x, float y, float z, float *Y) {
    const float s3 = 1.7320508075688772f, s15 = 3.872983346207417f, s6 = 2.449489742783178f;
    const float s10 = 3.1622776601683795f, s5 = 2.23606797749979f, s35 = 5.916079783099616f;
    const float c43 = 2.091650066335189f;   // sqrt(35/2)/2
    const float c41 = 0.7905694150420949f;  // sqrt(5/2)/2
    float x2 = x * x, y2 = y * y, z2 = z * z;
    Y[0] = y;
    Y[1] = z;
    Y[2] = x;
    Y[3] = s3 * x * y;
    Y[4] = s3 * y * z;
    Y[5] = 0.5f * (3.0f * z2 - 1.0f);
    Y[6] = s3 * x * z;
    Y[7] = 0.5f * s3 * (x2 - y2);
    Y[8] = 0.25f * s10 * y * (3.0f * x2 - y2);
    Y[9] = s15 * x * y * z;
    Y[10] = 0.25f * s6 * y * (5.0f * z2 - 1.0f);
    Y[11] = 0.5f * z * (5.0f * z2 - 3.0f);
    Y[12] = 0.25f * s6 * x * (5.0f * z2 - 1.0f);
    Y[13] = 0.5f * s15 * z * (x2 - y2);
    Y[14] = 0.25f * s10 * x * (x2 - 3.0f * y2);
    Y[15] = 0.5f * s35 * x * y * (x2 - y2);
    Y[16] = c43 * y * z * (3.0f * x2 - y2);
    Y[17] = 0.5f * s5 * x * y * (7.0f * z2 - 1.0f);
    Y[18] = c41 * y * z * (7.0f * z2 - 3.0f);
    Y[19] = 0.125f * (35.0f * z2 * z2 - 30.0f * z2 + 3.0f);
    Y[20] = c41 * x * z * (7.0f * z2 - 3.0f);
    Y[21] = 0.25f * s5 * (x2 - y2) * (7.0f * z2 - 1.0f);
    Y[22] = c43 * x * z * (x2 - 3.0f * y2);
    Y[23] = 0.125f * s35 * (x2 * x2 - 6.0f * x2 * y2 + y2 * y2);
}

// sum_lm Q[lm] * grad Y_lm, with the polynomials above differentiated in x, y, z
// as independent variables (the caller projects out the radial part).
__host__ __device__ inline void harmonics_grad_dot(float x, float y, float z, const float *Q, float &gx,
                                                   float &gy, float &gz) {
    const float s3 = 1.7320508075688772f, s15 = 3.872983346207417f, s6 = 2.449489742783178f;
    const float s10 = 3.1622776601683795f, s5 = 2.23606797749979f, s35 = 5.916079783099616f;
    const float c43 = 2.091650066335189f, c41 = 0.7905694150420949f;
    float x2 = x * x, y2 = y * y, z2 = z * z;
    float ax = 0.f, ay = 0.f, az = 0.f;
    // l = 1
    ay += Q[0];
    az += Q[1];
    ax += Q[2];
    // l = 2
    ax += Q[3] * s3 * y;               ay += Q[3] * s3 * x;
    ay += Q[4] * s3 * z;               az += Q[4] * s3 * y;
    az += Q[5] * 3.0f * z;
    ax += Q[6] * s3 * z;               az += Q[6] * s3 * x;
    ax += Q[7] * s3 * x;               ay -= Q[7] * s3 * y;
    // l = 3
    ax += Q[8] * 1.5f * s10 * x * y;   ay += Q[8] * 0.75f * s10 * (x2 - y2);
    ax += Q[9] * s15 * y * z;          ay += Q[9] * s15 * x * z;          az += Q[9] * s15 * x * y;
    ay += Q[10] * 0.25f * s6 * (5.0f * z2 - 1.0f);                         az += Q[10] * 2.5f * s6 * y * z;
    az += Q[11] * (7.5f * z2 - 1.5f);
    ax += Q[12] * 0.25f * s6 * (5.0f * z2 - 1.0f);                         az += Q[12] * 2.5f * s6 * x * z;
    ax += Q[13] * s15 * x * z;         ay -= Q[13] * s15 * y * z;         az += Q[13] * 0.5f * s15 * (x2 - y2);
    ax += Q[14] * 0.75f * s10 * (x2 - y2);                                 ay -= Q[14] * 1.5f * s10 * x * y;
    // l = 4
    ax += Q[15] * 0.5f * s35 * (3.0f * x2 * y - y2 * y);
    ay += Q[15] * 0.5f * s35 * (x2 * x - 3.0f * x * y2);
    ax += Q[16] * c43 * 6.0f * x * y * z;
    ay += Q[16] * c43 * 3.0f * z * (x2 - y2);
    az += Q[16] * c43 * y * (3.0f * x2 - y2);
    ax += Q[17] * 0.5f * s5 * y * (7.0f * z2 - 1.0f);
    ay += Q[17] * 0.5f * s5 * x * (7.0f * z2 - 1.0f);
    az += Q[17] * 7.0f * s5 * x * y * z;
    ay += Q[18] * c41 * z * (7.0f * z2 - 3.0f);
    az += Q[18] * c41 * y * (21.0f * z2 - 3.0f);
    az += Q[19] * (17.5f * z2 * z - 7.5f * z);
    ax += Q[20] * c41 * z * (7.0f * z2 - 3.0f);
    az += Q[20] * c41 * x * (21.0f * z2 - 3.0f);
    ax += Q[21] * 0.5f * s5 * x * (7.0f * z2 - 1.0f);
    ay -= Q[21] * 0.5f * s5 * y * (7.0f * z2 - 1.0f);
    az += Q[21] * 3.5f * s5 * z * (x2 - y2);
    ax += Q[22] * c43 * 3.0f * z * (x2 - y2);
    ay -= Q[22] * c43 * 6.0f * x * y * z;
    az += Q[22] * c43 * x * (x2 - 3.0f * y2);
    ax += Q[23] * 0.5f * s35 * (x2 * x - 3.0f * x * y2);
    ay += Q[23] * 0.5f * s35 * (y2 * y - 3.0f * x2 * y);
    gx = ax;
    gy = ay;
    gz = az;
}

// The same gradient split in two steps, for several Q at one direction: the nonzero
// partial derivatives dY_lm/dx, /dy, /dz (16 each; lm indices in HG_X, HG_Y, HG_Z),
// then 48 FMAs per Q.
constexpr int HG_X[16] = {2, 3, 6, 7, 8, 9, 12, 13, 14, 15, 16, 17, 20, 21, 22, 23};
constexpr int HG_Y[16] = {0, 3, 4, 7, 8, 9, 10, 13, 14, 15, 16, 17, 18, 21, 22, 23};
constexpr int HG_Z[16] = {1, 4, 5, 6, 9, 10, 11, 12, 13, 16, 17, 18, 19, 20, 21, 22};
struct HarmonicsGrad {
    float cx[16], cy[16], cz[16];
};
__device__ inline HarmonicsGrad harmonics_grad(float x, float y, float z) {
    const float s3 = 1.7320508075688772f, s15 = 3.872983346207417f, s6 = 2.449489742783178f;
    const float s10 = 3.1622776601683795f, s5 = 2.23606797749979f, s35 = 5.916079783099616f;
    const float c43 = 2.091650066335189f, c41 = 0.7905694150420949f;
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    const float xy = x * y, xz = x * z, yz = y * z, xyz = xy * z;
    const float dxy = x2 - y2, z5 = 5.0f * z2 - 1.0f, z7 = 7.0f * z2 - 1.0f, z73 = 7.0f * z2 - 3.0f;
    const float z21 = 21.0f * z2 - 3.0f;
    HarmonicsGrad h;
    // d/dx for lm = 2 3 6 7 8 9 12 13 14 15 16 17 20 21 22 23
    h.cx[0] = 1.0f;
    h.cx[1] = s3 * y;
    h.cx[2] = s3 * z;
    h.cx[3] = s3 * x;
    h.cx[4] = 1.5f * s10 * xy;
    h.cx[5] = s15 * yz;
    h.cx[6] = 0.25f * s6 * z5;
    h.cx[7] = s15 * xz;
    h.cx[8] = 0.75f * s10 * dxy;
    h.cx[9] = 0.5f * s35 * (3.0f * x2 * y - y2 * y);
    h.cx[10] = c43 * 6.0f * xyz;
    h.cx[11] = 0.5f * s5 * y * z7;
    h.cx[12] = c41 * z * z73;
    h.cx[13] = 0.5f * s5 * x * z7;
    h.cx[14] = c43 * 3.0f * z * dxy;
    h.cx[15] = 0.5f * s35 * (x2 * x - 3.0f * x * y2);
    // d/dy for lm = 0 3 4 7 8 9 10 13 14 15 16 17 18 21 22 23
    h.cy[0] = 1.0f;
    h.cy[1] = s3 * x;
    h.cy[2] = s3 * z;
    h.cy[3] = -s3 * y;
    h.cy[4] = 0.75f * s10 * dxy;
    h.cy[5] = s15 * xz;
    h.cy[6] = 0.25f * s6 * z5;
    h.cy[7] = -s15 * yz;
    h.cy[8] = -1.5f * s10 * xy;
    h.cy[9] = 0.5f * s35 * (x2 * x - 3.0f * x * y2);
    h.cy[10] = c43 * 3.0f * z * dxy;
    h.cy[11] = 0.5f * s5 * x * z7;
    h.cy[12] = c41 * z * z73;
    h.cy[13] = -0.5f * s5 * y * z7;
    h.cy[14] = -c43 * 6.0f * xyz;
    h.cy[15] = 0.5f * s35 * (y2 * y - 3.0f * x2 * y);
    // d/dz for lm = 1 4 5 6 9 10 11 12 13 16 17 18 19 20 21 22
    h.cz[0] = 1.0f;
    h.cz[1] = s3 * y;
    h.cz[2] = 3.0f * z;
    h.cz[3] = s3 * x;
    h.cz[4] = s15 * xy;
    h.cz[5] = 2.5f * s6 * yz;
    h.cz[6] = 7.5f * z2 - 1.5f;
    h.cz[7] = 2.5f * s6 * xz;
    h.cz[8] = 0.5f * s15 * dxy;
    h.cz[9] = c43 * y * (3.0f * x2 - y2);
    h.cz[10] = 7.0f * s5 * xyz;
    h.cz[11] = c41 * y * z21;
    h.cz[12] = 17.5f * z2 * z - 7.5f * z;
    h.cz[13] = c41 * x * z21;
    h.cz[14] = 3.5f * s5 * z * dxy;
    h.cz[15] = c43 * x * (x2 - 3.0f * y2);
    return h;
}
__device__ inline void harmonics_grad_apply(const HarmonicsGrad &h, const float *Q, float &gx, float &gy,
                                            float &gz) {
    float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        ax = fmaf(h.cx[i], Q[HG_X[i]], ax);
        ay = fmaf(h.cy[i], Q[HG_Y[i]], ay);
        az = fmaf(h.cz[i], Q[HG_Z[i]], az);
    }
    gx = ax;
    gy = ay;
    gz = az;
}

// Directional derivative of each polynomial above along (vx, vy, vz):
// Yd[lm] = grad Y_lm(x, y, z) . v  (the caller passes a tangential v to obtain the
// derivative on the sphere).
__host__ __device__ inline void harmonics_jvp(float x, float y, float z, float vx, float vy, float vz,
                                              float *Yd) {
    const float s3 = 1.7320508075688772f, s15 = 3.872983346207417f, s6 = 2.449489742783178f;
    const float s10 = 3.1622776601683795f, s5 = 2.23606797749979f, s35 = 5.916079783099616f;
    const float c43 = 2.091650066335189f, c41 = 0.7905694150420949f;
    float x2 = x * x, y2 = y * y, z2 = z * z;
    Yd[0] = vy;
    Yd[1] = vz;
    Yd[2] = vx;
    Yd[3] = s3 * (y * vx + x * vy);
    Yd[4] = s3 * (z * vy + y * vz);
    Yd[5] = 3.0f * z * vz;
    Yd[6] = s3 * (z * vx + x * vz);
    Yd[7] = s3 * (x * vx - y * vy);
    Yd[8] = 1.5f * s10 * x * y * vx + 0.75f * s10 * (x2 - y2) * vy;
    Yd[9] = s15 * (y * z * vx + x * z * vy + x * y * vz);
    Yd[10] = 0.25f * s6 * (5.0f * z2 - 1.0f) * vy + 2.5f * s6 * y * z * vz;
    Yd[11] = (7.5f * z2 - 1.5f) * vz;
    Yd[12] = 0.25f * s6 * (5.0f * z2 - 1.0f) * vx + 2.5f * s6 * x * z * vz;
    Yd[13] = s15 * x * z * vx - s15 * y * z * vy + 0.5f * s15 * (x2 - y2) * vz;
    Yd[14] = 0.75f * s10 * (x2 - y2) * vx - 1.5f * s10 * x * y * vy;
    Yd[15] = 0.5f * s35 * ((3.0f * x2 * y - y2 * y) * vx + (x2 * x - 3.0f * x * y2) * vy);
    Yd[16] = c43 * (6.0f * x * y * z * vx + 3.0f * z * (x2 - y2) * vy + y * (3.0f * x2 - y2) * vz);
    Yd[17] = 0.5f * s5 * (7.0f * z2 - 1.0f) * (y * vx + x * vy) + 7.0f * s5 * x * y * z * vz;
    Yd[18] = c41 * (z * (7.0f * z2 - 3.0f) * vy + y * (21.0f * z2 - 3.0f) * vz);
    Yd[19] = (17.5f * z2 * z - 7.5f * z) * vz;
    Yd[20] = c41 * (z * (7.0f * z2 - 3.0f) * vx + x * (21.0f * z2 - 3.0f) * vz);
    Yd[21] = 0.5f * s5 * (7.0f * z2 - 1.0f) * (x * vx - y * vy) + 3.5f * s5 * z * (x2 - y2) * vz;
    Yd[22] = c43 * (3.0f * z * (x2 - y2) * vx - 6.0f * x * y * z * vy + x * (x2 - 3.0f * y2) * vz);
    Yd[23] = 0.5f * s35 * ((x2 * x - 3.0f * x * y2) * vx + (y2 * y - 3.0f * x2 * y) * vy);
}

}  // namespace qnep
