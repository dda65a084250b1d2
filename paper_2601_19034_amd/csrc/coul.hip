// Electrostatics on the corrected screened charges q' = q + delta:
//  * real space (mode 1, Sec. 2.2.1 Eq. 6; static pair force Eq. 15): per-atom
//    potential phi^r_i = k_e sum_j q'_j erfc(alpha r)/r, static force and virial;
//  * direct Ewald reciprocal part (Sec. 2.2.2 Eqs. 7-9, Sec. 2.3.2 Eqs. 18, 21, 22)
//    over the half set of wave vectors (S(-k) = S(k)*), with phases k.r = 2 pi n.s
//    formed in FP64 turns and reduced to [-1/2, 1/2] before the FP32 sin/cos;
//  * self and background terms (Sec. 2.2.3 Eq. 10) and the mean potential used by
//    the chain rule through the neutrality correction.
#include "plan.h"

namespace qnep {

// ---------------------------------------------------------------- real space
// RS_LANES lanes share one sorted atom i and walk the segments of its bin stencil
// (trimmed to the cutoff sphere in orthorhombic cells) with stride RS_LANES.  A
// candidate is decided by its FP32 displacement; the pair terms are evaluated without
// a branch (a candidate outside the cutoff, or i itself, gets weight zero) and give
// phi^r_i, the static pair force
// F_i = -k_e q'_i sum_j q'_j [erfc(a r)/r + 2a e^{-a^2 r^2}/sqrt(pi)] r_ij / r^2
// and the pair virial (each unordered pair is seen from both atoms with weight 1/2).
constexpr int RS_LANES = 8;
constexpr int RS_APB = 256 / RS_LANES;  // atoms per work-group
constexpr int RS_SEG = 64;              // segments of one atom held in LDS at a time
static_assert(RS_LANES <= PARTIALS_LANES_MAX, "partials buffer sized for PARTIALS_LANES_MAX lanes per atom");

// positions with the corrected charge q' in w: one 16-byte load per candidate
__global__ void k_pack_charges(int N, const float4 *__restrict__ xyzt, const float *__restrict__ qraw,
                               const double *__restrict__ scalars, float4 *__restrict__ xyzq) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float4 p = xyzt[i];
    xyzq[i] = make_float4(p.x, p.y, p.z, qraw[i] + (float)scalars[S_DELTA]);
}

// one candidate j (image shift sh) of atom i; w = 0 discards it
__device__ __forceinline__ void rs_pair(const float4 &pi, const float4 &pj, const float4 &sh, float w, float rc2f,
                                        float alpha, float c2, float (&acc)[10]) {
    // FP32 displacement: exactly antisymmetric in (i, j); across the seam its error
    // (~ulp of the box length) is negligible for this soft pair term
    const float dx = (pj.x - pi.x) + sh.x, dy = (pj.y - pi.y) + sh.y, dz = (pj.z - pi.z) + sh.z;
    const float r2 = dx * dx + dy * dy + dz * dz;
    const bool in = r2 < rc2f && r2 > 0.0f;  // r2 = 0 only for i itself
    const float qj = in ? pj.w * w : 0.0f;
    const float rr = in ? r2 : 1.0f;
    const float ir = __builtin_amdgcn_rsqf(rr);
    const float ar = alpha * (rr * ir);
    const float ex = __expf(-ar * ar);
    const float ec = erfc_as(ar, ex);
    const float eir = ec * ir;
    acc[0] = fmaf(qj, eir, acc[0]);
    const float B = qj * fmaf(c2, ex, eir) * ir * ir;
    const float bx = B * dx, by = B * dy, bz = B * dz;
    acc[1] += bx;
    acc[2] += by;
    acc[3] += bz;
    acc[4] = fmaf(bx, dx, acc[4]);
    acc[5] = fmaf(by, dy, acc[5]);
    acc[6] = fmaf(bz, dz, acc[6]);
    acc[7] = fmaf(bx, dy, acc[7]);
    acc[8] = fmaf(bx, dz, acc[8]);
    acc[9] = fmaf(by, dz, acc[9]);
}

__global__ __launch_bounds__(256) void k_real_space(int N, const float4 *__restrict__ xyzq, Cell c, Stencil st,
                                                    const int *__restrict__ start, double rc2,
                                                    const float *__restrict__ qraw,
                                                    const double *__restrict__ scalars, float alpha,
                                                    float *__restrict__ phi, float *__restrict__ Fst,
                                                    float *__restrict__ Vat, double *__restrict__ partials) {
    __shared__ int2 seg[RS_APB][RS_SEG];
    __shared__ float4 shift_tab[SEG_NIMG];
    const int nimg = 2 * st.R + 1;
    for (int k = threadIdx.x; k < nimg * nimg * nimg; k += blockDim.x) {
        int n0, n1, n2;
        image_of(k, st.R, n0, n1, n2);
        const ImageShift sh(c, n0, n1, n2);
        shift_tab[k] = make_float4(sh.fx, sh.fy, sh.fz, 0.0f);
    }
    const int a = threadIdx.x / RS_LANES, sub = threadIdx.x % RS_LANES;
    const int i = xcd_block() * RS_APB + a;
    const bool live = i < N;
    const float4 pi = xyzq[live ? i : 0];
    const AtomBin ab = atom_bin(pi, c, st);
    const float rc2f = (float)rc2;
    const float c2 = 2.0f * alpha * 0.5641895835477563f;  // 2 alpha / sqrt(pi)
    float acc[10];  // phi, B r (3), B r r (xx yy zz xy xz yz)
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[k] = 0.f;
    for (int r0 = 0; r0 < st.nrows; r0 += st.rows_chunk) {  // the same trip count in every lane
        __syncthreads();  // the previous chunk's walk is done with the table
        const int ns = stencil_segments<RS_LANES>(st, c, ab, live, sub, r0, min(st.rows_chunk, st.nrows - r0),
                                                  start, seg[a]);
        __syncthreads();
        // this lane takes candidates sub, sub + RS_LANES, ... of the concatenation, two
        // per pass with both loads issued before either is used
        SegWalk wk(seg[a], ns, sub);
        while (wk.valid()) {
            const int jA = wk.atom(), gA = wk.image();
            wk.advance(seg[a], RS_LANES);
            const bool hasB = wk.valid();
            const int jB = hasB ? wk.atom() : jA, gB = hasB ? wk.image() : gA;
            if (hasB) wk.advance(seg[a], RS_LANES);
            const float4 pa = xyzq[jA], pb = xyzq[jB];
            const float4 sa = shift_tab[gA], sb = shift_tab[gB];
            rs_pair(pi, pa, sa, 1.0f, rc2f, alpha, c2, acc);
            rs_pair(pi, pb, sb, hasB ? 1.0f : 0.0f, rc2f, alpha, c2, acc);
        }
    }
#pragma unroll
    for (int k = 0; k < 10; ++k)
#pragma unroll
        for (int o = RS_LANES / 2; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o, 64);
    double red[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (live && sub == 0) {
        const float qi = qraw[i] + (float)scalars[S_DELTA];
        const float ke = (float)KE;
        phi[i] = ke * acc[0];
        Fst[i] = -ke * qi * acc[1];
        Fst[(size_t)N + i] = -ke * qi * acc[2];
        Fst[(size_t)2 * N + i] = -ke * qi * acc[3];
        red[0] = 0.5 * (double)qi * (double)(ke * acc[0]);
        red[1] = (double)qi * (double)qi;
        const double hw = 0.5 * KE * (double)qi;
        red[2] = hw * acc[4]; red[3] = hw * acc[7]; red[4] = hw * acc[8];
        red[5] = hw * acc[7]; red[6] = hw * acc[5]; red[7] = hw * acc[9];
        red[8] = hw * acc[8]; red[9] = hw * acc[9]; red[10] = hw * acc[6];
        if (Vat) {  // per atom: half of each pair virial (xx yy zz xy xz yz)
            const float hwf = 0.5f * ke * qi;
            Vat[i] = hwf * acc[4];
            Vat[(size_t)N + i] = hwf * acc[5];
            Vat[(size_t)2 * N + i] = hwf * acc[6];
            Vat[(size_t)3 * N + i] = hwf * acc[7];
            Vat[(size_t)4 * N + i] = hwf * acc[8];
            Vat[(size_t)5 * N + i] = hwf * acc[9];
        }
    }
    block_partials<11>(red, partials);
}

hipError_t launch_real_space(const Plan &p) {
    float *Vat = p.out.virial_atom ? p.Vat : nullptr;
    if (p.mode != 1) {
        hipError_t e = fill_zero(p.phi, sizeof(float) * (size_t)p.N, p.stream);
        if (e == hipSuccess && Vat) e = fill_zero(Vat, sizeof(float) * 6 * (size_t)p.N, p.stream);
        if (e != hipSuccess) return e;
        return fill_zero(p.Fst, sizeof(float) * 3 * (size_t)p.N, p.stream);
    }
    hipLaunchKernelGGL(k_pack_charges, dim3((p.N + 255) / 256), dim3(256), 0, p.stream, p.N, p.xyzt, p.qraw,
                       p.scalars, p.xyzq);
    stage_mark(p, ST_OTHER, 1);
    Stencil st;
    if (!stencil_setup(st, p.nc, p.mC, p.cell.h, p.rc_coul, RS_SEG)) return hipErrorInvalidValue;
    const int G = (p.N + RS_APB - 1) / RS_APB;
    hipLaunchKernelGGL(k_real_space, dim3(G), dim3(256), 0, p.stream, p.N, p.xyzq, p.cell, st, p.cell_start,
                       p.rc_coul * p.rc_coul, p.qraw, p.scalars, (float)p.alpha, p.phi, p.Fst, Vat, p.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    stage_mark(p, ST_REAL, 1);
    return reduce_partials(p, G, 11, S_UREAL, false);  // S_UREAL, S_QSQ, S_WREAL[9]
}

// ---------------------------------------------------------------- Ewald
// Builds the half set {n : n3 > 0, or n3 = 0 and n2 > 0, or n3 = n2 = 0 and n1 > 0}
// with |k| within kmax, k = 2 pi h^{-1} n, in box order (deterministic).  One block.
__global__ void k_kvectors(Cell c, int M0, int M1, int M2, double kmax2, int inclusive, double alpha,
                           double vol, int64_t cap, float4 *__restrict__ kv, int4 *__restrict__ kn,
                           int *__restrict__ kcount) {
    __shared__ int scan[1024];
    __shared__ int base;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    const int n0 = 2 * M0 + 1, n1w = 2 * M1 + 1;
    const int64_t total = (int64_t)n0 * n1w * (M2 + 1);
    for (int64_t b = 0; b < total; b += 1024) {
        int64_t idx = b + threadIdx.x;
        int keep = 0;
        int a0 = 0, a1 = 0, a2 = 0;
        double kx = 0, ky = 0, kz = 0, k2 = 0;
        if (idx < total) {
            a2 = (int)(idx / ((int64_t)n0 * n1w));
            int rem = (int)(idx % ((int64_t)n0 * n1w));
            a1 = rem / n0 - M1;
            a0 = rem % n0 - M0;
            bool half = a2 > 0 || (a2 == 0 && (a1 > 0 || (a1 == 0 && a0 > 0)));
            if (half) {
                kx = 2.0 * PI_D * (c.hinv[0] * a0 + c.hinv[1] * a1 + c.hinv[2] * a2);
                ky = 2.0 * PI_D * (c.hinv[3] * a0 + c.hinv[4] * a1 + c.hinv[5] * a2);
                kz = 2.0 * PI_D * (c.hinv[6] * a0 + c.hinv[7] * a1 + c.hinv[8] * a2);
                k2 = kx * kx + ky * ky + kz * kz;
                keep = inclusive ? (k2 <= kmax2 * (1.0 + 1e-9)) : (k2 < kmax2 * (1.0 - 1e-9));
            }
        }
        scan[threadIdx.x] = keep;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            int t = threadIdx.x >= (unsigned)o ? scan[threadIdx.x - o] : 0;
            __syncthreads();
            scan[threadIdx.x] += t;
            __syncthreads();
        }
        if (keep) {
            int64_t pos = base + scan[threadIdx.x] - 1;
            if (pos < cap) {
                double G = 2.0 * PI_D / vol * exp(-k2 / (4.0 * alpha * alpha)) / k2;
                kv[pos] = make_float4((float)kx, (float)ky, (float)kz, (float)G);
                kn[pos] = make_int4(a0, a1, a2, 0);
            }
        }
        __syncthreads();
        if (threadIdx.x == 1023) base += scan[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *kcount = base < cap ? base : (int)cap;
}

// fractional coordinates wrapped to [0, 1) in FP64
__device__ inline void frac_coords(double x, double y, double z, const Cell &c, double &s0, double &s1,
                                   double &s2) {
    s0 = x * c.hinv[0] + y * c.hinv[3] + z * c.hinv[6];
    s1 = x * c.hinv[1] + y * c.hinv[4] + z * c.hinv[7];
    s2 = x * c.hinv[2] + y * c.hinv[5] + z * c.hinv[8];
    s0 -= floor(s0);
    s1 -= floor(s1);
    s2 -= floor(s2);
}

// cos and sin of 2 pi n.s
__device__ inline void phase_cs(int n0, int n1, int n2, double s0, double s1, double s2, float &cs, float &sn) {
    double t = (double)n0 * s0 + (double)n1 * s1 + (double)n2 * s2;
    t -= rint(t);
    sincospif(2.0f * (float)t, &sn, &cs);
}

constexpr int EW_CHUNK = 512;

// partial structure factors: block (kb, chunk); each thread owns one wave vector
__global__ __launch_bounds__(256) void k_structure_factor(int N, const float4 *__restrict__ xyzt, Cell c,
                                                          const float *__restrict__ qraw,
                                                          const double *__restrict__ scalars,
                                                          const int4 *__restrict__ kn,
                                                          const int *__restrict__ kcount, int64_t cap,
                                                          float2 *__restrict__ Spart) {
    __shared__ double sx[256], sy[256], sz[256];
    __shared__ float sq[256];
    const int nk = *kcount;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int a0 = blockIdx.y * EW_CHUNK, a1 = min(N, a0 + EW_CHUNK);
    const float delta = (float)scalars[S_DELTA];
    int4 n = k < nk ? kn[k] : make_int4(0, 0, 0, 0);
    float re = 0.f, im = 0.f;
    for (int t0 = a0; t0 < a1; t0 += 256) {
        int a = t0 + threadIdx.x;
        if (a < a1) {
            double s0, s1, s2;
            const float4 pa = xyzt[a];
            frac_coords(pa.x, pa.y, pa.z, c, s0, s1, s2);
            sx[threadIdx.x] = s0;
            sy[threadIdx.x] = s1;
            sz[threadIdx.x] = s2;
            sq[threadIdx.x] = qraw[a] + delta;
        }
        __syncthreads();
        const int m = min(256, a1 - t0);
        if (k < nk) {
            for (int u = 0; u < m; ++u) {
                float cs, sn;
                phase_cs(n.x, n.y, n.z, sx[u], sy[u], sz[u], cs, sn);
                re = fmaf(sq[u], cs, re);
                im = fmaf(-sq[u], sn, im);
            }
        }
        __syncthreads();
    }
    if (k < nk) Spart[(size_t)blockIdx.y * cap + k] = make_float2(re, im);
}

// S(k) = sum over chunks (FP64); energy 2 k_e G |S|^2 and virial 2 k_e G |S|^2 B(k)
__global__ __launch_bounds__(256) void k_structure_reduce(int nchunks, const float2 *__restrict__ Spart,
                                                          const float4 *__restrict__ kv,
                                                          const int *__restrict__ kcount, int64_t cap,
                                                          double alpha, float2 *__restrict__ Sk,
                                                          double *__restrict__ partials) {
    const int nk = *kcount;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double red[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (k < nk) {
        double re = 0.0, im = 0.0;
        for (int ch = 0; ch < nchunks; ++ch) {
            float2 v = Spart[(size_t)ch * cap + k];
            re += v.x;
            im += v.y;
        }
        Sk[k] = make_float2((float)re, (float)im);
        float4 q = kv[k];
        double kx = q.x, ky = q.y, kz = q.z, G = q.w;
        double k2 = kx * kx + ky * ky + kz * kz;
        double e = 2.0 * KE * G * (re * re + im * im);
        double cB = 2.0 / (4.0 * alpha * alpha) + 2.0 / k2;
        double kk[3] = {kx, ky, kz};
        red[0] = e;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) red[1 + 3 * a + b] = e * ((a == b ? 1.0 : 0.0) - cB * kk[a] * kk[b]);
    }
    block_partials<10>(red, partials);
}

// phi^k_i = 4 k_e sum_half G Re[S e^{i k.r_i}],  F^k_i = 4 k_e q'_i sum_half k G Im[S e^{i k.r_i}]
__global__ __launch_bounds__(256) void k_ewald_atoms(int N, const float4 *__restrict__ xyzt, Cell c,
                                                     const float *__restrict__ qraw,
                                                     const double *__restrict__ scalars,
                                                     const float4 *__restrict__ kv, const int4 *__restrict__ kn,
                                                     const float2 *__restrict__ Sk, const int *__restrict__ kcount,
                                                     float *__restrict__ phi, float *__restrict__ Fst) {
    __shared__ int4 ln[256];
    __shared__ float4 lk[256];
    __shared__ float2 ls[256];
    const int nk = *kcount;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double s0 = 0, s1 = 0, s2 = 0;
    if (i < N) {
        const float4 pa = xyzt[i];
        frac_coords(pa.x, pa.y, pa.z, c, s0, s1, s2);
    }
    float ph = 0.f, fx = 0.f, fy = 0.f, fz = 0.f;
    for (int t0 = 0; t0 < nk; t0 += 256) {
        int k = t0 + threadIdx.x;
        if (k < nk) {
            ln[threadIdx.x] = kn[k];
            lk[threadIdx.x] = kv[k];
            ls[threadIdx.x] = Sk[k];
        }
        __syncthreads();
        const int m = min(256, nk - t0);
        if (i < N) {
            for (int u = 0; u < m; ++u) {
                float cs, sn;
                int4 n = ln[u];
                phase_cs(n.x, n.y, n.z, s0, s1, s2, cs, sn);
                float2 S = ls[u];
                float4 q = lk[u];
                float re = S.x * cs - S.y * sn;
                float im = S.x * sn + S.y * cs;
                ph = fmaf(q.w, re, ph);
                float gi = q.w * im;
                fx = fmaf(q.x, gi, fx);
                fy = fmaf(q.y, gi, fy);
                fz = fmaf(q.z, gi, fz);
            }
        }
        __syncthreads();
    }
    if (i < N) {
        const float qi = qraw[i] + (float)scalars[S_DELTA];
        const float k4 = 4.0f * (float)KE;
        phi[i] += k4 * ph;
        Fst[i] += k4 * qi * fx;
        Fst[(size_t)N + i] += k4 * qi * fy;
        Fst[(size_t)2 * N + i] += k4 * qi * fz;
    }
}

// per-atom reciprocal virial (Eq. 20) over the half set: W^k_i = 2 k_e q'_i sum_half G
// Re[S e^{i k.r_i}] B(k), B = I - (2/(4 alpha^2) + 2/k^2) k k; added to Vat
__global__ __launch_bounds__(256) void k_ewald_virial_atoms(int N, const float4 *__restrict__ xyzt, Cell c,
                                                            float alpha, const float *__restrict__ qraw,
                                                            const double *__restrict__ scalars,
                                                            const float4 *__restrict__ kv,
                                                            const int4 *__restrict__ kn,
                                                            const float2 *__restrict__ Sk,
                                                            const int *__restrict__ kcount, float *__restrict__ Vat) {
    __shared__ int4 ln[256];
    __shared__ float4 lk[256];
    __shared__ float2 ls[256];
    const int nk = *kcount;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const float cB0 = 2.0f / (4.0f * alpha * alpha);
    double s0 = 0, s1 = 0, s2 = 0;
    if (i < N) {
        const float4 pa = xyzt[i];
        frac_coords(pa.x, pa.y, pa.z, c, s0, s1, s2);
    }
    float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // xx yy zz xy xz yz
    for (int t0 = 0; t0 < nk; t0 += 256) {
        int k = t0 + threadIdx.x;
        if (k < nk) {
            ln[threadIdx.x] = kn[k];
            lk[threadIdx.x] = kv[k];
            ls[threadIdx.x] = Sk[k];
        }
        __syncthreads();
        const int m = min(256, nk - t0);
        if (i < N) {
            for (int u = 0; u < m; ++u) {
                float cs, sn;
                int4 n = ln[u];
                phase_cs(n.x, n.y, n.z, s0, s1, s2, cs, sn);
                const float2 S = ls[u];
                const float4 q = lk[u];
                const float gre = q.w * (S.x * cs - S.y * sn);
                const float k2 = q.x * q.x + q.y * q.y + q.z * q.z;
                const float cb = gre * (cB0 + 2.0f / k2);
                v[0] = fmaf(-cb * q.x, q.x, v[0] + gre);
                v[1] = fmaf(-cb * q.y, q.y, v[1] + gre);
                v[2] = fmaf(-cb * q.z, q.z, v[2] + gre);
                v[3] = fmaf(-cb * q.x, q.y, v[3]);
                v[4] = fmaf(-cb * q.x, q.z, v[4]);
                v[5] = fmaf(-cb * q.y, q.z, v[5]);
            }
        }
        __syncthreads();
    }
    if (i < N) {
        const float f = 2.0f * (float)KE * (qraw[i] + (float)scalars[S_DELTA]);
#pragma unroll
        for (int k = 0; k < 6; ++k) Vat[(size_t)k * N + i] += f * v[k];
    }
}

hipError_t launch_ewald(const Plan &p) {
    int4 *kn = (int4 *)(p.kvec + p.nk_cap);
    hipLaunchKernelGGL(k_kvectors, dim3(1), dim3(1024), 0, p.stream, p.cell, p.nk_box[0], p.nk_box[1],
                       p.nk_box[2], p.kmax * p.kmax, p.kinc, p.alpha, p.vol, p.nk_cap, p.kvec, kn, p.kcount);
    const int kb = (int)((p.nk_cap + 255) / 256);
    hipLaunchKernelGGL(k_structure_factor, dim3(kb, p.s_chunks), dim3(256), 0, p.stream, p.N, p.xyzt,
                       p.cell, p.qraw, p.scalars, (const int4 *)kn, p.kcount, p.nk_cap, p.Spart);
    hipLaunchKernelGGL(k_structure_reduce, dim3(kb), dim3(256), 0, p.stream, p.s_chunks, p.Spart, p.kvec,
                       p.kcount, p.nk_cap, p.alpha, p.Sk, p.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = reduce_partials(p, kb, 10, S_UK, false);  // S_UK, S_WK[9]
    if (e != hipSuccess) return e;
    stage_mark(p, ST_EWALD_SK, 4);
    const int G = (p.N + 255) / 256;
    hipLaunchKernelGGL(k_ewald_atoms, dim3(G), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell, p.qraw,
                       p.scalars, p.kvec, (const int4 *)kn, p.Sk, p.kcount, p.phi, p.Fst);
    if (p.out.virial_atom)
        hipLaunchKernelGGL(k_ewald_virial_atoms, dim3(G), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell,
                           (float)p.alpha, p.qraw, p.scalars, p.kvec, (const int4 *)kn, p.Sk, p.kcount, p.Vat);
    stage_mark(p, ST_EWALD_ATOMS, p.out.virial_atom ? 2 : 1);
    return hipGetLastError();
}

// ---------------------------------------------------------------- potential centring
// phi_i += self (-2 k_e alpha q'_i / sqrt(pi)) and background terms (mode 1);
// FP64 partials of sum phi for the mean used in chi_i = phi_i - mean(phi).
__global__ __launch_bounds__(256) void k_phi_total(int N, int mode, float alpha, double vol, double qtot,
                                                   const float *__restrict__ qraw,
                                                   const double *__restrict__ scalars,
                                                   const float *__restrict__ theta, int64_t off_s,
                                                   float *__restrict__ phi, double *__restrict__ partials) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double red[1] = {0.0};
    if (i < N) {
        float v = phi[i];
        if (mode == 1) {
            const float qi = qraw[i] + (float)scalars[S_DELTA];
            const double Qs = qtot / (double)theta[off_s];
            v += -2.0f * (float)KE * alpha * 0.5641895835477563f * qi;
            v += (float)(-KE * PI_D * Qs / (vol * (double)alpha * (double)alpha));
            phi[i] = v;
        }
        red[0] = v;
    }
    block_partials<1>(red, partials);
}

__global__ void k_phi_mean(int N, double *__restrict__ scalars) {
    if (threadIdx.x == 0) scalars[S_PHIBAR] = scalars[S_SUMPHI] / (double)N;
}

hipError_t launch_phi_mean(const Plan &p) {
    const int G = (p.N + 255) / 256;
    hipLaunchKernelGGL(k_phi_total, dim3(G), dim3(256), 0, p.stream, p.N, p.mode, (float)p.alpha, p.vol, p.qtot,
                       p.qraw, p.scalars, p.theta, p.off_s, p.phi, p.partials);
    hipError_t e = reduce_partials(p, G, 1, S_SUMPHI, false);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_phi_mean, dim3(1), dim3(64), 0, p.stream, p.N, p.scalars);
    return hipGetLastError();
}

}  // namespace qnep
