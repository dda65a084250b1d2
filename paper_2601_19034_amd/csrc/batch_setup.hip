// Batched evaluation, setup part: parameter-independent geometry of many small
// periodic structures (neighbour lists, k-sets, phase tables and the Ewald pair
// matrices), built once per set of structures.
//
//  * descriptor neighbour lists with explicit FP32 displacement vectors (all periodic
//    images, so boxes smaller than a cutoff are handled), angular pairs first;
//  * the Ewald sum (Sec. 2.2, Eqs. 6-10) written as a pair kernel: with
//    U_ES = 1/2 sum_ij q'_i q'_j A_ij, the matrix A collects the real-space images,
//    the reciprocal sum over the k-set, the self term and the neutralising background;
//    G_ij = grad A(r_j - r_i) gives the static forces F_i = q'_i sum_j G_ij q'_j
//    (Eqs. 15, 18) and V_ij = dA_ij/d(strain) the electrostatic virial
//    W = 1/2 q'^T V q' (Eqs. 21, 22).  A and V come from per-atom phase tables
//    e^{i k.r} over the half k-set, so no transcendental is evaluated per (pair, k).
#include "batch.h"
#include "nep_math.h"
#include "plan.h"

namespace qnep {

// last s with key(s) <= x over a non-decreasing key
template <class F>
__device__ inline int last_not_above(int S, int64_t x, F key) {
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (key(mid) <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline void frac_of(const BatchStruct &b, double x, double y, double z, double *s) {
#pragma unroll
    for (int a = 0; a < 3; ++a) s[a] = x * b.hinv[a] + y * b.hinv[3 + a] + z * b.hinv[6 + a];
}

// ---------------------------------------------------------------- lists
// Per atom: every (j, n) with |r_j - r_i + n.h| < rc_R, (j, n) != (i, 0); pairs inside
// rc_A first, and inside each part grouped by the neighbour's species.  Displacements are formed in FP64 from the fractional difference
// reduced to [-1/2, 1/2] and rounded once to FP32.
__global__ __launch_bounds__(256) void k_b_lists(const BatchStruct *__restrict__ st, int S, int64_t n_total,
                                                 const float *__restrict__ pos, const int *__restrict__ type, int T,
                                                 float rcR, float rcA, float4 *__restrict__ list,
                                                 int *__restrict__ cntR, int *__restrict__ cntA, int capR,
                                                 int *__restrict__ ts, int32_t *__restrict__ flags) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_total) return;
    const int s = last_not_above(S, g, [&](int k) { return st[k].atom0; });
    const BatchStruct &b = st[s];
    const int i = (int)(g - b.atom0);
    int ti = type[g];
    if (ti < 0 || ti >= T) {
        atomicOr(flags, QNEP_FLAG_BAD_SPECIES);
        ti = 0;
    }
    ts[g] = ti;
    double si[3];
    frac_of(b, pos[g], pos[n_total + g], pos[2 * n_total + g], si);
    const double rR2 = (double)rcR * rcR, rA2 = (double)rcA * rcA;
    float4 *row = list + g * capR;
    int nR = 0, nA = 0;
    for (int pass = 0; pass < 2; ++pass)
        for (int tsel = 0; tsel < T; ++tsel) {
        for (int j = 0; j < b.n; ++j) {
            const int64_t gj = b.atom0 + j;
            int tj = type[gj];
            tj = (tj < 0 || tj >= T) ? 0 : tj;
            if (tj != tsel) continue;
            double sj[3];
            frac_of(b, pos[gj], pos[n_total + gj], pos[2 * n_total + gj], sj);
            double ds[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) ds[a] = (sj[a] - si[a]) - rint(sj[a] - si[a]);
            for (int n0 = -b.mR[0]; n0 <= b.mR[0]; ++n0)
                for (int n1 = -b.mR[1]; n1 <= b.mR[1]; ++n1)
                    for (int n2 = -b.mR[2]; n2 <= b.mR[2]; ++n2) {
                        if (j == i && n0 == 0 && n1 == 0 && n2 == 0) continue;
                        const double f0 = ds[0] + n0, f1 = ds[1] + n1, f2 = ds[2] + n2;
                        const double dx = f0 * b.h[0] + f1 * b.h[3] + f2 * b.h[6];
                        const double dy = f0 * b.h[1] + f1 * b.h[4] + f2 * b.h[7];
                        const double dz = f0 * b.h[2] + f1 * b.h[5] + f2 * b.h[8];
                        const double r2 = dx * dx + dy * dy + dz * dz;
                        const bool ang = r2 < rA2;
                        if (pass == 0 ? !ang : (ang || r2 >= rR2)) continue;
                        if (nR < capR)
                            row[nR] = make_float4((float)dx, (float)dy, (float)dz,
                                                  __int_as_float(j | (tj << 24)));
                        ++nR;
                        if (pass == 0) ++nA;
                    }
        }
        }
    if (nR > capR) atomicOr(flags, QNEP_FLAG_RADIAL_OVERFLOW);
    cntR[g] = nR < capR ? nR : capR;
    cntA[g] = nA < capR ? nA : capR;
}

// ---------------------------------------------------------------- k-set
// One block per structure: the half set of k = 2 pi h^{-T} n (n != 0, first nonzero
// component of (n_2, n_1, n_0) positive) with |k| <= kmax (or < kmax), the same rule
// as the single-structure path.  Stored as (k, w) with w = 4 k_e (2 pi / Omega)
// exp(-k^2 / 4 alpha^2) / k^2 (the half-set weight of the pair kernel), compacted in
// enumeration order.
__global__ __launch_bounds__(256) void k_b_kvec(const BatchStruct *__restrict__ st, double kmax, int kinc,
                                                double alpha, float4 *__restrict__ kv, int *__restrict__ kcount) {
    const BatchStruct &b = st[blockIdx.x];
    __shared__ int wc[4];
    const int M0 = b.kbox[0], M1 = b.kbox[1], M2 = b.kbox[2];
    const int64_t n0w = 2 * M0 + 1, n1w = 2 * M1 + 1;
    const int64_t ncand = (int64_t)(M2 + 1) * n1w * n0w;
    const double km2 = kmax * kmax;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int base = 0;
    for (int64_t c0 = 0; c0 < ncand; c0 += 256) {
        const int64_t c = c0 + threadIdx.x;
        bool keep = false;
        double kx = 0, ky = 0, kz = 0, k2 = 1;
        if (c < ncand) {
            const int a0 = (int)(c % n0w) - M0;
            const int64_t rem = c / n0w;
            const int a1 = (int)(rem % n1w) - M1;
            const int a2 = (int)(rem / n1w);
            const bool half = a2 > 0 || (a2 == 0 && (a1 > 0 || (a1 == 0 && a0 > 0)));
            kx = 2.0 * PI_D * (b.hinv[0] * a0 + b.hinv[1] * a1 + b.hinv[2] * a2);
            ky = 2.0 * PI_D * (b.hinv[3] * a0 + b.hinv[4] * a1 + b.hinv[5] * a2);
            kz = 2.0 * PI_D * (b.hinv[6] * a0 + b.hinv[7] * a1 + b.hinv[8] * a2);
            k2 = kx * kx + ky * ky + kz * kz;
            keep = half && (kinc ? (k2 <= km2 * (1.0 + 1e-9)) : (k2 < km2 * (1.0 - 1e-9)));
        }
        const uint64_t m = __ballot(keep);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wc[w] = __popcll(m);
        __syncthreads();
        int off = base;
        for (int u = 0; u < w; ++u) off += wc[u];
        const int tot = wc[0] + wc[1] + wc[2] + wc[3];
        if (keep) {
            const int slot = off + before;
            if (slot < b.kcap) {
                const double wk = 4.0 * KE * (2.0 * PI_D / b.vol) * exp(-k2 / (4.0 * alpha * alpha)) / k2;
                kv[b.k0 + slot] = make_float4((float)kx, (float)ky, (float)kz, (float)wk);
            }
        }
        base += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) kcount[blockIdx.x] = base < b.kcap ? base : b.kcap;
}

// Phase table (cos k.r_i, sin k.r_i) per structure, [k][i].  The phase is formed in
// turns from FP64 fractional coordinates (k.r = 2 pi n.s), reduced to [-1/2, 1/2] and
// evaluated in FP32.
__global__ __launch_bounds__(256) void k_b_phase(const BatchStruct *__restrict__ st, int S, int64_t total,
                                                 const float *__restrict__ pos, int64_t n_total,
                                                 const float4 *__restrict__ kv, const int *__restrict__ kcount,
                                                 float2 *__restrict__ ph) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int s = last_not_above(S, e, [&](int k) { return st[k].ph0; });
    const BatchStruct &b = st[s];
    const int64_t local = e - b.ph0;
    const int k = (int)(local / b.n), i = (int)(local % b.n);
    if (k >= kcount[s]) return;
    const int64_t g = b.atom0 + i;
    const double x = pos[g], y = pos[n_total + g], z = pos[2 * n_total + g];
    // n = h k / (2 pi): recover the integer vector from the stored k in FP64
    const float4 kk = kv[b.k0 + k];
    double nv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        nv[a] = rint((b.h[3 * a] * kk.x + b.h[3 * a + 1] * kk.y + b.h[3 * a + 2] * kk.z) / (2.0 * PI_D));
    double sf[3];
    frac_of(b, x, y, z, sf);
    double t = nv[0] * sf[0] + nv[1] * sf[1] + nv[2] * sf[2];
    t -= rint(t);
    float sn, cs;
    sincospif((float)(2.0 * t), &sn, &cs);
    ph[b.ph0 + (int64_t)k * b.n + i] = make_float2(cs, sn);
}

// ---------------------------------------------------------------- pair matrices
// One 16 x 16 tile of (i, j) per block.  Components (stored [comp][j][i]):
//   0: A_ij, 1-3: G_ij = grad A at d = r_j - r_i, 4-9: V_ij (xx, yy, zz, xy, xz, yz).
// Real space (mode 1): k_e erfc(a r)/r over images within rc (Eq. 6) with
//   u'(r) = -k_e [erfc(a r)/r^2 + 2a/sqrt(pi) exp(-a^2 r^2)/r], G += u' d/r,
//   V_ab += -u' d_a d_b / r.
// Reciprocal: sum over the half k-set of w cos(k.d), -w k sin(k.d) and
//   w (delta_ab - (2/(4a^2) + 2/k^2) k_a k_b) cos(k.d)  (Eqs. 7-9, 21, 22).
// Self (mode 1): -2 k_e a/sqrt(pi) on the diagonal (Eq. 10).  Background (mode 1, for
// a net charge): -k_e pi/(Omega a^2) on every entry and on V_aa.
__global__ __launch_bounds__(256) void k_b_matrices(const BatchStruct *__restrict__ st, int S,
                                                    const float *__restrict__ pos, int64_t n_total,
                                                    const float4 *__restrict__ kv, const int *__restrict__ kcount,
                                                    const float2 *__restrict__ ph, int mode, double alpha,
                                                    double rc, int ncomp, float *__restrict__ mats) {
    __shared__ float4 skv[64];
    __shared__ float2 spi[64][16], spj[64][16];
    const int64_t tile = blockIdx.x;
    const int s = last_not_above(S, tile, [&](int k) { return st[k].tile0; });
    const BatchStruct &b = st[s];
    const int n = b.n, nt = (n + 15) / 16;
    const int64_t local = tile - b.tile0;
    const int bi = (int)(local % nt), bj = (int)(local / nt);
    const int li = threadIdx.x & 15, lj = threadIdx.x >> 4;
    const int i = bi * 16 + li, j = bj * 16 + lj;
    const bool valid = i < n && j < n;
    double acc[BATCH_COMP_VIRIAL];
#pragma unroll
    for (int c = 0; c < BATCH_COMP_VIRIAL; ++c) acc[c] = 0.0;
    const bool vir = ncomp == BATCH_COMP_VIRIAL;
    const float cA2 = (float)(2.0 / (4.0 * alpha * alpha));
    const int nk = kcount[s];
    for (int k0 = 0; k0 < nk; k0 += 64) {
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * 32; e += 256) {
            const int kk = e >> 5, a = e & 31;
            const int k = k0 + kk;
            const int atom = a < 16 ? bi * 16 + a : bj * 16 + (a - 16);
            float2 v = make_float2(0.f, 0.f);
            if (k < nk && atom < n) v = ph[b.ph0 + (int64_t)k * n + atom];
            if (a < 16) spi[kk][a] = v;
            else spj[kk][a - 16] = v;
        }
        if (threadIdx.x < 64)
            skv[threadIdx.x] = (k0 + (int)threadIdx.x < nk) ? kv[b.k0 + k0 + threadIdx.x] : make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        float a4[BATCH_COMP_VIRIAL];
#pragma unroll
        for (int c = 0; c < BATCH_COMP_VIRIAL; ++c) a4[c] = 0.f;
        const int kend = nk - k0 < 64 ? nk - k0 : 64;
        for (int kk = 0; kk < kend; ++kk) {
            const float2 pi = spi[kk][li], pj = spj[kk][lj];
            const float cs = fmaf(pj.x, pi.x, pj.y * pi.y);   // cos k.(r_j - r_i)
            const float sn = fmaf(pj.y, pi.x, -pj.x * pi.y);  // sin k.(r_j - r_i)
            const float4 k = skv[kk];
            const float wc = k.w * cs, ws = k.w * sn;
            a4[0] += wc;
            a4[1] -= ws * k.x;
            a4[2] -= ws * k.y;
            a4[3] -= ws * k.z;
            if (vir) {
                const float k2 = k.x * k.x + k.y * k.y + k.z * k.z;
                const float cb = wc * (cA2 + 2.0f / k2);
                a4[4] += wc - cb * k.x * k.x;
                a4[5] += wc - cb * k.y * k.y;
                a4[6] += wc - cb * k.z * k.z;
                a4[7] -= cb * k.x * k.y;
                a4[8] -= cb * k.x * k.z;
                a4[9] -= cb * k.y * k.z;
            }
        }
#pragma unroll
        for (int c = 0; c < BATCH_COMP_VIRIAL; ++c) acc[c] += a4[c];
    }
    if (!valid) return;
    if (mode == 1) {
        const int64_t gi = b.atom0 + i, gj = b.atom0 + j;
        double si[3], sj[3], ds[3];
        frac_of(b, pos[gi], pos[n_total + gi], pos[2 * n_total + gi], si);
        frac_of(b, pos[gj], pos[n_total + gj], pos[2 * n_total + gj], sj);
#pragma unroll
        for (int a = 0; a < 3; ++a) ds[a] = (sj[a] - si[a]) - rint(sj[a] - si[a]);
        const double rc2 = rc * rc, tsp = 2.0 * alpha / sqrt(PI_D);
        for (int n0 = -b.mC[0]; n0 <= b.mC[0]; ++n0)
            for (int n1 = -b.mC[1]; n1 <= b.mC[1]; ++n1)
                for (int n2 = -b.mC[2]; n2 <= b.mC[2]; ++n2) {
                    if (i == j && n0 == 0 && n1 == 0 && n2 == 0) continue;
                    const double f0 = ds[0] + n0, f1 = ds[1] + n1, f2 = ds[2] + n2;
                    const double dx = f0 * b.h[0] + f1 * b.h[3] + f2 * b.h[6];
                    const double dy = f0 * b.h[1] + f1 * b.h[4] + f2 * b.h[7];
                    const double dz = f0 * b.h[2] + f1 * b.h[5] + f2 * b.h[8];
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 >= rc2) continue;
                    const double r = sqrt(r2), ir = 1.0 / r;
                    const double ec = erfc(alpha * r);
                    acc[0] += KE * ec * ir;
                    const double du = -KE * (ec * ir * ir + tsp * exp(-alpha * alpha * r2) * ir);
                    const double g = du * ir;
                    acc[1] += g * dx;
                    acc[2] += g * dy;
                    acc[3] += g * dz;
                    if (vir) {
                        acc[4] -= g * dx * dx;
                        acc[5] -= g * dy * dy;
                        acc[6] -= g * dz * dz;
                        acc[7] -= g * dx * dy;
                        acc[8] -= g * dx * dz;
                        acc[9] -= g * dy * dz;
                    }
                }
        if (i == j) acc[0] -= 2.0 * KE * alpha / sqrt(PI_D);
        const double abg = -KE * PI_D / (b.vol * alpha * alpha);
        acc[0] += abg;
        if (vir) {
            acc[4] += abg;
            acc[5] += abg;
            acc[6] += abg;
        }
    }
    const int64_t nn = (int64_t)n * n;
    for (int c = 0; c < ncomp; ++c) mats[b.mat0 + c * nn + (int64_t)j * n + i] = (float)acc[c];
}

hipError_t batch_setup(const BatchStruct *st, int S, int64_t n_total, int64_t n_tiles, int64_t ph_total,
                       const float *pos, const int *type, int T, float rcR, float rcA, float4 *list, int *cntR,
                       int *cntA, int capR, int *ts, int32_t *flags, const qnep_es_params &es, float4 *kv,
                       int *kcount, float2 *ph, int ncomp, float *mats, hipStream_t stream) {
    hipLaunchKernelGGL(k_b_lists, dim3((unsigned)((n_total + 255) / 256)), dim3(256), 0, stream, st, S, n_total, pos,
                       type, T, rcR, rcA, list, cntR, cntA, capR, ts, flags);
    hipLaunchKernelGGL(k_b_kvec, dim3(S), dim3(256), 0, stream, st, es.kmax, es.kmax_inclusive ? 1 : 0, es.alpha, kv,
                       kcount);
    if (ph_total > 0)
        hipLaunchKernelGGL(k_b_phase, dim3((unsigned)((ph_total + 255) / 256)), dim3(256), 0, stream, st, S, ph_total,
                           pos, n_total, kv, kcount, ph);
    hipLaunchKernelGGL(k_b_matrices, dim3((unsigned)n_tiles), dim3(256), 0, stream, st, S, pos, n_total, kv, kcount,
                       ph, es.mode, es.alpha, es.rc_coul, ncomp, mats);
    return hipGetLastError();
}

}  // namespace qnep
