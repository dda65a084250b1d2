// Batched evaluation: many small periodic structures, each under many candidate
// parameter vectors, in one persistent launch, with the energy, force and
// total-charge terms of the training loss (Sec. 2.5).
//
// Setup (independent of the parameters, once per set of structures):
//  * descriptor neighbour lists with explicit FP32 displacement vectors (all periodic
//    images, so boxes smaller than a cutoff are handled), angular pairs first;
//  * the Ewald sum (Sec. 2.2, Eqs. 6-10) written as a pair kernel: with
//    U_ES = 1/2 sum_ij q'_i q'_j A_ij, the matrix A collects the real-space images,
//    the reciprocal sum over the k-set, the self term and the neutralising background;
//    G_ij = grad A(r_j - r_i) gives the static forces F_i = q'_i sum_j G_ij q'_j
//    (Eqs. 15, 18) and V_ij = dA_ij/d(strain) the electrostatic virial
//    W = 1/2 q'^T V q' (Eqs. 21, 22).  A and V come from per-atom phase tables
//    e^{i k.r} over the half k-set, so no transcendental is evaluated per (pair, k).
//
// Evaluation: one workgroup per (structure, candidate) work item pulled from an
// atomic queue (largest structures first).  Per item: parameters staged in LDS,
// descriptors (Sec. 2.1), network (Eq. 1), charge scaling and neutrality correction
// (Sec. 2.5), potentials phi = A q', chi = phi - mean(phi), partial forces
// F_ij = g_i . dD_i/dr_ij with g_i = dU_i/dD + chi_i dq_i/dD (Sec. 2.3), F_j
// accumulated with LDS atomics, then E, W and the losses.
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
// rc_A first.  Displacements are formed in FP64 from the fractional difference
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
    for (int pass = 0; pass < 2; ++pass) {
        for (int j = 0; j < b.n; ++j) {
            const int64_t gj = b.atom0 + j;
            double sj[3];
            frac_of(b, pos[gj], pos[n_total + gj], pos[2 * n_total + gj], sj);
            int tj = type[gj];
            tj = (tj < 0 || tj >= T) ? 0 : tj;
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

// ---------------------------------------------------------------- persistent evaluation
// sums NV doubles over the block; every thread receives the totals
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == 0) red[w * NV + k] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = red[k] + red[NV + k] + red[2 * NV + k] + red[3 * NV + k];
    __syncthreads();
}

// sum over the G lanes of an aligned lane group (all lanes receive the total)
__device__ inline float group_sum(float v, int G) {
    for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int T, int NR, int NA, int NB>
__global__ __launch_bounds__(BATCH_THREADS) void k_batch_eval(BatchArgs a, int item_begin, int item_end,
                                                              int4 groups) {
    constexpr int NDES = NR + 4 * NA;
    extern __shared__ float lds[];
    __shared__ double red[4 * 16];
    __shared__ int s_item;
    float *th = lds;                             // parameters of the candidate
    float *qv = lds + a.n_theta;                 // q' per atom
    float *phi = qv + a.max_atoms;               // potential, then chi
    float *fx = phi + a.max_atoms, *fy = fx + a.max_atoms, *fz = fy + a.max_atoms;
    const int tid = threadIdx.x;
    const int M = a.max_atoms;
    float *scr = a.scratch + (size_t)blockIdx.x * (3 * NDES + LM * NA) * M;
    float *sD = scr, *sA = scr + (size_t)NDES * M, *sgU = sA + (size_t)LM * NA * M, *sgq = sgU + (size_t)NDES * M;
    const float *cR = th, *cA = th + a.off_cA;
    const float *nnet = th + a.off_nn;

    for (;;) {
        if (tid == 0) s_item = item_begin + atomicAdd(a.counter, 1);
        __syncthreads();
        const int item = s_item;
        if (item >= item_end) break;
        const int s = a.order[item / a.C], c = item % a.C;
        const BatchStruct &b = a.st[s];
        const int n = b.n;
        const int G = b.group == 0 ? groups.x : (b.group == 1 ? groups.y : (b.group == 2 ? groups.z : groups.w));
        const int per_round = BATCH_THREADS / G;
        const int lig = tid % G, grp = tid / G;
        const float *thc = a.thetas + (size_t)c * a.n_theta;
        for (int k = tid; k < a.n_theta; k += BATCH_THREADS) th[k] = thc[k];
        __syncthreads();
        const float sc = th[a.off_s];
        const float b1E = th[a.off_b1E];

        // ---- descriptors
        for (int i0 = 0; i0 < n; i0 += per_round) {
            const int i = i0 + grp;
            const bool act = i < n;
            const int64_t g = b.atom0 + (act ? i : 0);
            const int tI = act ? a.types[g] : 0;
            const float4 *row = a.list + g * a.capR;
            const int nR = act ? a.cntR[g] : 0, nA = act ? a.cntA[g] : 0;
            float B[T][NB];
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int k = 0; k < NB; ++k) B[t][k] = 0.f;
            float Am[NA][LM];
#pragma unroll
            for (int q = 0; q < NA; ++q)
#pragma unroll
                for (int m = 0; m < LM; ++m) Am[q][m] = 0.f;
            for (int p = lig; p < nR; p += G) {
                const float4 e = row[p];
                const int tj = __float_as_int(e.w) >> 24;
                const float r = sqrtf(e.x * e.x + e.y * e.y + e.z * e.z);
                float f[NB], df[NB];
                cheb_basis<NB>(r, a.rcR, f, df);
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    const float msk = tj == t ? 1.f : 0.f;
#pragma unroll
                    for (int k = 0; k < NB; ++k) B[t][k] = fmaf(msk, f[k], B[t][k]);
                }
                if (p < nA) {
                    cheb_basis<NB>(r, a.rcA, f, df);
                    const float *cp = cA + (tI * T + tj) * NA * NB;
                    const float ir = 1.0f / r;
                    float Y[LM];
                    harmonics(e.x * ir, e.y * ir, e.z * ir, Y);
#pragma unroll
                    for (int q = 0; q < NA; ++q) {
                        float gn = 0.f;
#pragma unroll
                        for (int k = 0; k < NB; ++k) gn = fmaf(cp[q * NB + k], f[k], gn);
#pragma unroll
                        for (int m = 0; m < LM; ++m) Am[q][m] = fmaf(gn, Y[m], Am[q][m]);
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int k = 0; k < NB; ++k) B[t][k] = group_sum(B[t][k], G);
#pragma unroll
            for (int q = 0; q < NA; ++q)
#pragma unroll
                for (int m = 0; m < LM; ++m) Am[q][m] = group_sum(Am[q][m], G);
            if (act) {
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    if (q % G != lig) continue;
                    float acc = 0.f;
#pragma unroll
                    for (int t = 0; t < T; ++t)
#pragma unroll
                        for (int k = 0; k < NB; ++k) acc = fmaf(cR[((tI * T + t) * NR + q) * NB + k], B[t][k], acc);
                    sD[(size_t)q * M + i] = acc;
                }
#pragma unroll
                for (int q = 0; q < NA; ++q) {
                    if ((NR + q) % G != lig) continue;
                    float s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
#pragma unroll
                    for (int m = 0; m < 3; ++m) s1 = fmaf(Am[q][m], Am[q][m], s1);
#pragma unroll
                    for (int m = 3; m < 8; ++m) s2 = fmaf(Am[q][m], Am[q][m], s2);
#pragma unroll
                    for (int m = 8; m < 15; ++m) s3 = fmaf(Am[q][m], Am[q][m], s3);
#pragma unroll
                    for (int m = 15; m < 24; ++m) s4 = fmaf(Am[q][m], Am[q][m], s4);
                    sD[(size_t)(NR + 0 * NA + q) * M + i] = s1;
                    sD[(size_t)(NR + 1 * NA + q) * M + i] = s2;
                    sD[(size_t)(NR + 2 * NA + q) * M + i] = s3;
                    sD[(size_t)(NR + 3 * NA + q) * M + i] = s4;
#pragma unroll
                    for (int m = 0; m < LM; ++m) sA[(size_t)(q * LM + m) * M + i] = Am[q][m];
                }
            }
        }
        __syncthreads();

        // ---- network (FP32): hidden units split over the lanes of a group
        double accU = 0.0, accQ = 0.0;
        for (int i0 = 0; i0 < n; i0 += per_round) {
            const int i = i0 + grp;
            const bool act = i < n;
            const int tI = act ? a.types[b.atom0 + i] : 0;
            float Dv[NDES];
#pragma unroll
            for (int d = 0; d < NDES; ++d) Dv[d] = act ? sD[(size_t)d * M + i] : 0.f;
            const float *W0 = nnet + tI * a.per_species;
            const float *b0 = W0 + a.H * NDES, *w1E = b0 + a.H, *w1q = w1E + a.H;
            float gu[NDES], gqv[NDES];
#pragma unroll
            for (int d = 0; d < NDES; ++d) gu[d] = gqv[d] = 0.f;
            float up = 0.f, qp = 0.f;
            for (int jn = lig; jn < a.H; jn += G) {
                const float *w = W0 + jn * NDES;
                float z = -b0[jn];
#pragma unroll
                for (int d = 0; d < NDES; ++d) z = fmaf(w[d], Dv[d], z);
                const float hh = tanhf(z);
                up = fmaf(w1E[jn], hh, up);
                qp = fmaf(w1q[jn], hh, qp);
                const float dh = 1.0f - hh * hh;
                const float ae = dh * w1E[jn], aq = dh * w1q[jn];
#pragma unroll
                for (int d = 0; d < NDES; ++d) {
                    gu[d] = fmaf(ae, w[d], gu[d]);
                    gqv[d] = fmaf(aq, w[d], gqv[d]);
                }
            }
            up = group_sum(up, G);
            qp = group_sum(qp, G);
#pragma unroll
            for (int d = 0; d < NDES; ++d) {
                gu[d] = group_sum(gu[d], G);
                gqv[d] = group_sum(gqv[d], G);
            }
            if (act) {
#pragma unroll
                for (int d = 0; d < NDES; ++d) {
                    if (d % G != lig) continue;
                    sgU[(size_t)d * M + i] = gu[d];
                    sgq[(size_t)d * M + i] = gqv[d];
                }
                if (lig == 0) {
                    const float qi = qp - w1q[a.H];  // b1q follows w1q
                    qv[i] = qi;
                    accU += (double)(up - b1E);
                    accQ += (double)qi;
                }
            }
        }
        double r1[2] = {accU, accQ};
        block_sum<2>(r1, red);
        const double sumU = r1[0], sumq = r1[1];
        // neutrality correction on the scaled charges: q~' = s q + (Q - s sum q)/N, q' = q~'/s
        const float delta = (float)((a.qtot / (double)sc - sumq) / n);
        for (int i = tid; i < n; i += BATCH_THREADS) qv[i] += delta;
        __syncthreads();

        // ---- electrostatics: y = M q' for every stored component
        double accP = 0.0, accE = 0.0, wes[6] = {0, 0, 0, 0, 0, 0};
        {
            const int64_t nn = (int64_t)n * n;
            const float *Mb = a.mats + b.mat0;
            const int units = a.ncomp * n;
            for (int u = tid; u < units; u += BATCH_THREADS) {
                const int comp = u / n, i = u - comp * n;
                const float *col = Mb + comp * nn + i;
                float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
                int j = 0;
                for (; j + 3 < n; j += 4) {
                    s0 = fmaf(col[(int64_t)j * n], qv[j], s0);
                    s1 = fmaf(col[(int64_t)(j + 1) * n], qv[j + 1], s1);
                    s2 = fmaf(col[(int64_t)(j + 2) * n], qv[j + 2], s2);
                    s3 = fmaf(col[(int64_t)(j + 3) * n], qv[j + 3], s3);
                }
                for (; j < n; ++j) s0 = fmaf(col[(int64_t)j * n], qv[j], s0);
                const float y = (s0 + s1) + (s2 + s3);
                const float qi = qv[i];
                if (comp == 0) {
                    phi[i] = y;
                    accP += (double)y;
                    accE += 0.5 * (double)qi * (double)y;
                } else if (comp == 1) {
                    fx[i] = qi * y;
                } else if (comp == 2) {
                    fy[i] = qi * y;
                } else if (comp == 3) {
                    fz[i] = qi * y;
                } else {
                    const double v = 0.5 * (double)qi * (double)y;
                    wes[0] += comp == 4 ? v : 0.0;
                    wes[1] += comp == 5 ? v : 0.0;
                    wes[2] += comp == 6 ? v : 0.0;
                    wes[3] += comp == 7 ? v : 0.0;
                    wes[4] += comp == 8 ? v : 0.0;
                    wes[5] += comp == 9 ? v : 0.0;
                }
            }
        }
        double r2[8] = {accP, accE, wes[0], wes[1], wes[2], wes[3], wes[4], wes[5]};
        block_sum<8>(r2, red);
        const float phibar = (float)(r2[0] / n);
        const double Ues = r2[1];
        for (int i = tid; i < n; i += BATCH_THREADS) phi[i] -= phibar;  // chi
        __syncthreads();

        // ---- partial forces
        float m9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int i0 = 0; i0 < n; i0 += per_round) {
            const int i = i0 + grp;
            const bool act = i < n;
            const int64_t g = b.atom0 + (act ? i : 0);
            const int tI = act ? a.types[g] : 0;
            const float chi = act ? phi[i] : 0.f;
            const float4 *row = a.list + g * a.capR;
            const int nR = act ? a.cntR[g] : 0, nA = act ? a.cntA[g] : 0;
            float ox = 0.f, oy = 0.f, oz = 0.f;
            {  // radial: e[t][k] = sum_n g_n cR[ti][t][n][k],  F_ij = (sum_k e[tj][k] f_k'(r)) r_hat
                float gR[NR];
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    gR[q] = act ? fmaf(chi, sgq[(size_t)q * M + i], sgU[(size_t)q * M + i]) : 0.f;
                float ev[T][NB];
#pragma unroll
                for (int t = 0; t < T; ++t)
#pragma unroll
                    for (int k = 0; k < NB; ++k) {
                        float acc = 0.f;
#pragma unroll
                        for (int q = 0; q < NR; ++q) acc = fmaf(gR[q], cR[((tI * T + t) * NR + q) * NB + k], acc);
                        ev[t][k] = acc;
                    }
                for (int p = lig; p < nR; p += G) {
                    const float4 e = row[p];
                    const int code = __float_as_int(e.w);
                    const int tj = code >> 24, j = code & 0xFFFFFF;
                    const float r = sqrtf(e.x * e.x + e.y * e.y + e.z * e.z);
                    float f[NB], df[NB];
                    cheb_basis<NB>(r, a.rcR, f, df);
                    float w = 0.f;
#pragma unroll
                    for (int t = 0; t < T; ++t) {
                        float acc = 0.f;
#pragma unroll
                        for (int k = 0; k < NB; ++k) acc = fmaf(ev[t][k], df[k], acc);
                        w = tj == t ? acc : w;
                    }
                    const float ir = w / r;
                    const float Fx = ir * e.x, Fy = ir * e.y, Fz = ir * e.z;
                    ox += Fx;
                    oy += Fy;
                    oz += Fz;
                    atomicAdd(&fx[j], -Fx);
                    atomicAdd(&fy[j], -Fy);
                    atomicAdd(&fz[j], -Fz);
                    m9[0] -= Fx * e.x; m9[1] -= Fx * e.y; m9[2] -= Fx * e.z;
                    m9[3] -= Fy * e.x; m9[4] -= Fy * e.y; m9[5] -= Fy * e.z;
                    m9[6] -= Fz * e.x; m9[7] -= Fz * e.y; m9[8] -= Fz * e.z;
                }
            }
            {  // angular: At_nlm = 2 g_nl A_nlm; per pair the derivative of sum At_nlm g_n Y_lm
                float At[NA][LM];
#pragma unroll
                for (int q = 0; q < NA; ++q) {
                    float Gl[4];
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        const size_t rw = (size_t)(NR + l * NA + q) * M + i;
                        Gl[l] = act ? 2.0f * fmaf(chi, sgq[rw], sgU[rw]) : 0.f;
                    }
#pragma unroll
                    for (int m = 0; m < LM; ++m) {
                        const int l = m < 3 ? 0 : (m < 8 ? 1 : (m < 15 ? 2 : 3));
                        At[q][m] = act ? Gl[l] * sA[(size_t)(q * LM + m) * M + i] : 0.f;
                    }
                }
                for (int p = lig; p < nA; p += G) {
                    const float4 e = row[p];
                    const int code = __float_as_int(e.w);
                    const int tj = code >> 24, j = code & 0xFFFFFF;
                    const float r = sqrtf(e.x * e.x + e.y * e.y + e.z * e.z);
                    const float ir = 1.0f / r;
                    const float ux = e.x * ir, uy = e.y * ir, uz = e.z * ir;
                    float f[NB], df[NB];
                    cheb_basis<NB>(r, a.rcA, f, df);
                    const float *cp = cA + (tI * T + tj) * NA * NB;
                    float gn[NA], dgn[NA];
#pragma unroll
                    for (int q = 0; q < NA; ++q) {
                        float s0 = 0.f, s1 = 0.f;
#pragma unroll
                        for (int k = 0; k < NB; ++k) {
                            s0 = fmaf(cp[q * NB + k], f[k], s0);
                            s1 = fmaf(cp[q * NB + k], df[k], s1);
                        }
                        gn[q] = s0;
                        dgn[q] = s1;
                    }
                    float Y[LM];
                    harmonics(ux, uy, uz, Y);
                    float radial = 0.f;
                    float Qv[LM];
#pragma unroll
                    for (int m = 0; m < LM; ++m) Qv[m] = 0.f;
#pragma unroll
                    for (int q = 0; q < NA; ++q) {
                        float Pn = 0.f;
#pragma unroll
                        for (int m = 0; m < LM; ++m) {
                            Pn = fmaf(At[q][m], Y[m], Pn);
                            Qv[m] = fmaf(At[q][m], gn[q], Qv[m]);
                        }
                        radial = fmaf(dgn[q], Pn, radial);
                    }
                    float gx, gy, gz;
                    harmonics_grad_dot(ux, uy, uz, Qv, gx, gy, gz);
                    const float ug = ux * gx + uy * gy + uz * gz;
                    const float Fx = radial * ux + (gx - ug * ux) * ir;
                    const float Fy = radial * uy + (gy - ug * uy) * ir;
                    const float Fz = radial * uz + (gz - ug * uz) * ir;
                    ox += Fx;
                    oy += Fy;
                    oz += Fz;
                    atomicAdd(&fx[j], -Fx);
                    atomicAdd(&fy[j], -Fy);
                    atomicAdd(&fz[j], -Fz);
                    m9[0] -= Fx * e.x; m9[1] -= Fx * e.y; m9[2] -= Fx * e.z;
                    m9[3] -= Fy * e.x; m9[4] -= Fy * e.y; m9[5] -= Fy * e.z;
                    m9[6] -= Fz * e.x; m9[7] -= Fz * e.y; m9[8] -= Fz * e.z;
                }
            }
            ox = group_sum(ox, G);
            oy = group_sum(oy, G);
            oz = group_sum(oz, G);
            if (act && lig == 0) {
                atomicAdd(&fx[i], ox);
                atomicAdd(&fy[i], oy);
                atomicAdd(&fz[i], oz);
            }
        }
        __syncthreads();

        // ---- outputs and losses
        double accF = 0.0;
        for (int i = tid; i < n; i += BATCH_THREADS) {
            const int64_t g = b.atom0 + i;
            const float Fx = fx[i], Fy = fy[i], Fz = fz[i];
            const double ex = (double)Fx - a.F_ref[g], ey = (double)Fy - a.F_ref[a.n_total + g],
                         ez = (double)Fz - a.F_ref[2 * a.n_total + g];
            accF += ex * ex + ey * ey + ez * ez;
            if (a.forces) {
                float *F = a.forces + (size_t)c * 3 * a.n_total;
                F[g] = Fx;
                F[a.n_total + g] = Fy;
                F[2 * a.n_total + g] = Fz;
            }
            if (a.charges) a.charges[(size_t)c * a.n_total + g] = sc * qv[i];
        }
        double r3[10] = {accF, m9[0], m9[1], m9[2], m9[3], m9[4], m9[5], m9[6], m9[7], m9[8]};
        block_sum<10>(r3, red);
        if (tid == 0) {
            const size_t sc_idx = (size_t)s * a.C + c;
            const double E = sumU + Ues;
            const double sq = (double)sc * sumq;
            a.losses[3 * sc_idx + 0] = (float)(fabs(E - a.E_ref[s]) / n);
            a.losses[3 * sc_idx + 1] = (float)sqrt(r3[0] / (3.0 * n));
            a.losses[3 * sc_idx + 2] = (float)fabs(sq - a.qtot);
            if (a.energy) a.energy[sc_idx] = E;
            if (a.virial) {
                double *W = a.virial + 9 * sc_idx;
                for (int k = 0; k < 9; ++k) W[k] = r3[1 + k];
                if (a.ncomp == BATCH_COMP_VIRIAL) {
                    W[0] += r2[2]; W[4] += r2[3]; W[8] += r2[4];
                    W[1] += r2[5]; W[3] += r2[5];
                    W[2] += r2[6]; W[6] += r2[6];
                    W[5] += r2[7]; W[7] += r2[7];
                }
            }
            double *st4 = a.stats + 4 * sc_idx;
            st4[0] = E;
            st4[1] = r3[0];
            st4[2] = sq;
            st4[3] = (double)n;
        }
        __syncthreads();
    }
}

// Loss per candidate (Sec. 2.5): lambda_e RMSE(E/N) + lambda_f RMSE(F) + lambda_Q RMSE(Q)
// + lambda_1 |theta|_1 + lambda_2 |theta|_2^2, sums over structures in a fixed order.
__global__ __launch_bounds__(256) void k_b_loss(const double *__restrict__ stats, const double *__restrict__ E_ref,
                                                const float *__restrict__ thetas, int64_t n_theta, int S, int C,
                                                double qtot, double le, double lf, double lq, double l1, double l2,
                                                double *__restrict__ loss) {
    __shared__ double red[4 * 16];
    const int c = blockIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int s = threadIdx.x; s < S; s += blockDim.x) {
        const double *st4 = stats + 4 * ((size_t)s * C + c);
        const double de = (st4[0] - E_ref[s]) / st4[3];
        const double dq = st4[2] - qtot;
        v[0] += de * de;
        v[1] += st4[1];
        v[2] += 3.0 * st4[3];
        v[3] += dq * dq;
    }
    const float *th = thetas + (size_t)c * n_theta;
    for (int64_t k = threadIdx.x; k < n_theta; k += blockDim.x) {
        const double x = th[k];
        v[4] += fabs(x);
        v[5] += x * x;
    }
    block_sum<6>(v, red);
    if (threadIdx.x == 0)
        loss[c] = le * sqrt(v[0] / S) + lf * sqrt(v[1] / v[2]) + lq * sqrt(v[3] / S) + l1 * v[4] + l2 * v[5];
}

// ---------------------------------------------------------------- launchers
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

#define QNEP_BATCH_DISPATCH(T_, NR_, NA_, NB_)                                                              \
    if (T == T_ && NR == NR_ && NA == NA_ && NB == NB_) {                                                   \
        if (lds_bytes > 65536) {                                                                            \
            hipError_t e0 = hipFuncSetAttribute((const void *)k_batch_eval<T_, NR_, NA_, NB_>,             \
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes); \
            if (e0 != hipSuccess) return e0;                                                                \
        }                                                                                                   \
        hipLaunchKernelGGL((k_batch_eval<T_, NR_, NA_, NB_>), dim3(n_slots), dim3(BATCH_THREADS), lds_bytes, \
                           stream, a, item_begin, item_end, groups);                                        \
        return hipGetLastError();                                                                           \
    }

bool batch_supported(int T, int NR, int NA, int NB) {
    return T >= 1 && T <= 4 && NB == 9 && ((NR == 5 && NA == 5) || (NR == 9 && NA == 7));
}

hipError_t batch_eval(const BatchArgs &a, int T, int NR, int NA, int NB, int n_slots, int item_begin,
                      int item_end, int4 groups, hipStream_t stream) {
    const size_t lds_bytes = sizeof(float) * ((size_t)a.n_theta + 5 * (size_t)a.max_atoms);
    QNEP_BATCH_DISPATCH(1, 5, 5, 9)
    QNEP_BATCH_DISPATCH(2, 5, 5, 9)
    QNEP_BATCH_DISPATCH(3, 5, 5, 9)
    QNEP_BATCH_DISPATCH(4, 5, 5, 9)
    QNEP_BATCH_DISPATCH(1, 9, 7, 9)
    QNEP_BATCH_DISPATCH(2, 9, 7, 9)
    QNEP_BATCH_DISPATCH(3, 9, 7, 9)
    QNEP_BATCH_DISPATCH(4, 9, 7, 9)
    return hipErrorInvalidValue;
}

hipError_t batch_loss(const double *stats, const double *E_ref, const float *thetas, int64_t n_theta, int S, int C,
                      double qtot, const double *lam, double *loss, hipStream_t stream) {
    hipLaunchKernelGGL(k_b_loss, dim3(C), dim3(256), 0, stream, stats, E_ref, thetas, n_theta, S, C, qtot, lam[0],
                       lam[1], lam[2], lam[3], lam[4], loss);
    return hipGetLastError();
}

}  // namespace qnep
