// NEP descriptors, partial forces and the assembly of F, W and Z*.
//
//  * descriptors (Sec. 2.1; published NEP3/NEP4 form): radial q_n = sum_j g_n(r_ij),
//    computed through per-species basis sums B_{t,k} = sum_{j in t} f_k(r_ij) so that
//    the species-pair coefficients are applied once per atom; angular moments
//    A_nlm = sum_j g_n(r_ij) Y_lm(r_ij) and q_nl = sum_m A_nlm^2 (the Legendre double
//    sum by the addition theorem).
//  * partial forces F_ij = g_i . dD^i/dr_ij with g_i = dU_i/dD + chi_i dq_i/dD
//    (Sec. 2.3, Eqs. 14, 16, 17, 19, 23), chi_i = phi_i - mean(phi) carrying the chain
//    rule through the neutrality correction; charge derivatives a_ij = s dq_i/dD .
//    dD^i/dr_ij for the Born charges (Sec. 2.4, Eq. 28).
//  * F_i = sum_j (F_ij - F_ji) (Eq. 11), W = -sum F_ij (x) r_ij, and
//    Z_i = q~'_i I + 1/2 sum_j (r_ij (x) a_ij - r_ji (x) a_ji) (Eq. 28).
// Radial reverse terms are gathered from per-atom coefficient tables; angular
// reverse terms through a pair buffer and a search of the neighbour's list.
#include "nep_math.h"
#include "plan.h"

namespace qnep {

// padded row length of the per-atom radial coefficient tables (16-byte multiples)
template <int NB>
struct Pad4 {
    static constexpr int v = (NB + 3) / 4 * 4;
};

// ---------------------------------------------------------------- descriptors
template <int T, int NR, int NA, int NB>
__global__ __launch_bounds__(256) void k_descriptors(int N, const float4 *__restrict__ xyzt, Cell c, float rcR,
                                                     float rcA, const uint32_t *__restrict__ listR,
                                                     const int *__restrict__ cntR, int capR,
                                                     const uint32_t *__restrict__ listA,
                                                     const int *__restrict__ cntA, int capA,
                                                     const float *__restrict__ theta, int64_t off_cR,
                                                     int64_t off_cA, float *__restrict__ D,
                                                     float *__restrict__ Amom, float *__restrict__ Bsum) {
    __shared__ float cR[T * T * NR * NB];
    __shared__ float cA[T * T * NA * NB];
    for (int k = threadIdx.x; k < T * T * NR * NB; k += blockDim.x) cR[k] = theta[off_cR + k];
    for (int k = threadIdx.x; k < T * T * NA * NB; k += blockDim.x) cA[k] = theta[off_cA + k];
    __syncthreads();
    const int i = xcd_block() * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float4 pi = xyzt[i];
    const int ti = species_of(pi);
    // ---- radial
    float B[T][NB];
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int k = 0; k < NB; ++k) B[t][k] = 0.0f;
    const int nR = cntR[i];
    // software pipeline: list entries two pairs ahead, neighbour positions one ahead
    const uint32_t *lr = listR + (size_t)i * capR;
    uint32_t e_a = nR > 0 ? lr[0] : 0u, e_b = nR > 1 ? lr[1] : 0u;
    float4 p_a = nR > 0 ? xyzt[nb_index(e_a)] : pi;
    for (int s = 0; s < nR; ++s) {
        const uint32_t e = e_a;
        const float4 pj = p_a;
        e_a = e_b;
        if (s + 1 < nR) p_a = xyzt[nb_index(e_b)];
        if (s + 2 < nR) e_b = lr[s + 2];
        const float3 d = pair_displacement(pi, pj, e, c);
        const float r = sqrtf(d.x * d.x + d.y * d.y + d.z * d.z);
        float f[NB], df[NB];
        cheb_basis<NB>(r, rcR, f, df);
        const int tj = species_of(pj);
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const float m = (tj == t) ? 1.0f : 0.0f;
#pragma unroll
            for (int k = 0; k < NB; ++k) B[t][k] = fmaf(m, f[k], B[t][k]);
        }
    }
#pragma unroll
    for (int n = 0; n < NR; ++n) {
        float acc = 0.0f;
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int k = 0; k < NB; ++k) acc = fmaf(cR[((ti * T + t) * NR + n) * NB + k], B[t][k], acc);
        D[(size_t)n * N + i] = acc;
    }
    if (Bsum) {  // per-species radial basis sums B_{t,k} (used by the parameter gradient)
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int k = 0; k < NB; ++k) Bsum[(size_t)(t * NB + k) * N + i] = B[t][k];
    }
    // ---- angular
    float A[NA][LM];
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int q = 0; q < LM; ++q) A[n][q] = 0.0f;
    const int nA = cntA[i];
    const uint32_t *la = listA + (size_t)i * capA;
    uint32_t a_a = nA > 0 ? la[0] : 0u, a_b = nA > 1 ? la[1] : 0u;
    float4 q_a = nA > 0 ? xyzt[nb_index(a_a)] : pi;
    for (int s = 0; s < nA; ++s) {
        const uint32_t e = a_a;
        const float4 pj = q_a;
        a_a = a_b;
        if (s + 1 < nA) q_a = xyzt[nb_index(a_b)];
        if (s + 2 < nA) a_b = la[s + 2];
        const float3 d = pair_displacement(pi, pj, e, c);
        const float r = sqrtf(d.x * d.x + d.y * d.y + d.z * d.z);
        float f[NB], df[NB];
        cheb_basis<NB>(r, rcA, f, df);
        const float *cp = &cA[(ti * T + species_of(pj)) * NA * NB];
        float g[NA];
#pragma unroll
        for (int n = 0; n < NA; ++n) {
            float acc = 0.0f;
#pragma unroll
            for (int k = 0; k < NB; ++k) acc = fmaf(cp[n * NB + k], f[k], acc);
            g[n] = acc;
        }
        const float ir = 1.0f / r;
        float Y[LM];
        harmonics(d.x * ir, d.y * ir, d.z * ir, Y);
#pragma unroll
        for (int n = 0; n < NA; ++n)
#pragma unroll
            for (int q = 0; q < LM; ++q) A[n][q] = fmaf(g[n], Y[q], A[n][q]);
    }
#pragma unroll
    for (int n = 0; n < NA; ++n) {
#pragma unroll
        for (int q = 0; q < LM; ++q) Amom[(size_t)(n * LM + q) * N + i] = A[n][q];
        float s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
#pragma unroll
        for (int q = 0; q < 3; ++q) s1 = fmaf(A[n][q], A[n][q], s1);
#pragma unroll
        for (int q = 3; q < 8; ++q) s2 = fmaf(A[n][q], A[n][q], s2);
#pragma unroll
        for (int q = 8; q < 15; ++q) s3 = fmaf(A[n][q], A[n][q], s3);
#pragma unroll
        for (int q = 15; q < 24; ++q) s4 = fmaf(A[n][q], A[n][q], s4);
        D[(size_t)(NR + 0 * NA + n) * N + i] = s1;
        D[(size_t)(NR + 1 * NA + n) * N + i] = s2;
        D[(size_t)(NR + 2 * NA + n) * N + i] = s3;
        D[(size_t)(NR + 3 * NA + n) * N + i] = s4;
    }
}

// ---------------------------------------------------------------- gradient tables
// Per atom: chi_i = phi_i - mean(phi); radial coefficient tables
//   hE[t][k] = sum_n (gU_n + chi gq_n) cR[ti][t][n][k],  hq[t][k] = s sum_n gq_n cR[ti][t][n][k]
// stored atom-major, one record of REC floats per (atom, species t) holding the two
// rows interleaved, (hE[t][0], hq[t][0], hE[t][1], hq[t][1], ...), padded to 16 bytes:
// a neighbour's rows for one species are REC / 4 aligned vector loads.
template <int NB>
struct RadRec {
    static constexpr int v = (2 * NB + 3) / 4 * 4;  // floats per record
};

template <int T, int NR, int NB>
__global__ __launch_bounds__(256) void k_radial_tables(int N, const int *__restrict__ ts,
                                                       const float *__restrict__ gU, const float *__restrict__ gq,
                                                       const float *__restrict__ phi,
                                                       const double *__restrict__ scalars,
                                                       const float *__restrict__ theta, int64_t off_cR,
                                                       int64_t off_s, float *__restrict__ hT) {
    constexpr int REC = RadRec<NB>::v;
    __shared__ float cR[T * T * NR * NB];
    for (int k = threadIdx.x; k < T * T * NR * NB; k += blockDim.x) cR[k] = theta[off_cR + k];
    __syncthreads();
    const int i = xcd_block() * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float s = theta[off_s];
    const float chi = (float)((double)phi[i] - scalars[S_PHIBAR]);
    const int ti = ts[i];
    float GE[NR], GQ[NR];
#pragma unroll
    for (int n = 0; n < NR; ++n) {
        float a = gU[(size_t)n * N + i], b = gq[(size_t)n * N + i];
        GE[n] = fmaf(chi, b, a);
        GQ[n] = s * b;
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
        float v[REC];
#pragma unroll
        for (int k = 0; k < REC / 2; ++k) {
            float e = 0.f, q = 0.f;
            if (k < NB) {
#pragma unroll
                for (int n = 0; n < NR; ++n) {
                    float cv = cR[((ti * T + t) * NR + n) * NB + k];
                    e = fmaf(GE[n], cv, e);
                    q = fmaf(GQ[n], cv, q);
                }
            }
            v[2 * k] = e;
            v[2 * k + 1] = q;
        }
        float4 *out = reinterpret_cast<float4 *>(hT + ((size_t)i * T + t) * REC);
#pragma unroll
        for (int k4 = 0; k4 < REC / 4; ++k4)
            out[k4] = make_float4(v[4 * k4], v[4 * k4 + 1], v[4 * k4 + 2], v[4 * k4 + 3]);
    }
}

// ---------------------------------------------------------------- radial forces
// F_ij = sigma_ij u, sigma_ij = sum_k hE_i[tj][k] f_k'(r); a_ij = rho_ij u likewise.
// F_i = sum_j (sigma_ij + sigma_ji) u_ij, Z_i += 1/2 sum_j (rho_ij - rho_ji) r u (x) u,
// W -= sum_j sigma_ij r u (x) u (own partial forces only).
// RF_LANES lanes share one atom and split its neighbours; the sums are combined
// across the lane group with butterfly shuffles.
constexpr int RF_LANES = 8;
static_assert(RF_LANES <= PARTIALS_LANES_MAX, "partials buffer sized for PARTIALS_LANES_MAX lanes per atom");

// With VAT the per-atom virial W_i += r_ij (x) F_ji = -sigma_ji r u (x) u (Eq. 12) is
// added to Vat as well.  ISO (isolated systems, Born charges of Eq. 27): the pair part
// of Z_i is sum_j r_ij (x) a_ji = -rho_ji r u (x) u, and S_i = sum_j (a_ji - a_ij) =
// -(rho_ij + rho_ji) u goes to Siso for the centroid term of the assembly.
template <int T, int NB, bool VAT, bool ISO>
__global__ __launch_bounds__(256) void k_radial_forces(int N, const float4 *__restrict__ xyzt, Cell c, float rcR,
                                                       const uint32_t *__restrict__ listR,
                                                       const int *__restrict__ cntR, int capR,
                                                       const float *__restrict__ hT, float *__restrict__ Fnep,
                                                       float *__restrict__ Znep, float *__restrict__ Vat,
                                                       float *__restrict__ Siso, double *__restrict__ partials) {
    constexpr int REC = RadRec<NB>::v, R4 = REC / 4, APB = 256 / RF_LANES;
    // this atom's own T records, read for every pair, sit in LDS: the vector memory
    // path is left to the neighbours' records
    __shared__ float4 own[APB][T * R4];
    const int gtid = xcd_block() * blockDim.x + threadIdx.x;
    const int i = gtid / RF_LANES, sub = gtid % RF_LANES, a = threadIdx.x / RF_LANES;
    for (int q = sub; q < T * R4; q += RF_LANES)
        own[a][q] = i < N ? reinterpret_cast<const float4 *>(hT + (size_t)i * T * REC)[q]
                          : make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    constexpr int NACC = 15 + (VAT ? 6 : 0) + (ISO ? 3 : 0), KS = 15 + (VAT ? 6 : 0);
    float acc[NACC];  // F (3), Z (xx yy zz xy xz yz), W (same order)[, per-atom W (same order)][, S (3)]
#pragma unroll
    for (int k = 0; k < NACC; ++k) acc[k] = 0.f;
    if (i < N) {
        const float4 pi = xyzt[i];
        const int ti = species_of(pi);
        const int nR = cntR[i];
        // software pipeline: list entries two passes ahead; the neighbour's position and
        // its record for this atom's species one pass ahead
        const uint32_t *lr = listR + (size_t)i * capR;
        uint32_t e_a = sub < nR ? lr[sub] : 0u, e_b = sub + RF_LANES < nR ? lr[sub + RF_LANES] : 0u;
        float4 pj_n = pi, xr_n[R4];
        auto fetch = [&](uint32_t en) {
            const float4 *nrec = reinterpret_cast<const float4 *>(hT + ((size_t)nb_index(en) * T + ti) * REC);
#pragma unroll
            for (int k4 = 0; k4 < R4; ++k4) xr_n[k4] = nrec[k4];
            pj_n = xyzt[nb_index(en)];
        };
        if (sub < nR) fetch(e_a);
        for (int s = sub; s < nR; s += RF_LANES) {
            const uint32_t e = e_a;
            const float4 pj = pj_n;
            float4 xr[R4];
#pragma unroll
            for (int k4 = 0; k4 < R4; ++k4) xr[k4] = xr_n[k4];
            e_a = e_b;
            if (s + RF_LANES < nR) fetch(e_a);
            if (s + 2 * RF_LANES < nR) e_b = lr[s + 2 * RF_LANES];
            // this atom's record for the neighbour's species
            const int tj = species_of(pj);
            float4 ar[R4];
#pragma unroll
            for (int k4 = 0; k4 < R4; ++k4) ar[k4] = own[a][tj * R4 + k4];
            const float3 d = pair_displacement(pi, pj, e, c);
            const float r = sqrtf(d.x * d.x + d.y * d.y + d.z * d.z);
            float f[NB], df[NB];
            cheb_basis<NB>(r, rcR, f, df);
            float sij = 0.f, rij = 0.f, sji = 0.f, rji = 0.f;
#pragma unroll
            for (int k4 = 0; k4 < R4; ++k4) {
                const float4 a = ar[k4], x = xr[k4];
                // (hE_k, hq_k, hE_k+1, hq_k+1)
                const int k = 2 * k4;
                if (k < NB) {
                    sij = fmaf(a.x, df[k], sij);
                    rij = fmaf(a.y, df[k], rij);
                    sji = fmaf(x.x, df[k], sji);
                    rji = fmaf(x.y, df[k], rji);
                }
                if (k + 1 < NB) {
                    sij = fmaf(a.z, df[k + 1], sij);
                    rij = fmaf(a.w, df[k + 1], rij);
                    sji = fmaf(x.z, df[k + 1], sji);
                    rji = fmaf(x.w, df[k + 1], rji);
                }
            }
            const float ir = 1.0f / r;
            const float ux = d.x * ir, uy = d.y * ir, uz = d.z * ir;
            const float sf = sij + sji;
            acc[0] = fmaf(sf, ux, acc[0]);
            acc[1] = fmaf(sf, uy, acc[1]);
            acc[2] = fmaf(sf, uz, acc[2]);
            const float zr = ISO ? -rji * r : 0.5f * (rij - rji) * r, wr = -sij * r;
            if constexpr (ISO) {
                const float sr = -(rij + rji);
                acc[KS] = fmaf(sr, ux, acc[KS]);
                acc[KS + 1] = fmaf(sr, uy, acc[KS + 1]);
                acc[KS + 2] = fmaf(sr, uz, acc[KS + 2]);
            }
            const float uu[6] = {ux * ux, uy * uy, uz * uz, ux * uy, ux * uz, uy * uz};
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                acc[3 + k] = fmaf(zr, uu[k], acc[3 + k]);
                acc[9 + k] = fmaf(wr, uu[k], acc[9 + k]);
            }
            if constexpr (VAT) {
                const float wa = -sji * r;
#pragma unroll
                for (int k = 0; k < 6; ++k) acc[15 + k] = fmaf(wa, uu[k], acc[15 + k]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NACC; ++k)
#pragma unroll
        for (int o = RF_LANES / 2; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o, 64);
    double w[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (i < N && sub == 0) {
        Fnep[i] = acc[0];
        Fnep[(size_t)N + i] = acc[1];
        Fnep[(size_t)2 * N + i] = acc[2];
        const float zxx = acc[3], zyy = acc[4], zzz = acc[5], zxy = acc[6], zxz = acc[7], zyz = acc[8];
        Znep[(size_t)0 * N + i] = zxx;
        Znep[(size_t)1 * N + i] = zxy;
        Znep[(size_t)2 * N + i] = zxz;
        Znep[(size_t)3 * N + i] = zxy;
        Znep[(size_t)4 * N + i] = zyy;
        Znep[(size_t)5 * N + i] = zyz;
        Znep[(size_t)6 * N + i] = zxz;
        Znep[(size_t)7 * N + i] = zyz;
        Znep[(size_t)8 * N + i] = zzz;
        w[0] = acc[9]; w[4] = acc[10]; w[8] = acc[11];
        w[1] = w[3] = acc[12];
        w[2] = w[6] = acc[13];
        w[5] = w[7] = acc[14];
        if constexpr (VAT) {
#pragma unroll
            for (int k = 0; k < 6; ++k) Vat[(size_t)k * N + i] += acc[15 + k];
        }
        if constexpr (ISO) {
#pragma unroll
            for (int k = 0; k < 3; ++k) Siso[(size_t)k * N + i] = acc[KS + k];
        }
    }
    block_partials<9>(w, partials);
}

// ---------------------------------------------------------------- angular forces
// Atilde_nlm = 2 G_nl A_nlm with G the upstream gradient, for two gradients at once:
// energy G = dU/dD + chi dq/dD and charge G = s dq/dD.  Per pair and gradient:
// P_n = sum_lm Atilde_nlm Y_lm, Q_lm = sum_n Atilde_nlm g_n,
// F_ij = u sum_n g_n' P_n + (I - u u^T) (sum_lm Q_lm grad Y_lm) / r.
// AF_LANES lanes share one atom and split its angular neighbours; the two Atilde
// tables of the atom are built once in LDS (the lanes split their entries) and read
// by every lane, so the pair geometry (basis, radial functions, harmonics) is
// evaluated once for both gradients.  Writes the pair buffer (F_ij of the energy and
// a_ij of the charge gradient side by side, one 32-byte slot per pair), adds the own
// force and Z contributions, and the virial partials.
constexpr int AF_LANES = 8;
constexpr int AF_APB = 256 / AF_LANES;  // atoms per work-group
static_assert(AF_LANES <= PARTIALS_LANES_MAX, "partials buffer sized for PARTIALS_LANES_MAX lanes per atom");

// one gradient's pair force from its Atilde table (rows of LM = 24 floats, 16-byte aligned)
template <int NA>
__device__ __forceinline__ float3 angular_pair(const float4 *__restrict__ At4, const float (&g)[8],
                                               const float (&dg)[8], const float (&Y)[LM],
                                               const HarmonicsGrad &hg, float ux, float uy, float uz, float ir) {
    float radial = 0.f;
    float Qv[LM];
#pragma unroll
    for (int q = 0; q < LM; ++q) Qv[q] = 0.f;
#pragma unroll
    for (int n = 0; n < NA; ++n) {
        float Pn = 0.f;
#pragma unroll
        for (int q4 = 0; q4 < LM / 4; ++q4) {
            const float4 a4 = At4[n * (LM / 4) + q4];
            const float a[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                Pn = fmaf(a[e], Y[4 * q4 + e], Pn);
                Qv[4 * q4 + e] = fmaf(a[e], g[n], Qv[4 * q4 + e]);
            }
        }
        radial = fmaf(dg[n], Pn, radial);
    }
    float gx, gy, gz;
    harmonics_grad_apply(hg, Qv, gx, gy, gz);
    const float ug = ux * gx + uy * gy + uz * gz;
    return make_float3(radial * ux + (gx - ug * ux) * ir, radial * uy + (gy - ug * uy) * ir,
                       radial * uz + (gz - ug * uz) * ir);
}

// ISO (isolated systems): the own a_ij enter Z only through S_i -= a_ij (Siso).
template <int T, int NR, int NA, int NB, bool ISO>
__global__ __launch_bounds__(256) void k_angular_forces(
    int N, const float4 *__restrict__ xyzt, Cell c, float rcA, const uint32_t *__restrict__ listA,
    const int *__restrict__ cntA, int capA, const float *__restrict__ Amom, const float *__restrict__ gU,
    const float *__restrict__ gq, const float *__restrict__ phi, const double *__restrict__ scalars,
    const float *__restrict__ theta, int64_t off_cA, int64_t off_s, float4 *__restrict__ pairFA,
    float *__restrict__ Fnep, float *__restrict__ Znep, float *__restrict__ Siso, double *__restrict__ partials) {
    constexpr int NAL = NA * LM;
    static_assert(NA <= 8 && LM % 4 == 0, "angular table layout");
    // cA8[ti tj][k][n], n padded to 8: the two float4 of one k serve all g_n
    __shared__ __align__(16) float cA8[T * T * NB * 8];
    __shared__ __align__(16) float AtE[AF_APB][NAL];
    __shared__ __align__(16) float AtQ[AF_APB][NAL];
    for (int k = threadIdx.x; k < T * T * NB * 8; k += blockDim.x) {
        const int tp = k / (NB * 8), kb = (k / 8) % NB, n = k % 8;
        cA8[k] = n < NA ? theta[off_cA + (int64_t)(tp * NA + n) * NB + kb] : 0.0f;
    }
    const int a = threadIdx.x / AF_LANES, sub = threadIdx.x % AF_LANES;
    const int i = xcd_block() * AF_APB + a;
    const bool live = i < N;
    if (live) {
        const float s = theta[off_s];
        const float chi = (float)((double)phi[i] - scalars[S_PHIBAR]);
        for (int k = sub; k < NAL; k += AF_LANES) {
            const int n = k / LM, q = k - n * LM;
            const int l = q < 3 ? 0 : (q < 8 ? 1 : (q < 15 ? 2 : 3));
            const size_t row = (size_t)(NR + l * NA + n) * N + i;
            const float b = gq[row], am = Amom[(size_t)k * N + i];
            AtE[a][k] = 2.0f * fmaf(chi, b, gU[row]) * am;
            AtQ[a][k] = 2.0f * s * b * am;
        }
    }
    __syncthreads();
    constexpr int NACC = ISO ? 24 : 21;
    float acc[NACC];  // own force (3), virial W_ab -= F_a r_b (9), Z_ab += 1/2 r_a a_b (9) [ISO: S -= a (3)]
#pragma unroll
    for (int k = 0; k < NACC; ++k) acc[k] = 0.f;
    if (live) {
        const float4 pi = xyzt[i];
        const int ti = species_of(pi);
        const int nA = cntA[i];
        const uint32_t *lrow = listA + (size_t)i * capA;
        // list entries two passes ahead, neighbour positions one pass ahead
        uint32_t e_a = sub < nA ? lrow[sub] : 0u, e_b = sub + AF_LANES < nA ? lrow[sub + AF_LANES] : 0u;
        float4 pj_n = sub < nA ? xyzt[nb_index(e_a)] : pi;
        for (int sl = sub; sl < nA; sl += AF_LANES) {
            const uint32_t e = e_a;
            const float4 pj = pj_n;
            e_a = e_b;
            if (sl + AF_LANES < nA) pj_n = xyzt[nb_index(e_a)];
            if (sl + 2 * AF_LANES < nA) e_b = lrow[sl + 2 * AF_LANES];
            const float3 d = pair_displacement(pi, pj, e, c);
            const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
            const float ir = __builtin_amdgcn_rsqf(r2);  // v_rsq_f32, 1 ulp
            const float r = r2 * ir;
            const float ux = d.x * ir, uy = d.y * ir, uz = d.z * ir;
            float f[NB], df[NB];
            cheb_basis<NB>(r, rcA, f, df);
            const float4 *cp = reinterpret_cast<const float4 *>(&cA8[(ti * T + species_of(pj)) * NB * 8]);
            float g[8], dg[8];
#pragma unroll
            for (int n = 0; n < 8; ++n) g[n] = dg[n] = 0.f;
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const float4 c0 = cp[2 * k], c1 = cp[2 * k + 1];
                const float cv[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
                for (int n = 0; n < NA; ++n) {
                    g[n] = fmaf(cv[n], f[k], g[n]);
                    dg[n] = fmaf(cv[n], df[k], dg[n]);
                }
            }
            float Y[LM];
            harmonics(ux, uy, uz, Y);
            // an offset the compiler cannot prove loop-invariant, so that the tables are
            // read from LDS per pair instead of being hoisted into registers
            int row = a * (NAL / 4);
            asm volatile("" : "+v"(row));
            const HarmonicsGrad hg = harmonics_grad(ux, uy, uz);
            const float3 F =
                angular_pair<NA>(reinterpret_cast<const float4 *>(&AtE[0][0]) + row, g, dg, Y, hg, ux, uy, uz, ir);
            const float3 A =
                angular_pair<NA>(reinterpret_cast<const float4 *>(&AtQ[0][0]) + row, g, dg, Y, hg, ux, uy, uz, ir);
            pairFA[((size_t)i * capA + sl) * 2] = make_float4(F.x, F.y, F.z, 0.f);
            pairFA[((size_t)i * capA + sl) * 2 + 1] = make_float4(A.x, A.y, A.z, 0.f);
            const float fv[3] = {F.x, F.y, F.z}, av[3] = {A.x, A.y, A.z}, dv[3] = {d.x, d.y, d.z};
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                acc[x] += fv[x];
#pragma unroll
                for (int y = 0; y < 3; ++y) {
                    acc[3 + 3 * x + y] = fmaf(-fv[x], dv[y], acc[3 + 3 * x + y]);
                    if constexpr (!ISO) acc[12 + 3 * x + y] = fmaf(0.5f * dv[x], av[y], acc[12 + 3 * x + y]);
                }
                if constexpr (ISO) acc[21 + x] -= av[x];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NACC; ++k)
#pragma unroll
        for (int o = AF_LANES / 2; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o, 64);
    double w[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (live && sub == 0) {
        Fnep[i] += acc[0];
        Fnep[(size_t)N + i] += acc[1];
        Fnep[(size_t)2 * N + i] += acc[2];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            w[k] = acc[3 + k];
            Znep[(size_t)k * N + i] += acc[12 + k];
        }
        if constexpr (ISO) {
#pragma unroll
            for (int k = 0; k < 3; ++k) Siso[(size_t)k * N + i] += acc[21 + k];
        }
    }
    block_partials<9>(w, partials);
}

// The slot of `want` in atom j's angular list (-1 if absent); rows are 16-byte aligned.
// The first FS_AHEAD 16-byte groups of the row are loaded together with its length (one
// round trip covers lists of up to 4 FS_AHEAD entries; longer rows continue in order),
// in a separate step, so that the row of the next pair can be loaded while the current
// pair's slot is read.
constexpr int FS_AHEAD = 6;

struct RowProbe {
    uint4 v[FS_AHEAD];
    int nj;
};

__device__ inline void probe_load(const uint32_t *__restrict__ listA, const int *__restrict__ cntA, int j, int capA,
                                  RowProbe &rp) {
    const uint4 *row = reinterpret_cast<const uint4 *>(listA + (size_t)j * capA);
    const int ng = capA / 4 < FS_AHEAD ? capA / 4 : FS_AHEAD;
#pragma unroll
    for (int t = 0; t < FS_AHEAD; ++t) rp.v[t] = t < ng ? row[t] : make_uint4(0u, 0u, 0u, 0u);
    rp.nj = cntA[j];
}

__device__ inline int probe_match(const uint32_t *__restrict__ listA, int j, int capA, const RowProbe &rp,
                                  uint32_t want) {
    const int ng = capA / 4 < FS_AHEAD ? capA / 4 : FS_AHEAD, nj = rp.nj;
#pragma unroll
    for (int t = 0; t < FS_AHEAD; ++t) {
        const int b = 4 * t;
        if (t < ng) {
            if (rp.v[t].x == want && b < nj) return b;
            if (rp.v[t].y == want && b + 1 < nj) return b + 1;
            if (rp.v[t].z == want && b + 2 < nj) return b + 2;
            if (rp.v[t].w == want && b + 3 < nj) return b + 3;
        }
    }
    const uint4 *row = reinterpret_cast<const uint4 *>(listA + (size_t)j * capA);
    for (int t4 = ng; 4 * t4 < nj; ++t4) {
        const uint4 u = row[t4];
        const int b = 4 * t4;
        if (u.x == want) return b;
        if (u.y == want && b + 1 < nj) return b + 1;
        if (u.z == want && b + 2 < nj) return b + 2;
        if (u.w == want && b + 3 < nj) return b + 3;
    }
    return -1;
}

// ---------------------------------------------------------------- assembly
// Adds the angular reverse terms -F_ji and -1/2 r_ji (x) a_ji found in each
// neighbour's pair buffer, the static electrostatic forces and the diagonal q~'_i,
// writes F, Z*, q', q~' in input order and FP64 partials of P = sum_i q~'_i r_i.
// AS_LANES lanes share one atom and split its angular neighbours.
constexpr int AS_LANES = 8;
static_assert(AS_LANES <= PARTIALS_LANES_MAX, "partials buffer sized for PARTIALS_LANES_MAX lanes per atom");

// With an external field E the force gains sum_a E_a Z_i[a][:] (Eq. 29).  With VAT the
// per-atom virial is completed (angular reverse terms r_ij (x) F_ji, Eq. 12, and the
// background U_bg I / N) from the symmetric parts gathered in Vat and written out.
struct AssembleExtra {
    float ex, ey, ez;   // external field
    float ubg_coef;     // -k_e pi Q^2 / (2 Omega alpha^2 N) (mode 1), times 1/s^2 on the device
    const float *Vat;   // symmetric per-atom virial parts [6][N]
    float *vatom;       // output [9][N], input order
    const float *Siso;  // isolated systems: sum_j (a_ji - a_ij) from the radial and angular kernels
};

// ISO (isolated systems, Eq. 27 with the corrected charges): Z_i = q~'_i I +
// sum_j r_ij (x) a_ji + (r_i - rbar) (x) sum_j (a_ji - a_ij), r_i the caller's position and
// rbar the centroid.
template <bool VAT, bool ISO>
__global__ __launch_bounds__(256) void k_assemble(
    int N, const float4 *__restrict__ xyzt, Cell c, const uint32_t *__restrict__ listA,
    const int *__restrict__ cntA, int capA, const float4 *__restrict__ pairFA,
    const float *__restrict__ Fnep, const float *__restrict__ Znep, const float *__restrict__ Fst,
    const float *__restrict__ qraw, const double *__restrict__ scalars, const float *__restrict__ theta,
    int64_t off_s, const int *__restrict__ perm, const float *__restrict__ pos, float *__restrict__ forces,
    float *__restrict__ bec, float *__restrict__ charges, float *__restrict__ charges_naked, AssembleExtra ext,
    double *__restrict__ partials) {
    const int gtid = xcd_block() * blockDim.x + threadIdx.x;
    const int i = gtid / AS_LANES, sub = gtid % AS_LANES;
    constexpr int NACC = 12 + (VAT ? 9 : 0) + (ISO ? 3 : 0), KS = 12 + (VAT ? 9 : 0);
    float acc[NACC];  // F (3), Z (9)[, per-atom W (9)][, S (3)]
#pragma unroll
    for (int k = 0; k < NACC; ++k) acc[k] = 0.f;
    if (i < N) {
        const float4 pi = xyzt[i];
        const int nA = cntA[i];
        const uint32_t *lrow = listA + (size_t)i * capA;
        // list entries two passes ahead, the start of the neighbour's row one pass ahead
        uint32_t e_next = sub < nA ? lrow[sub] : 0u, e_nn = sub + AS_LANES < nA ? lrow[sub + AS_LANES] : 0u;
        RowProbe rp_next;
        if (sub < nA) probe_load(listA, cntA, nb_index(e_next), capA, rp_next);
        for (int sl = sub; sl < nA; sl += AS_LANES) {
            const uint32_t e = e_next;
            const RowProbe rp = rp_next;
            const int j = nb_index(e);
            const int found = probe_match(listA, j, capA, rp, nb_reverse(e, i));
            float4 fji = make_float4(0.f, 0.f, 0.f, 0.f), aji = fji;
            if (found >= 0) {
                fji = pairFA[((size_t)j * capA + found) * 2];
                aji = pairFA[((size_t)j * capA + found) * 2 + 1];
            }
            if (sl + AS_LANES < nA) {
                e_next = e_nn;
                probe_load(listA, cntA, nb_index(e_next), capA, rp_next);
            }
            if (sl + 2 * AS_LANES < nA) e_nn = lrow[sl + 2 * AS_LANES];
            if (found < 0) continue;  // pair at the cutoff on one side only: contributes zero
            acc[0] -= fji.x;
            acc[1] -= fji.y;
            acc[2] -= fji.z;
            const float3 d = displacement(pi, xyzt, e, c);  // r_ij = -r_ji
            // -1/2 r_ji (x) a_ji = +1/2 r_ij (x) a_ji (ISO: r_ij (x) a_ji)
            const float hz = ISO ? 1.0f : 0.5f;
            const float dv[3] = {hz * d.x, hz * d.y, hz * d.z}, av[3] = {aji.x, aji.y, aji.z};
            if constexpr (ISO) {
                acc[KS] += aji.x;
                acc[KS + 1] += aji.y;
                acc[KS + 2] += aji.z;
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) acc[3 + 3 * a + b] = fmaf(dv[a], av[b], acc[3 + 3 * a + b]);
            if constexpr (VAT) {  // W_i += r_ij (x) F_ji
                const float dd[3] = {d.x, d.y, d.z}, fv[3] = {fji.x, fji.y, fji.z};
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) acc[12 + 3 * a + b] = fmaf(dd[a], fv[b], acc[12 + 3 * a + b]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NACC; ++k)
#pragma unroll
        for (int o = AS_LANES / 2; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o, 64);
    double pv[3] = {0, 0, 0};
    if (i < N && sub == 0) {
        const float s = theta[off_s];
        const float qp = (float)((double)qraw[i] + scalars[S_DELTA]);  // q'
        const float qt = s * qp;                                        // q~'
        const int o = perm[i];
        float z[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const float diag = (k == 0 || k == 4 || k == 8) ? qt : 0.0f;
            z[k] = Znep[(size_t)k * N + i] + acc[3 + k] + diag;
        }
        if constexpr (ISO) {
            float sv[3], rv[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                sv[a] = ext.Siso[(size_t)a * N + i] + acc[KS + a];
                rv[a] = (float)((double)pos[(size_t)a * N + o] - scalars[S_CENT + a] / (double)N);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) z[3 * a + b] = fmaf(rv[a], sv[b], z[3 * a + b]);
        }
        if (forces) {
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const float fext = ext.ex * z[b] + ext.ey * z[3 + b] + ext.ez * z[6 + b];
                forces[(size_t)b * N + o] = Fnep[(size_t)b * N + i] + Fst[(size_t)b * N + i] + acc[b] + fext;
            }
        }
        if (bec) {
#pragma unroll
            for (int k = 0; k < 9; ++k) bec[(size_t)k * N + o] = z[k];
        }
        if constexpr (VAT) {
            // symmetric parts (xx yy zz xy xz yz) + angular reverse terms + background
            const int sym[9] = {0, 3, 4, 3, 1, 5, 4, 5, 2};
            const float ubg = ext.ubg_coef / (s * s);
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const float diag = (k == 0 || k == 4 || k == 8) ? ubg : 0.0f;
                ext.vatom[(size_t)k * N + o] = ext.Vat[(size_t)sym[k] * N + i] + acc[12 + k] + diag;
            }
        }
        if (charges) charges[o] = qp;
        if (charges_naked) charges_naked[o] = qt;
        // polarization with the caller's coordinates (Eq. 26)
        const double qd = (double)s * ((double)qraw[i] + scalars[S_DELTA]);
        pv[0] = qd * (double)pos[o];
        pv[1] = qd * (double)pos[(size_t)N + o];
        pv[2] = qd * (double)pos[(size_t)2 * N + o];
    }
    block_partials<3>(pv, partials);
}

// ---------------------------------------------------------------- launchers
template <int T, int NR, int NA, int NB>
static hipError_t run_descriptors(const Plan &p) {
    const int G = (p.N + 255) / 256;
    hipLaunchKernelGGL((k_descriptors<T, NR, NA, NB>), dim3(G), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell,
                       (float)p.rcR, (float)p.rcA, p.listR, p.cntR, p.capR, p.listA, p.cntA, p.capA, p.theta, p.off_cR,
                       p.off_cA, p.D, p.Amom, p.Bsum);
    return hipGetLastError();
}

template <int T, int NR, int NA, int NB>
static hipError_t run_forces(const Plan &p) {
    const int G = (p.N + 255) / 256;
    hipLaunchKernelGGL((k_radial_tables<T, NR, NB>), dim3(G), dim3(256), 0, p.stream, p.N, p.ts, p.gU, p.gq,
                       p.phi, p.scalars, p.theta, p.off_cR, p.off_s, p.hT);
    const int GR = (int)(((int64_t)p.N * RF_LANES + 255) / 256);
    const bool vat = p.out.virial_atom != nullptr, iso = p.iso != 0;
#define QNEP_RADIAL(V, I)                                                                                        \
    hipLaunchKernelGGL((k_radial_forces<T, NB, V, I>), dim3(GR), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell,      \
                       (float)p.rcR, p.listR, p.cntR, p.capR, p.hT, p.Fnep, p.Znep, p.Vat, p.Siso, p.partials)
    if (vat && iso) QNEP_RADIAL(true, true);
    else if (vat) QNEP_RADIAL(true, false);
    else if (iso) QNEP_RADIAL(false, true);
    else QNEP_RADIAL(false, false);
#undef QNEP_RADIAL
    hipError_t e = reduce_partials(p, GR, 9, S_WNEP, false);
    if (e != hipSuccess) return e;
    stage_mark(p, ST_RADIAL, 3);
    const int GF = (p.N + AF_APB - 1) / AF_APB;
#define QNEP_ANGULAR(I)                                                                                          \
    hipLaunchKernelGGL((k_angular_forces<T, NR, NA, NB, I>), dim3(GF), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell, \
                       (float)p.rcA, p.listA, p.cntA, p.capA, p.Amom, p.gU, p.gq, p.phi, p.scalars, p.theta,       \
                       p.off_cA, p.off_s, (float4 *)p.pairFA, p.Fnep, p.Znep, p.Siso, p.partials)
    if (iso) QNEP_ANGULAR(true);
    else QNEP_ANGULAR(false);
#undef QNEP_ANGULAR
    stage_mark(p, ST_ANG);
    e = reduce_partials(p, GF, 9, S_WNEP, true);
    if (e != hipSuccess) return e;
    stage_mark(p, ST_OTHER);
    const int GA = (int)(((int64_t)p.N * AS_LANES + 255) / 256);
    AssembleExtra ext{p.efield[0], p.efield[1], p.efield[2],
                      (p.mode == 1 && !iso)
                          ? (float)(-KE * PI_D * p.qtot * p.qtot / (2.0 * p.vol * p.alpha * p.alpha * p.N))
                          : 0.0f,
                      p.Vat, p.out.virial_atom, p.Siso};
#define QNEP_ASSEMBLE(V, I)                                                                                      \
    hipLaunchKernelGGL((k_assemble<V, I>), dim3(GA), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell, p.listA, p.cntA, \
                       p.capA, (const float4 *)p.pairFA, p.Fnep, p.Znep, p.Fst, p.qraw, p.scalars, p.theta,       \
                       p.off_s, p.perm, p.pos, p.out.forces, p.out.bec, p.out.charges, p.out.charges_naked, ext,  \
                       p.partials)
    if (vat && iso) QNEP_ASSEMBLE(true, true);
    else if (vat) QNEP_ASSEMBLE(true, false);
    else if (iso) QNEP_ASSEMBLE(false, true);
    else QNEP_ASSEMBLE(false, false);
#undef QNEP_ASSEMBLE
    e = reduce_partials(p, GA, 3, S_POL, false);
    stage_mark(p, ST_ASSEMBLE, 2);
    return e;
}

// compiled hyper-parameter sets: (T, n_max_R + 1, n_max_A + 1, basis + 1), l_max = 4
#define QNEP_DISPATCH(FN)                                                                                  \
    if (p.NBR == 9 && p.NBA == 9 && p.LMAX == 4) {                                                         \
        if (p.NR == 5 && p.NA == 5) {                                                                      \
            if (p.T == 1) return FN<1, 5, 5, 9>(p);                                                        \
            if (p.T == 2) return FN<2, 5, 5, 9>(p);                                                        \
            if (p.T == 3) return FN<3, 5, 5, 9>(p);                                                        \
            if (p.T == 4) return FN<4, 5, 5, 9>(p);                                                        \
        }                                                                                                  \
        if (p.NR == 9 && p.NA == 7) {                                                                      \
            if (p.T == 1) return FN<1, 9, 7, 9>(p);                                                        \
            if (p.T == 2) return FN<2, 9, 7, 9>(p);                                                        \
            if (p.T == 3) return FN<3, 9, 7, 9>(p);                                                        \
            if (p.T == 4) return FN<4, 9, 7, 9>(p);                                                        \
        }                                                                                                  \
    }                                                                                                      \
    return hipErrorInvalidValue;

hipError_t launch_descriptors(const Plan &p) { QNEP_DISPATCH(run_descriptors) }
hipError_t launch_forces(const Plan &p) { QNEP_DISPATCH(run_forces) }

bool nep_supported(int T, int NR, int NA, int NBR, int NBA, int LMAX) {
    if (NBR != 9 || NBA != 9 || LMAX != 4 || T < 1 || T > 4) return false;
    return (NR == 5 && NA == 5) || (NR == 9 && NA == 7);
}

int radial_record_floats(int NB) { return (2 * NB + 3) / 4 * 4; }

}  // namespace qnep
