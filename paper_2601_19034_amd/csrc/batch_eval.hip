// Batched evaluation, per-item part: one persistent launch over (structure, candidate)
// work items pulled from an atomic queue (largest structures first), and the adjoint
// launch that returns the gradient of the training loss (Sec. 2.5) with respect to
// every parameter.
//
// Forward item: parameters staged in LDS, descriptors (Sec. 2.1), network (Eq. 1),
// charge scaling and neutrality correction (Sec. 2.5), potentials phi = A q' from the
// Ewald pair matrix, chi = phi - mean(phi), partial forces F_ij = g_i . dD_i/dr_ij with
// g_i = dU_i/dD + chi_i dq_i/dD (Sec. 2.3) accumulated in FP64 LDS, then E, W and the
// losses Delta_e = |E - E_ref|/N, Delta_f = RMS(F - F_ref), Delta_Q = |s sum q - Q|.
//
// Adjoint item (reverse mode through the force computation).  With upstream weights
// eps_E = dL/dE, u_i = dL/dF_i and eps_Q = dL/dQ from the aggregated loss, the item's
// objective is J = eps_E E + sum_i u_i . F_i + eps_Q s sum_i q_i.  The force part is
// rewritten as sum_i g_i . nu_i with nu_i = sum_p (dD_i/dd_p) (u_i - u_j(p)) (a tangent
// of the descriptors along the displacement perturbations) plus the quadratic form
// q'^T B q' with B = sum_a diag(u_a) G_a for the static Coulomb forces.  Its gradient
// needs the tangent sums dB_i[t][k] = sum_{p in t} f'_k r' and dA_nlm, the network's
// second-order terms (zeta = sigma (rho - 2 h a z'), tau = a sigma with sigma = 1 - h^2,
// z' = W0 nu, a = w1E + chi w1q, rho = eps_E w1E + qbar w1q) and the charge adjoint
// qbar' = eps_E phi + B q' + B^T q' + A (kappa - mean kappa), kappa_i = w1q . (sigma z').
#include "batch.h"
#include "mfma.h"
#include "nep_math.h"
#include "plan.h"

namespace qnep {

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
__device__ inline double group_sum_d(double v, int G) {
    for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline int lm_degree(int m) { return m < 3 ? 0 : (m < 8 ? 1 : (m < 15 ? 2 : 3)); }

// work item shared by the phases
struct Item {
    int s, c, n, G, lig, grp, per_round, cls;
    int64_t atom0, mat0;
};

// Lanes per atom of the descriptor sums and of the FP32 network's hidden-unit sums, per
// size class: fixed (not tuned), so that the FP32 order of those sums, and with it every
// output, does not depend on the autotuner's choice for the other phases (the forces
// accumulate in fixed point, independent of the order).
__constant__ int kDescGroups[BATCH_CLASSES] = {8, 4, 2, 1};

__device__ inline Item make_item(const BatchArgs &a, int item, int4 groups) {
    Item it;
    it.s = a.order[item / a.C];
    it.c = item % a.C;
    const BatchStruct &b = a.st[it.s];
    it.n = b.n;
    it.atom0 = b.atom0;
    it.mat0 = b.mat0;
    it.cls = b.group;
    it.G = b.group == 0 ? groups.x : (b.group == 1 ? groups.y : (b.group == 2 ? groups.z : groups.w));
    it.per_round = BATCH_THREADS / it.G;
    it.lig = threadIdx.x % it.G;
    it.grp = threadIdx.x / it.G;
    return it;
}

// ---------------------------------------------------------------- descriptors
// D (radial then angular l-major), A_nlm and optionally the per-species radial basis
// sums B[t][k] of every atom, SoA with stride M.
template <int T, int NR, int NA, int NB>
__device__ __forceinline__ void item_descriptors(const BatchArgs &a, const Item &it, const float *th, int M,
                                                 float *sD, float *sA, float *sB, int MA) {
    const float *cR = th, *cA = th + a.off_cA;
    const int G = kDescGroups[it.cls], lig = threadIdx.x % G, grp = threadIdx.x / G, per_round = BATCH_THREADS / G;
    for (int i0 = 0; i0 < it.n; i0 += per_round) {
        const int i = i0 + grp;
        const bool act = i < it.n;
        const int64_t g = it.atom0 + (act ? i : 0);
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
        if (!act) continue;
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
        if (sB) {
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int k = 0; k < NB; ++k)
                    if ((t * NB + k) % G == lig) sB[(size_t)(t * NB + k) * M + i] = B[t][k];
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
            for (int m = 0; m < LM; ++m) sA[(size_t)(q * LM + m) * MA + i] = Am[q][m];
        }
    }
}

// ---------------------------------------------------------------- network
// U_i, q_i, dU/dD and dq/dD of every atom.  FP32: hidden units split over the lanes
// of a group.  BF16 (a.prec != FP32 and !fp32): matrix cores in transposed form so
// that no operand is re-laid out through LDS: per 16-atom tile and species t,
//   Z^T = W0_t D^T (atoms of other species zeroed in the B operand),
//   gU^T = W0_t^T G^T with G = (1 - h^2) w1E (and likewise for q).
// The lane holding column `row` of Z^T holds hidden units 16 jt + 4 lg + e, exactly
// the B-operand elements of G^T it needs for the backward product.
template <int T, int NR, int NA>
__device__ __forceinline__ void item_network(const BatchArgs &a, const Item &it, const float *th, int M,
                                             const float *sD, float *sgU, float *sgq, float *qv, double &accU,
                                             double &accQ, bool fp32, int MG) {
    constexpr int NDES = NR + 4 * NA;
    const float *nnet = th + a.off_nn;
    const float b1E = th[a.off_b1E];
    const int tid = threadIdx.x;
    if (!fp32 && a.prec != QNEP_MLP_FP32) {
        constexpr int KDT = (NDES + 15) / 16;
        const int lane = tid & 63, wave = tid >> 6;
        const int li = lane & 15, lg = lane >> 4;
        const int fmask = forward_mask(a.prec), bmask = backward_mask(a.prec);
        const int nJT = (a.H + 15) >> 4;
        for (int tt = wave; tt < (it.n + 15) / 16; tt += BATCH_THREADS / 64) {
            const int row = 16 * tt + li;
            const bool rok = row < it.n;
            const int tr = rok ? a.types[it.atom0 + row] : -1;
            float dv[KDT][4];
#pragma unroll
            for (int kk = 0; kk < KDT; ++kk)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = 16 * kk + 4 * lg + e;
                    dv[kk][e] = (rok && k < NDES) ? sD[(size_t)k * M + row] : 0.f;
                }
            floatx4 acc[4];
#pragma unroll
            for (int jt = 0; jt < 4; ++jt) acc[jt] = floatx4{0.f, 0.f, 0.f, 0.f};
            for (int t = 0; t < T; ++t) {
                if (__ballot(tr == t) == 0) continue;
                const float *W0 = nnet + t * a.per_species;
#pragma unroll
                for (int kk = 0; kk < KDT; ++kk) {
                    float bo[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) bo[e] = tr == t ? dv[kk][e] : 0.f;
#pragma unroll
                    for (int jt = 0; jt < 4; ++jt) {
                        if (jt >= nJT) continue;
                        float ao[4];
                        const int j = 16 * jt + li;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int k = 16 * kk + 4 * lg + e;
                            ao[e] = (j < a.H && k < NDES) ? W0[j * NDES + k] : 0.f;
                        }
                        acc[jt] = mfma_split_rt(ao, bo, acc[jt], fmask);
                    }
                }
            }
            const int tl = tr < 0 ? 0 : tr;
            const float *W0l = nnet + tl * a.per_species;
            const float *b0 = W0l + a.H * NDES, *w1E = b0 + a.H, *w1q = w1E + a.H;
            float up = 0.f, qp = 0.f, ge[4][4], gqq[4][4];
#pragma unroll
            for (int jt = 0; jt < 4; ++jt)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int j = 16 * jt + 4 * lg + e;
                    ge[jt][e] = gqq[jt][e] = 0.f;
                    if (jt < nJT && j < a.H) {
                        const float hh = tanh_fast(acc[jt][e] - b0[j]);
                        up = fmaf(w1E[j], hh, up);
                        qp = fmaf(w1q[j], hh, qp);
                        const float dh = 1.0f - hh * hh;
                        ge[jt][e] = dh * w1E[j];
                        gqq[jt][e] = dh * w1q[j];
                    }
                }
            up += __shfl_xor(up, 16, 64);
            up += __shfl_xor(up, 32, 64);
            qp += __shfl_xor(qp, 16, 64);
            qp += __shfl_xor(qp, 32, 64);
            if (rok && lg == 0) {
                const float qi = qp - w1q[a.H];
                qv[row] = qi;
                accU += (double)(up - b1E);
                accQ += (double)qi;
            }
            floatx4 gA[KDT], gB[KDT];
#pragma unroll
            for (int vt = 0; vt < KDT; ++vt) gA[vt] = gB[vt] = floatx4{0.f, 0.f, 0.f, 0.f};
            for (int t = 0; t < T; ++t) {
                if (__ballot(tr == t) == 0) continue;
                const float *W0 = nnet + t * a.per_species;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    if (jj >= nJT) continue;
                    float be[4], bq[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        be[e] = tr == t ? ge[jj][e] : 0.f;
                        bq[e] = tr == t ? gqq[jj][e] : 0.f;
                    }
#pragma unroll
                    for (int vt = 0; vt < KDT; ++vt) {
                        float ao[4];
                        const int v = 16 * vt + li;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int j = 16 * jj + 4 * lg + e;
                            ao[e] = (j < a.H && v < NDES) ? W0[j * NDES + v] : 0.f;
                        }
                        gA[vt] = mfma_split_rt(ao, be, gA[vt], bmask);
                        gB[vt] = mfma_split_rt(ao, bq, gB[vt], bmask);
                    }
                }
            }
            if (rok) {
#pragma unroll
                for (int vt = 0; vt < KDT; ++vt)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int v = 16 * vt + 4 * lg + e;
                        if (v < NDES) {
                            sgU[(size_t)v * MG + row] = gA[vt][e];
                            sgq[(size_t)v * MG + row] = gB[vt][e];
                        }
                    }
            }
        }
        return;
    }
    const int G = kDescGroups[it.cls], lig = threadIdx.x % G, grp = threadIdx.x / G, per_round = BATCH_THREADS / G;
    for (int i0 = 0; i0 < it.n; i0 += per_round) {
        const int i = i0 + grp;
        const bool act = i < it.n;
        const int tI = act ? a.types[it.atom0 + i] : 0;
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
        if (!act) continue;
#pragma unroll
        for (int d = 0; d < NDES; ++d) {
            if (d % G != lig) continue;
            sgU[(size_t)d * MG + i] = gu[d];
            sgq[(size_t)d * MG + i] = gqv[d];
        }
        if (lig == 0) {
            const float qi = qp - w1q[a.H];  // b1q follows w1q
            qv[i] = qi;
            accU += (double)(up - b1E);
            accQ += (double)qi;
        }
    }
}

// Work-groups per CU the item kernels are compiled for: two (at most 256 registers per
// lane, two waves per SIMD) for the n_max_A = 4 models, whose kernels spill only a
// little at that size and run 1.8x faster (forward) and 1.4x (adjoint) than at one
// wave per SIMD; one for the larger models, which would spill far more.
#define BATCH_MIN_BLOCKS(NA) ((NA) <= 5 ? 2 : 1)

// ---------------------------------------------------------------- forward launches
// Three launches per set of items: (1) k_batch_front, per item: parameters staged in
// LDS, descriptors, network, charge scaling and neutrality correction; the moments and
// the network gradients go to the item's block of a.persist and the corrected charges
// q' to a.qbuf[atom][candidate]; (2) k_batch_es_gemm, per structure: the Ewald pair
// matrices [comp][j][i] times the charges of all candidates [j][c] on the matrix cores
// (each matrix is read once for all candidates), into a.ybuf; (3) k_batch_back, per
// item: chi = phi - mean(phi), partial forces, energy, virial and losses.
template <int T, int NR, int NA, int NB>
__global__ __launch_bounds__(BATCH_THREADS, BATCH_MIN_BLOCKS(NA)) void k_batch_front(BatchArgs a, int item_begin, int item_end,
                                                               int4 groups) {
    constexpr int NDES = NR + 4 * NA;
    extern __shared__ double lds[];
    __shared__ double red[4 * 16];
    __shared__ int s_item;
    const int M = a.max_atoms;
    float *th = reinterpret_cast<float *>(lds);  // parameters of the candidate
    float *qv = th + a.n_theta;                   // q per atom
    const int tid = threadIdx.x;
    float *sD = a.scratch + (size_t)blockIdx.x * (3 * NDES + LM * NA) * M;
    for (;;) {
        if (tid == 0) s_item = item_begin + atomicAdd(a.counter, 1);
        __syncthreads();
        const int item = s_item;
        if (item >= item_end) break;
        const Item it = make_item(a, item, groups);
        const int n = it.n;
        float *sA = a.persist + (size_t)a.F * ((size_t)a.C * it.atom0 + (size_t)it.c * n);
        float *sgU = sA + (size_t)LM * NA * n, *sgq = sgU + (size_t)NDES * n;
        const float *thc = a.thetas + (size_t)it.c * a.n_theta;
        for (int k = tid; k < a.n_theta; k += BATCH_THREADS) th[k] = thc[k];
        __syncthreads();
        const float sc = th[a.off_s];
        item_descriptors<T, NR, NA, NB>(a, it, th, M, sD, sA, nullptr, n);
        __syncthreads();
        double accU = 0.0, accQ = 0.0;
        item_network<T, NR, NA>(a, it, th, M, sD, sgU, sgq, qv, accU, accQ, false, n);
        double r1[2] = {accU, accQ};
        block_sum<2>(r1, red);
        // neutrality correction on the scaled charges: q~' = s q + (Q - s sum q)/N, q' = q~'/s
        const float delta = (float)((a.qtot / (double)sc - r1[1]) / n);
        for (int i = tid; i < n; i += BATCH_THREADS) a.qbuf[(size_t)(it.atom0 + i) * a.C16 + it.c] = qv[i] + delta;
        if (tid == 0) {
            const size_t sc_idx = (size_t)it.s * a.C + it.c;
            a.iscal[2 * sc_idx] = r1[0];
            a.iscal[2 * sc_idx + 1] = r1[1];
        }
        __syncthreads();
    }
}

// y[c][comp][i] = sum_j M[comp][j][i] q'_c[j] for the structures of ranks [rank0, rank0 +
// gridDim.y), all candidates at once: block (row block of 128 rows (comp, i), structure),
// each wave 32 rows (two M-tiles) x 64 candidates (four N-tiles), four atoms j per step,
// v_mfma_f32_16x16x4f32 (lane l: A[i][k] at i = l % 16, k = l / 16; B[k][j] at
// j = l % 16, k = l / 16; D[i][j] at j = l % 16, i = 4 (l / 16) + e).
typedef float floatx4_t __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_batch_es_gemm(BatchArgs a, int rank0) {
    const int s = a.order[rank0 + blockIdx.y];
    const BatchStruct &b = a.st[s];
    const int n = b.n, rows = a.ncomp * n;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int row0 = blockIdx.x * 128 + wave * 32;
    if (row0 >= rows) return;  // the whole wave; no block-wide synchronization below
    const float *Mb = a.mats + b.mat0;
    const int64_t nn = (int64_t)n * n;
    const int m = l & 15, k = l >> 4;
    const int ra = row0 + m, rb = row0 + 16 + m;
    const bool va = ra < rows, vb = rb < rows;
    const int ca = va ? ra / n : 0, cb = vb ? rb / n : 0;
    const float *pa = Mb + ca * nn + (va ? ra - ca * n : 0);
    const float *pb = Mb + cb * nn + (vb ? rb - cb * n : 0);
    const float *Q = a.qbuf + (size_t)b.atom0 * a.C16;
    const int C = a.C;
    floatx4_t acc[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[u][t] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    for (int j0 = 0; j0 < n; j0 += 4) {
        const int j = j0 + k;
        const bool ok = j < n;
        const int jc = ok ? j : 0;
        const float xa = (ok && va) ? pa[(int64_t)jc * n] : 0.f;
        const float xb = (ok && vb) ? pb[(int64_t)jc * n] : 0.f;
        float bv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int c = 16 * t + m;
            bv[t] = (ok && c < C) ? Q[(size_t)jc * a.C16 + c] : 0.f;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            acc[0][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa, bv[t], acc[0][t], 0, 0, 0);
            acc[1][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xb, bv[t], acc[1][t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int c = 16 * t + m;
        if (c >= C) continue;
        float *y = a.ybuf + (size_t)a.ncomp * ((size_t)C * b.atom0 + (size_t)c * n);
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = row0 + 16 * u + 4 * k + e;
                if (row < rows) y[row] = acc[u][t][e];
            }
    }
}

template <int T, int NR, int NA, int NB>
__global__ __launch_bounds__(BATCH_THREADS, BATCH_MIN_BLOCKS(NA)) void k_batch_back(BatchArgs a, int item_begin, int item_end,
                                                              int4 groups) {
    constexpr int NDES = NR + 4 * NA;
    extern __shared__ double lds[];
    __shared__ double red[4 * 16];
    __shared__ int s_item;
    const int M = a.max_atoms;
    // forces accumulate in 64-bit fixed point (to_fixed) so that the sum does not
    // depend on the order of the LDS atomics (pair terms can be much larger than
    // their sum)
    unsigned long long *fx = reinterpret_cast<unsigned long long *>(lds), *fy = fx + M, *fz = fy + M;
    float *th = reinterpret_cast<float *>(fz + M);  // parameters of the candidate
    float *qv = th + a.n_theta;                      // q' per atom
    float *phi = qv + M;                             // potential, then chi
    const int tid = threadIdx.x;
    const float *cR = th, *cA = th + a.off_cA;

    for (;;) {
        if (tid == 0) s_item = item_begin + atomicAdd(a.counter, 1);
        __syncthreads();
        const int item = s_item;
        if (item >= item_end) break;
        const Item it = make_item(a, item, groups);
        const int n = it.n, G = it.G, lig = it.lig;
        const float *thc = a.thetas + (size_t)it.c * a.n_theta;
        for (int k = tid; k < a.n_theta; k += BATCH_THREADS) th[k] = thc[k];
        for (int i = tid; i < n; i += BATCH_THREADS) qv[i] = a.qbuf[(size_t)(it.atom0 + i) * a.C16 + it.c];
        __syncthreads();
        const float sc = th[a.off_s];
        const size_t sc_idx0 = (size_t)it.s * a.C + it.c;
        const double sumU = a.iscal[2 * sc_idx0], sumq = a.iscal[2 * sc_idx0 + 1];
        const float *sA = a.persist + (size_t)a.F * ((size_t)a.C * it.atom0 + (size_t)it.c * n);
        const float *sgU = sA + (size_t)LM * NA * n, *sgq = sgU + (size_t)NDES * n;

        // ---- electrostatics: y = M q' for every stored component (from the product launch)
        double accP = 0.0, accE = 0.0, wes[6] = {0, 0, 0, 0, 0, 0};
        {
            const float *yb = a.ybuf + (size_t)a.ncomp * ((size_t)a.C * it.atom0 + (size_t)it.c * n);
            const int units = a.ncomp * n;
            for (int u = tid; u < units; u += BATCH_THREADS) {
                const int comp = u / n, i = u - comp * n;
                const float y = yb[u];
                const float qi = qv[i];
                if (comp == 0) {
                    phi[i] = y;
                    accP += (double)y;
                    accE += 0.5 * (double)qi * (double)y;
                } else if (comp == 1) {
                    fx[i] = to_fixed((double)qi * y);
                } else if (comp == 2) {
                    fy[i] = to_fixed((double)qi * y);
                } else if (comp == 3) {
                    fz[i] = to_fixed((double)qi * y);
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
        for (int i0 = 0; i0 < n; i0 += it.per_round) {
            const int i = i0 + it.grp;
            const bool act = i < n;
            const int64_t g = it.atom0 + (act ? i : 0);
            const int tI = act ? a.types[g] : 0;
            const float chi = act ? phi[i] : 0.f;
            const float4 *row = a.list + g * a.capR;
            const int nR = act ? a.cntR[g] : 0, nA = act ? a.cntA[g] : 0;
            double ox = 0.0, oy = 0.0, oz = 0.0;
            {  // radial: e[t][k] = sum_n g_n cR[ti][t][n][k],  F_ij = (sum_k e[tj][k] f_k'(r)) r_hat
                float gR[NR];
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    gR[q] = act ? fmaf(chi, sgq[(size_t)q * n + i], sgU[(size_t)q * n + i]) : 0.f;
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
                    atomicAdd(&fx[j], to_fixed(-(double)Fx));
                    atomicAdd(&fy[j], to_fixed(-(double)Fy));
                    atomicAdd(&fz[j], to_fixed(-(double)Fz));
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
                        const size_t rw = (size_t)(NR + l * NA + q) * n + i;
                        Gl[l] = act ? 2.0f * fmaf(chi, sgq[rw], sgU[rw]) : 0.f;
                    }
#pragma unroll
                    for (int m = 0; m < LM; ++m) At[q][m] = act ? Gl[lm_degree(m)] * sA[(size_t)(q * LM + m) * n + i] : 0.f;
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
                    atomicAdd(&fx[j], to_fixed(-(double)Fx));
                    atomicAdd(&fy[j], to_fixed(-(double)Fy));
                    atomicAdd(&fz[j], to_fixed(-(double)Fz));
                    m9[0] -= Fx * e.x; m9[1] -= Fx * e.y; m9[2] -= Fx * e.z;
                    m9[3] -= Fy * e.x; m9[4] -= Fy * e.y; m9[5] -= Fy * e.z;
                    m9[6] -= Fz * e.x; m9[7] -= Fz * e.y; m9[8] -= Fz * e.z;
                }
            }
            ox = group_sum_d(ox, G);
            oy = group_sum_d(oy, G);
            oz = group_sum_d(oz, G);
            if (act && lig == 0) {
                atomicAdd(&fx[i], to_fixed(ox));
                atomicAdd(&fy[i], to_fixed(oy));
                atomicAdd(&fz[i], to_fixed(oz));
            }
        }
        __syncthreads();

        // ---- outputs and losses
        double accF = 0.0;
        for (int i = tid; i < n; i += BATCH_THREADS) {
            const int64_t g = it.atom0 + i;
            const float Fx = (float)from_fixed(fx[i]), Fy = (float)from_fixed(fy[i]), Fz = (float)from_fixed(fz[i]);
            const double ex = (double)Fx - a.F_ref[g], ey = (double)Fy - a.F_ref[a.n_total + g],
                         ez = (double)Fz - a.F_ref[2 * a.n_total + g];
            accF += ex * ex + ey * ey + ez * ez;
            if (a.forces) {
                float *F = a.forces + (size_t)it.c * 3 * a.n_total;
                F[g] = Fx;
                F[a.n_total + g] = Fy;
                F[2 * a.n_total + g] = Fz;
            }
            if (a.charges) a.charges[(size_t)it.c * a.n_total + g] = sc * qv[i];
        }
        double r3[10] = {accF, m9[0], m9[1], m9[2], m9[3], m9[4], m9[5], m9[6], m9[7], m9[8]};
        block_sum<10>(r3, red);
        if (tid == 0) {
            const size_t sc_idx = (size_t)it.s * a.C + it.c;
            const double E = sumU + Ues;
            const double sq = (double)sc * sumq;
            a.losses[3 * sc_idx + 0] = (float)(fabs(E - a.E_ref[it.s]) / n);
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

// ---------------------------------------------------------------- adjoint launch
template <int T, int NR, int NA, int NB>
__global__ __launch_bounds__(BATCH_THREADS, BATCH_MIN_BLOCKS(NA)) void k_batch_adjoint(BatchArgs a, AdjArgs g, int4 groups) {
    constexpr int NDES = NR + 4 * NA;
    extern __shared__ double lds[];
    __shared__ double red[4 * 16];
    __shared__ int s_item;
    __shared__ int s_first[MAX_T + 1];
    const int M = a.max_atoms, H = a.H;
    float *th = reinterpret_cast<float *>(lds);  // parameters of the candidate
    float *gth = th + a.n_theta;                 // gradient of this item
    float *qv = gth + a.n_theta;                 // q'
    float *phi = qv + M;                         // phi (not centred)
    float *kap = phi + M;                        // kappa, then kappa - mean
    float *qb = kap + M;                         // charge adjoints
    float *ux = qb + M, *uy = ux + M, *uz = uy + M;  // dL/dF
    int *sidx = reinterpret_cast<int *>(uz + M);     // atoms grouped by species
    const int tid = threadIdx.x;
    float *scr = g.scratch + (size_t)blockIdx.x * batch_adj_floats(T, NR, NA, NB, H) * M;
    float *sD = scr, *sA = sD + (size_t)NDES * M, *sgU = sA + (size_t)LM * NA * M, *sgq = sgU + (size_t)NDES * M;
    float *sB = sgq + (size_t)NDES * M, *sBd = sB + (size_t)T * NB * M, *sAd = sBd + (size_t)T * NB * M;
    float *sNu = sAd + (size_t)LM * NA * M, *sH = sNu + (size_t)NDES * M, *sZd = sH + (size_t)H * M;
    float *sZe = sZd + (size_t)H * M, *sTa = sZe + (size_t)H * M, *sDb = sTa + (size_t)H * M;
    float *sNb = sDb + (size_t)NDES * M;
    const float *cR = th, *cA = th + a.off_cA, *nnet = th + a.off_nn;
    const int n_items = a.S * a.C;

    for (;;) {
        if (tid == 0) s_item = atomicAdd(a.counter, 1);
        __syncthreads();
        const int item = s_item;
        if (item >= n_items) break;
        const Item it = make_item(a, item, groups);
        const int n = it.n, G = it.G, lig = it.lig;
        const float *thc = a.thetas + (size_t)it.c * a.n_theta;
        for (int k = tid; k < a.n_theta; k += BATCH_THREADS) {
            th[k] = thc[k];
            gth[k] = 0.f;
        }
        // atoms grouped by species (stable, deterministic)
        if (tid == 0) {
            int pos = 0;
            for (int t = 0; t < T; ++t) {
                s_first[t] = pos;
                for (int i = 0; i < n; ++i)
                    if (a.types[it.atom0 + i] == t) sidx[pos++] = i;
            }
            s_first[T] = pos;
        }
        __syncthreads();
        const float sc = th[a.off_s];
        // upstream weights of this item from the aggregated loss
        const double *st4 = a.stats + 4 * ((size_t)it.s * a.C + it.c);
        const double *rm = g.rmse + 4 * it.c;
        const double es = (st4[0] - a.E_ref[it.s]) / n;
        const float epsE = rm[0] > 0 ? (float)(g.lam[0] * es / (a.S * rm[0] * n)) : 0.f;
        const float kf = rm[1] > 0 ? (float)(g.lam[1] / (g.nf * rm[1])) : 0.f;
        const float epsQ = rm[2] > 0 ? (float)(g.lam[2] * (st4[2] - a.qtot) / (a.S * rm[2])) : 0.f;

        // ---- forward quantities
        item_descriptors<T, NR, NA, NB>(a, it, th, M, sD, sA, sB, M);
        __syncthreads();
        double accU = 0.0, accQ = 0.0;
        item_network<T, NR, NA>(a, it, th, M, sD, sgU, sgq, qv, accU, accQ, true, M);
        double r1[1] = {accQ};
        block_sum<1>(r1, red);
        const double sumq = r1[0];
        const float delta = (float)((a.qtot / (double)sc - sumq) / n);
        const float *Fc = g.forces + (size_t)it.c * 3 * a.n_total;
        for (int i = tid; i < n; i += BATCH_THREADS) {
            qv[i] += delta;
            const int64_t gi = it.atom0 + i;
            ux[i] = kf * (Fc[gi] - a.F_ref[gi]);
            uy[i] = kf * (Fc[a.n_total + gi] - a.F_ref[a.n_total + gi]);
            uz[i] = kf * (Fc[2 * a.n_total + gi] - a.F_ref[2 * a.n_total + gi]);
        }
        __syncthreads();
        // phi = A q' and sum_a u_ia (G_a q')_i: with the FP32 network the forward launch
        // of this gradient call formed the same products from the same q' (a.ybuf)
        const int64_t nn = (int64_t)n * n;
        const float *Mb = a.mats + it.mat0;
        double accP = 0.0;
        if (a.prec == QNEP_MLP_FP32) {
            const float *yb = a.ybuf + (size_t)a.ncomp * ((size_t)a.C * it.atom0 + (size_t)it.c * n);
            for (int i = tid; i < n; i += BATCH_THREADS) {
                const float s0 = yb[i], s1 = yb[n + i], s2 = yb[2 * n + i], s3 = yb[3 * n + i];
                phi[i] = s0;
                accP += (double)s0;
                qb[i] = ux[i] * s1 + uy[i] * s2 + uz[i] * s3;
            }
        } else {
            for (int i = tid; i < n; i += BATCH_THREADS) {
                float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
                for (int j = 0; j < n; ++j) {
                    const float qj = qv[j];
                    const int64_t o = (int64_t)j * n + i;
                    s0 = fmaf(Mb[o], qj, s0);
                    s1 = fmaf(Mb[nn + o], qj, s1);
                    s2 = fmaf(Mb[2 * nn + o], qj, s2);
                    s3 = fmaf(Mb[3 * nn + o], qj, s3);
                }
                phi[i] = s0;
                accP += (double)s0;
                qb[i] = ux[i] * s1 + uy[i] * s2 + uz[i] * s3;
            }
        }
        double r2[1] = {accP};
        block_sum<1>(r2, red);
        const float phibar = (float)(r2[0] / n);

        // ---- tangents along w_p = u_i - u_j: dB[t][k], dA_nlm and nu
        for (int i0 = 0; i0 < n; i0 += it.per_round) {
            const int i = i0 + it.grp;
            const bool act = i < n;
            const int64_t gi = it.atom0 + (act ? i : 0);
            const int tI = act ? a.types[gi] : 0;
            const float4 *row = a.list + gi * a.capR;
            const int nR = act ? a.cntR[gi] : 0, nA = act ? a.cntA[gi] : 0;
            const float uix = act ? ux[i] : 0.f, uiy = act ? uy[i] : 0.f, uiz = act ? uz[i] : 0.f;
            float Bd[T][NB];
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int k = 0; k < NB; ++k) Bd[t][k] = 0.f;
            float Ad[NA][LM];
#pragma unroll
            for (int q = 0; q < NA; ++q)
#pragma unroll
                for (int m = 0; m < LM; ++m) Ad[q][m] = 0.f;
            for (int p = lig; p < nR; p += G) {
                const float4 e = row[p];
                const int code = __float_as_int(e.w);
                const int tj = code >> 24, j = code & 0xFFFFFF;
                const float wx = uix - ux[j], wy = uiy - uy[j], wz = uiz - uz[j];
                const float r = sqrtf(e.x * e.x + e.y * e.y + e.z * e.z);
                const float ir = 1.0f / r;
                const float vx = e.x * ir, vy = e.y * ir, vz = e.z * ir;
                const float rd = vx * wx + vy * wy + vz * wz;  // r' along w
                float f[NB], df[NB];
                cheb_basis<NB>(r, a.rcR, f, df);
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    const float msk = tj == t ? rd : 0.f;
#pragma unroll
                    for (int k = 0; k < NB; ++k) Bd[t][k] = fmaf(msk, df[k], Bd[t][k]);
                }
                if (p < nA) {
                    cheb_basis<NB>(r, a.rcA, f, df);
                    const float *cp = cA + (tI * T + tj) * NA * NB;
                    float Y[LM], Yd[LM];
                    harmonics(vx, vy, vz, Y);
                    // tangential change of the direction: (w - u (u.w)) / r
                    harmonics_jvp(vx, vy, vz, (wx - vx * rd) * ir, (wy - vy * rd) * ir, (wz - vz * rd) * ir, Yd);
#pragma unroll
                    for (int q = 0; q < NA; ++q) {
                        float gn = 0.f, dgn = 0.f;
#pragma unroll
                        for (int k = 0; k < NB; ++k) {
                            gn = fmaf(cp[q * NB + k], f[k], gn);
                            dgn = fmaf(cp[q * NB + k], df[k], dgn);
                        }
                        const float gr = dgn * rd;
#pragma unroll
                        for (int m = 0; m < LM; ++m) Ad[q][m] = fmaf(gr, Y[m], fmaf(gn, Yd[m], Ad[q][m]));
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int k = 0; k < NB; ++k) Bd[t][k] = group_sum(Bd[t][k], G);
#pragma unroll
            for (int q = 0; q < NA; ++q)
#pragma unroll
                for (int m = 0; m < LM; ++m) Ad[q][m] = group_sum(Ad[q][m], G);
            if (!act) continue;
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int k = 0; k < NB; ++k)
                    if ((t * NB + k) % G == lig) sBd[(size_t)(t * NB + k) * M + i] = Bd[t][k];
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                if (q % G != lig) continue;
                float acc = 0.f;
#pragma unroll
                for (int t = 0; t < T; ++t)
#pragma unroll
                    for (int k = 0; k < NB; ++k) acc = fmaf(cR[((tI * T + t) * NR + q) * NB + k], Bd[t][k], acc);
                sNu[(size_t)q * M + i] = acc;
            }
#pragma unroll
            for (int q = 0; q < NA; ++q) {
                if ((NR + q) % G != lig) continue;
                float s4[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int m = 0; m < LM; ++m) {
                    s4[lm_degree(m)] = fmaf(sA[(size_t)(q * LM + m) * M + i], Ad[q][m], s4[lm_degree(m)]);
                    sAd[(size_t)(q * LM + m) * M + i] = Ad[q][m];
                }
#pragma unroll
                for (int l = 0; l < 4; ++l) sNu[(size_t)(NR + l * NA + q) * M + i] = 2.0f * s4[l];
            }
        }
        __syncthreads();

        // ---- network tangents: h, z' = W0 nu, kappa = w1q . (sigma z')
        for (int i0 = 0; i0 < n; i0 += it.per_round) {
            const int i = i0 + it.grp;
            const bool act = i < n;
            const int tI = act ? a.types[it.atom0 + i] : 0;
            float Dv[NDES], Nv[NDES];
#pragma unroll
            for (int d = 0; d < NDES; ++d) {
                Dv[d] = act ? sD[(size_t)d * M + i] : 0.f;
                Nv[d] = act ? sNu[(size_t)d * M + i] : 0.f;
            }
            const float *W0 = nnet + tI * a.per_species;
            const float *b0 = W0 + H * NDES, *w1q = b0 + 2 * H;
            float kp = 0.f;
            for (int jn = lig; jn < H; jn += G) {
                const float *w = W0 + jn * NDES;
                float z = -b0[jn], zd = 0.f;
#pragma unroll
                for (int d = 0; d < NDES; ++d) {
                    z = fmaf(w[d], Dv[d], z);
                    zd = fmaf(w[d], Nv[d], zd);
                }
                const float hh = tanhf(z);
                kp = fmaf(w1q[jn] * (1.0f - hh * hh), zd, kp);
                if (act) {
                    sH[(size_t)jn * M + i] = hh;
                    sZd[(size_t)jn * M + i] = zd;
                }
            }
            kp = group_sum(kp, G);
            if (act && lig == 0) kap[i] = kp;
        }
        __syncthreads();
        double r3[1] = {0.0};
        for (int i = tid; i < n; i += BATCH_THREADS) r3[0] += (double)kap[i];
        block_sum<1>(r3, red);
        const float kbar = (float)(r3[0] / n);
        for (int i = tid; i < n; i += BATCH_THREADS) kap[i] -= kbar;
        __syncthreads();

        // ---- charge adjoint: qbar' = eps_E phi + B q' + B^T q' + A (kappa - mean)
        double accB = 0.0;
        for (int i = tid; i < n; i += BATCH_THREADS) {
            float s0 = 0.f, s1 = 0.f;
            for (int j = 0; j < n; ++j) {
                const int64_t o = (int64_t)j * n + i;
                const float qj = qv[j];
                s0 = fmaf(Mb[o], kap[j], s0);
                s1 = fmaf(Mb[nn + o], ux[j] * qj, s1);
                s1 = fmaf(Mb[2 * nn + o], uy[j] * qj, s1);
                s1 = fmaf(Mb[3 * nn + o], uz[j] * qj, s1);
            }
            const float v = epsE * phi[i] + qb[i] - s1 + s0;
            accB += (double)v;
            qb[i] = v;  // only this thread reads qb[i]
        }
        double r4[1] = {accB};
        block_sum<1>(r4, red);
        const float qbm = (float)(r4[0] / n);
        for (int i = tid; i < n; i += BATCH_THREADS) qb[i] = qb[i] - qbm + epsQ * sc;
        __syncthreads();
        if (tid == 0) {
            gth[a.off_s] = (float)(-a.qtot / ((double)sc * sc * n) * r4[0] + epsQ * sumq);
            gth[a.off_b1E] = -epsE * n;
        }

        // ---- network adjoint per atom: zeta, tau, D-bar = W0^T zeta, nu-bar = W0^T tau
        for (int i0 = 0; i0 < n; i0 += it.per_round) {
            const int i = i0 + it.grp;
            const bool act = i < n;
            const int tI = act ? a.types[it.atom0 + i] : 0;
            const float chi = act ? phi[i] - phibar : 0.f;
            const float qbi = act ? qb[i] : 0.f;
            const float *W0 = nnet + tI * a.per_species;
            const float *w1E = W0 + H * NDES + H, *w1q = w1E + H;
            float db[NDES], nb[NDES];
#pragma unroll
            for (int d = 0; d < NDES; ++d) db[d] = nb[d] = 0.f;
            for (int jn = lig; jn < H; jn += G) {
                const float hh = act ? sH[(size_t)jn * M + i] : 0.f;
                const float zd = act ? sZd[(size_t)jn * M + i] : 0.f;
                const float sg = 1.0f - hh * hh;
                const float av = fmaf(chi, w1q[jn], w1E[jn]);
                const float rho = fmaf(epsE, w1E[jn], qbi * w1q[jn]);
                const float ze = sg * (rho - 2.0f * hh * av * zd);
                const float ta = av * sg;
                if (act) {
                    sZe[(size_t)jn * M + i] = ze;
                    sTa[(size_t)jn * M + i] = ta;
                }
                const float *w = W0 + jn * NDES;
#pragma unroll
                for (int d = 0; d < NDES; ++d) {
                    db[d] = fmaf(ze, w[d], db[d]);
                    nb[d] = fmaf(ta, w[d], nb[d]);
                }
            }
#pragma unroll
            for (int d = 0; d < NDES; ++d) {
                db[d] = group_sum(db[d], G);
                nb[d] = group_sum(nb[d], G);
            }
            if (!act) continue;
#pragma unroll
            for (int d = 0; d < NDES; ++d) {
                if (d % G != lig) continue;
                sDb[(size_t)d * M + i] = db[d];
                sNb[(size_t)d * M + i] = nb[d];
            }
        }
        __syncthreads();

        // ---- parameter gradients that are sums over the atoms of one species
        {
            const int per_sp = H * NDES + 3 * H + 1;
            const int nW = T * per_sp;
            const int nC = T * T * NR * NB;
            for (int e = tid; e < nW + nC; e += BATCH_THREADS) {
                float acc = 0.f;
                int64_t dst;
                if (e < nW) {
                    const int t = e / per_sp, r = e - t * per_sp;
                    const int i_lo = s_first[t], i_hi = s_first[t + 1];
                    dst = a.off_nn + (int64_t)t * a.per_species + r;
                    if (r < H * NDES) {  // W0[mu][d]
                        const int mu = r / NDES, d = r - mu * NDES;
                        for (int k = i_lo; k < i_hi; ++k) {
                            const int i = sidx[k];
                            acc = fmaf(sZe[(size_t)mu * M + i], sD[(size_t)d * M + i], acc);
                            acc = fmaf(sTa[(size_t)mu * M + i], sNu[(size_t)d * M + i], acc);
                        }
                    } else if (r < H * NDES + H) {  // b0
                        const int mu = r - H * NDES;
                        for (int k = i_lo; k < i_hi; ++k) acc -= sZe[(size_t)mu * M + sidx[k]];
                    } else if (r < H * NDES + 2 * H) {  // w1E
                        const int mu = r - H * NDES - H;
                        for (int k = i_lo; k < i_hi; ++k) {
                            const int i = sidx[k];
                            const float hh = sH[(size_t)mu * M + i];
                            acc += epsE * hh + (1.0f - hh * hh) * sZd[(size_t)mu * M + i];
                        }
                    } else if (r < H * NDES + 3 * H) {  // w1q
                        const int mu = r - H * NDES - 2 * H;
                        for (int k = i_lo; k < i_hi; ++k) {
                            const int i = sidx[k];
                            const float hh = sH[(size_t)mu * M + i];
                            const float chi = phi[i] - phibar;
                            acc += qb[i] * hh + chi * (1.0f - hh * hh) * sZd[(size_t)mu * M + i];
                        }
                    } else {  // b1q
                        for (int k = i_lo; k < i_hi; ++k) acc -= qb[sidx[k]];
                    }
                } else {  // cR[ti][t][q][k] = sum_{i in ti} Dbar_q B_i[t][k] + nubar_q dB_i[t][k]
                    const int r = e - nW;
                    const int k = r % NB, q = (r / NB) % NR, t = (r / (NB * NR)) % T, ti = r / (NB * NR * T);
                    dst = r;
                    for (int kk = s_first[ti]; kk < s_first[ti + 1]; ++kk) {
                        const int i = sidx[kk];
                        acc = fmaf(sDb[(size_t)q * M + i], sB[(size_t)(t * NB + k) * M + i], acc);
                        acc = fmaf(sNb[(size_t)q * M + i], sBd[(size_t)(t * NB + k) * M + i], acc);
                    }
                }
                gth[dst] = acc;
            }
        }
        __syncthreads();

        // ---- angular coefficients: two passes over the angular pairs of each atom
        // pass 0: Abar_nlm = 2 (Dbar_nl A_nlm + nubar_nl dA_nlm),  c += f_k sum_lm Abar Y
        // pass 1: Adbar_nlm = 2 nubar_nl A_nlm,  c += f_k' r' sum_lm Adbar Y + f_k sum_lm Adbar dY
        for (int pass = 0; pass < 2; ++pass) {
            for (int i0 = 0; i0 < n; i0 += it.per_round) {
                const int i = i0 + it.grp;
                const bool act = i < n;
                const int64_t gi = it.atom0 + (act ? i : 0);
                const int tI = act ? a.types[gi] : 0;
                const float4 *row = a.list + gi * a.capR;
                const int nA = act ? a.cntA[gi] : 0;
                float Tb[NA][LM];
#pragma unroll
                for (int q = 0; q < NA; ++q)
#pragma unroll
                    for (int m = 0; m < LM; ++m) {
                        const size_t rw = (size_t)(NR + lm_degree(m) * NA + q) * M + i;
                        const size_t ra = (size_t)(q * LM + m) * M + i;
                        float v = 0.f;
                        if (act) v = pass == 0 ? 2.0f * (sDb[rw] * sA[ra] + sNb[rw] * sAd[ra]) : 2.0f * sNb[rw] * sA[ra];
                        Tb[q][m] = v;
                    }
                const float uix = act ? ux[i] : 0.f, uiy = act ? uy[i] : 0.f, uiz = act ? uz[i] : 0.f;
                float acc[NA][NB];
#pragma unroll
                for (int q = 0; q < NA; ++q)
#pragma unroll
                    for (int k = 0; k < NB; ++k) acc[q][k] = 0.f;
                int tcur = -1;
                for (int p = lig; p < nA; p += G) {
                    const float4 e = row[p];
                    const int code = __float_as_int(e.w);
                    const int tj = code >> 24, j = code & 0xFFFFFF;
                    if (tj != tcur) {  // neighbours are grouped by species: flush the previous group
                        if (tcur >= 0) {
                            float *dstp = gth + a.off_cA + (tI * T + tcur) * NA * NB;
#pragma unroll
                            for (int q = 0; q < NA; ++q)
#pragma unroll
                                for (int k = 0; k < NB; ++k) {
                                    atomicAdd(&dstp[q * NB + k], acc[q][k]);
                                    acc[q][k] = 0.f;
                                }
                        }
                        tcur = tj;
                    }
                    const float r = sqrtf(e.x * e.x + e.y * e.y + e.z * e.z);
                    const float ir = 1.0f / r;
                    const float vx = e.x * ir, vy = e.y * ir, vz = e.z * ir;
                    float f[NB], df[NB];
                    cheb_basis<NB>(r, a.rcA, f, df);
                    float Y[LM];
                    harmonics(vx, vy, vz, Y);
                    if (pass == 0) {
#pragma unroll
                        for (int q = 0; q < NA; ++q) {
                            float P = 0.f;
#pragma unroll
                            for (int m = 0; m < LM; ++m) P = fmaf(Tb[q][m], Y[m], P);
#pragma unroll
                            for (int k = 0; k < NB; ++k) acc[q][k] = fmaf(f[k], P, acc[q][k]);
                        }
                    } else {
                        const float wx = uix - ux[j], wy = uiy - uy[j], wz = uiz - uz[j];
                        const float rd = vx * wx + vy * wy + vz * wz;
                        float Yd[LM];
                        harmonics_jvp(vx, vy, vz, (wx - vx * rd) * ir, (wy - vy * rd) * ir, (wz - vz * rd) * ir, Yd);
#pragma unroll
                        for (int q = 0; q < NA; ++q) {
                            float P2 = 0.f, P3 = 0.f;
#pragma unroll
                            for (int m = 0; m < LM; ++m) {
                                P2 = fmaf(Tb[q][m], Y[m], P2);
                                P3 = fmaf(Tb[q][m], Yd[m], P3);
                            }
                            P2 *= rd;
#pragma unroll
                            for (int k = 0; k < NB; ++k) acc[q][k] = fmaf(df[k], P2, fmaf(f[k], P3, acc[q][k]));
                        }
                    }
                }
                if (tcur >= 0) {
                    float *dstp = gth + a.off_cA + (tI * T + tcur) * NA * NB;
#pragma unroll
                    for (int q = 0; q < NA; ++q)
#pragma unroll
                        for (int k = 0; k < NB; ++k) atomicAdd(&dstp[q * NB + k], acc[q][k]);
                }
            }
        }
        __syncthreads();
        float *gout = g.grow + ((size_t)it.s * a.C + it.c) * a.n_theta;
        for (int k = tid; k < a.n_theta; k += BATCH_THREADS) gout[k] = gth[k];
        __syncthreads();
    }
}

// Loss per candidate (Sec. 2.5): lambda_e RMSE(E/N) + lambda_f RMSE(F) + lambda_Q RMSE(Q)
// + lambda_1 |theta|_1 + lambda_2 |theta|_2^2, sums over structures in a fixed order;
// the three RMSE values are kept for the adjoint.
__global__ __launch_bounds__(256) void k_b_loss(const double *__restrict__ stats, const double *__restrict__ E_ref,
                                                const float *__restrict__ thetas, int64_t n_theta, int S, int C,
                                                double qtot, double le, double lf, double lq, double l1, double l2,
                                                double *__restrict__ loss, double *__restrict__ rmse) {
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
    if (threadIdx.x == 0) {
        const double re = sqrt(v[0] / S), rf = sqrt(v[1] / v[2]), rq = sqrt(v[3] / S);
        if (loss) loss[c] = le * re + lf * rf + lq * rq + l1 * v[4] + l2 * v[5];
        if (rmse) {
            rmse[4 * c + 0] = re;
            rmse[4 * c + 1] = rf;
            rmse[4 * c + 2] = rq;
            rmse[4 * c + 3] = v[2];
        }
    }
}

// dL/dtheta_c = sum over structures (fixed order) + lambda_1 sign(theta) + 2 lambda_2 theta
__global__ __launch_bounds__(256) void k_b_grad_reduce(const float *__restrict__ grow, const float *__restrict__ thetas,
                                                       int64_t n_theta, int S, int C, double l1, double l2,
                                                       float *__restrict__ dthetas) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)C * n_theta) return;
    const int c = (int)(e / n_theta);
    const int64_t k = e - (int64_t)c * n_theta;
    double acc = 0.0;
    for (int s = 0; s < S; ++s) acc += (double)grow[((size_t)s * C + c) * n_theta + k];
    const double x = thetas[e];
    acc += l1 * (x > 0 ? 1.0 : (x < 0 ? -1.0 : 0.0)) + 2.0 * l2 * x;
    dthetas[e] = (float)acc;
}

// ---------------------------------------------------------------- launchers
bool batch_supported(int T, int NR, int NA, int NB) {
    return T >= 1 && T <= 4 && NB == 9 && ((NR == 5 && NA == 5) || (NR == 9 && NA == 7));
}

template <class K>
static hipError_t launch_persistent(K kernel, size_t lds_bytes, int n_slots, hipStream_t stream) {
    if (lds_bytes > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    (void)n_slots;
    (void)stream;
    return hipSuccess;
}

#define QNEP_BATCH_DISPATCH(T_, NR_, NA_, NB_)                                                              \
    if (T == T_ && NR == NR_ && NA == NA_ && NB == NB_) {                                                   \
        hipError_t e0 = launch_persistent(k_batch_front<T_, NR_, NA_, NB_>, lds_front, n_slots, stream);   \
        if (e0 == hipSuccess) e0 = launch_persistent(k_batch_back<T_, NR_, NA_, NB_>, lds_back, n_slots, stream); \
        if (e0 != hipSuccess) return e0;                                                                    \
        BatchArgs a1 = a, a3 = a;                                                                           \
        a3.counter = a.counter + 1;                                                                         \
        hipLaunchKernelGGL((k_batch_front<T_, NR_, NA_, NB_>), dim3(n_slots), dim3(BATCH_THREADS), lds_front, \
                           stream, a1, item_begin, item_end, groups);                                       \
        hipLaunchKernelGGL(k_batch_es_gemm, dim3(gx, rank_end - rank_begin), dim3(256), 0, stream, a,       \
                           rank_begin);                                                                     \
        hipLaunchKernelGGL((k_batch_back<T_, NR_, NA_, NB_>), dim3(n_slots), dim3(BATCH_THREADS), lds_back,  \
                           stream, a3, item_begin, item_end, groups);                                       \
        return hipGetLastError();                                                                           \
    }

// Items [item_begin, item_end) must cover whole structures (multiples of a.C); the
// caller zeroes a.counter[0..1].
hipError_t batch_eval(const BatchArgs &a, int T, int NR, int NA, int NB, int n_slots, int item_begin,
                      int item_end, int4 groups, hipStream_t stream) {
    if (item_begin % a.C != 0 || item_end % a.C != 0) return hipErrorInvalidValue;
    if (item_end <= item_begin) return hipSuccess;
    const size_t lds_front = sizeof(float) * ((size_t)a.n_theta + (size_t)a.max_atoms);
    const size_t lds_back =
        sizeof(double) * 3 * (size_t)a.max_atoms + sizeof(float) * ((size_t)a.n_theta + 2 * (size_t)a.max_atoms);
    const int rank_begin = item_begin / a.C, rank_end = item_end / a.C;
    const int gx = (a.ncomp * a.max_atoms + 127) / 128;
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
#undef QNEP_BATCH_DISPATCH

#define QNEP_ADJ_DISPATCH(T_, NR_, NA_, NB_)                                                                \
    if (T == T_ && NR == NR_ && NA == NA_ && NB == NB_) {                                                   \
        hipError_t e0 = launch_persistent(k_batch_adjoint<T_, NR_, NA_, NB_>, lds_bytes, n_slots, stream); \
        if (e0 != hipSuccess) return e0;                                                                    \
        hipLaunchKernelGGL((k_batch_adjoint<T_, NR_, NA_, NB_>), dim3(n_slots), dim3(BATCH_THREADS),       \
                           lds_bytes, stream, a, g, groups);                                                \
        return hipGetLastError();                                                                           \
    }

hipError_t batch_adjoint(const BatchArgs &a, const AdjArgs &g, int T, int NR, int NA, int NB, int n_slots,
                         int4 groups, hipStream_t stream) {
    const size_t lds_bytes = sizeof(float) * (2 * (size_t)a.n_theta + 8 * (size_t)a.max_atoms) +
                             sizeof(int) * (size_t)a.max_atoms;
    QNEP_ADJ_DISPATCH(1, 5, 5, 9)
    QNEP_ADJ_DISPATCH(2, 5, 5, 9)
    QNEP_ADJ_DISPATCH(3, 5, 5, 9)
    QNEP_ADJ_DISPATCH(4, 5, 5, 9)
    QNEP_ADJ_DISPATCH(1, 9, 7, 9)
    QNEP_ADJ_DISPATCH(2, 9, 7, 9)
    QNEP_ADJ_DISPATCH(3, 9, 7, 9)
    QNEP_ADJ_DISPATCH(4, 9, 7, 9)
    return hipErrorInvalidValue;
}
#undef QNEP_ADJ_DISPATCH

hipError_t batch_loss(const double *stats, const double *E_ref, const float *thetas, int64_t n_theta, int S, int C,
                      double qtot, const double *lam, double *loss, double *rmse, hipStream_t stream) {
    hipLaunchKernelGGL(k_b_loss, dim3(C), dim3(256), 0, stream, stats, E_ref, thetas, n_theta, S, C, qtot, lam[0],
                       lam[1], lam[2], lam[3], lam[4], loss, rmse);
    return hipGetLastError();
}

hipError_t batch_grad_reduce(const float *grow, const float *thetas, int64_t n_theta, int S, int C, double l1,
                             double l2, float *dthetas, hipStream_t stream) {
    const int64_t total = (int64_t)C * n_theta;
    hipLaunchKernelGGL(k_b_grad_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, grow, thetas,
                       n_theta, S, C, l1, l2, dthetas);
    return hipGetLastError();
}

}  // namespace qnep
