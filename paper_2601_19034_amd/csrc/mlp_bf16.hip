// BF16 matrix-core forms of the per-species network (Sec. 2.1 Eq. 1, Sec. 2.2):
//   Z = D W0_t^T, h = tanh(Z - b0_t), U = w1E_t . h - b1E, q = w1q_t . h - b1q_t,
//   dU/dD = [(1 - h^2) w1E_t] W0_t, dq/dD = [(1 - h^2) w1q_t] W0_t.
// One wave computes a tile of 16 consecutive (spatially sorted) atoms with
// v_mfma_f32_16x16x16_bf16 (BF16 inputs, FP32 accumulation), in transposed form:
//   Z^T = sum_t W0_t D_t^T   (columns = atoms; atoms of other species zeroed in B),
//   gU^T = sum_t W0_t^T G_t^T with G = (1 - h^2) w1E (and likewise for q).
// After the first product the lane that holds column `row` holds the hidden units
// 16 jt + 4 lg + e of that atom, which are exactly the B-operand elements of G^T the
// second product needs, so no activation goes through LDS.
// Precision: operands are split into BF16 hi + lo parts.  The forward product keeps
// hi*hi + hi*lo + lo*hi; the backward product keeps the split weights against the
// activation gradient's hi part (QNEP_MLP_BF16), or both splits (QNEP_MLP_BF16X3).  The
// descriptors enter tanh and through (1 - h^2) every force, so their rounding matters
// most; a single BF16 rounding of both operands misses 5 meV/A on the forces.
// The BF16 weight parts of the species present sit in LDS in the two layouts the
// products read (rows of W0 and rows of W0^T, four consecutive elements per lane).
#include "mfma.h"
#include "plan.h"

namespace qnep {

template <int KD, int KH, int BMASK>
__global__ __launch_bounds__(256) void k_mlp_bf16(int N, int T, int H, int ndes, const int *__restrict__ ts,
                                                  const float *__restrict__ D, const float *__restrict__ theta,
                                                  int64_t off_nn, int64_t per_species, int64_t off_b1E,
                                                  float *__restrict__ U, float *__restrict__ qraw,
                                                  float *__restrict__ gU, float *__restrict__ gq,
                                                  double *__restrict__ partials) {
    constexpr int RF = KD + 4, RB = KH + 4;  // padded row lengths (elements)
    constexpr bool BLO = (BMASK & SPLIT_A_LO) != 0;  // weights' lo part in the backward product
    extern __shared__ short wlds[];
    // [t][j][k] rows of W0 (forward, hi and lo) and [t][v][j] rows of W0^T (backward, hi [and lo])
    short *fh = wlds, *fl = fh + T * KH * RF, *bh = fl + T * KH * RF, *bl = bh + T * KD * RB;
    __shared__ float sb0[MAX_T][KH], sw1E[MAX_T][KH], sw1q[MAX_T][KH], sb1q[MAX_T];
    for (int idx = threadIdx.x; idx < T * KH * KD; idx += blockDim.x) {
        const int t = idx / (KH * KD), r = idx - t * KH * KD, j = r / KD, k = r - j * KD;
        const float w = (j < H && k < ndes) ? theta[off_nn + t * per_species + (int64_t)j * ndes + k] : 0.0f;
        const short h = to_bf16(w);
        const short l = to_bf16(w - __uint_as_float((uint32_t)(unsigned short)h << 16));
        fh[(t * KH + j) * RF + k] = h;
        fl[(t * KH + j) * RF + k] = l;
        bh[(t * KD + k) * RB + j] = h;
        if (BLO) bl[(t * KD + k) * RB + j] = l;
    }
    for (int idx = threadIdx.x; idx < T * KH; idx += blockDim.x) {
        const int t = idx / KH, j = idx % KH;
        const float *base = theta + off_nn + t * per_species + (int64_t)H * ndes;
        sb0[t][j] = j < H ? base[j] : 0.0f;
        sw1E[t][j] = j < H ? base[H + j] : 0.0f;
        sw1q[t][j] = j < H ? base[2 * H + j] : 0.0f;
        if (j == 0) sb1q[t] = base[3 * H];
    }
    __syncthreads();
    const float b1E = theta[off_b1E];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int ntiles = (N + 15) / 16;
    const int stride = gridDim.x * 4;
    const bf16x4 zero4 = {0, 0, 0, 0};
    double red[2] = {0.0, 0.0};
    // the descriptors and species of the wave's next tile are loaded while the current
    // tile is computed
    float dn[KD / 16][4];
    int tn;
    auto load_tile = [&](int tile) {
        const int row = 16 * tile + li;
        const bool rok = tile < ntiles && row < N;
        tn = rok ? ts[row] : -1;
#pragma unroll
        for (int kk = 0; kk < KD / 16; ++kk)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = 16 * kk + 4 * lg + e;
                dn[kk][e] = (rok && k < ndes) ? D[(size_t)k * N + row] : 0.0f;
            }
    };
    load_tile(blockIdx.x * 4 + wave);
    for (int tile = blockIdx.x * 4 + wave; tile < ntiles; tile += stride) {
        const int row = 16 * tile + li;
        const bool rok = row < N;
        const int tr = tn;
        bf16x4 dh[KD / 16], dl[KD / 16];
#pragma unroll
        for (int kk = 0; kk < KD / 16; ++kk) split_bf16(dn[kk], dh[kk], dl[kk]);
        load_tile(tile + stride);
        // ---- forward: Z^T (lane holds Z[row][16 jt + 4 lg + e])
        floatx4 acc[KH / 16];
#pragma unroll
        for (int jt = 0; jt < KH / 16; ++jt) acc[jt] = floatx4{0.f, 0.f, 0.f, 0.f};
        for (int t = 0; t < T; ++t) {
            if (__ballot(tr == t) == 0) continue;
#pragma unroll
            for (int kk = 0; kk < KD / 16; ++kk) {
                const bf16x4 b_h = tr == t ? dh[kk] : zero4, b_l = tr == t ? dl[kk] : zero4;
#pragma unroll
                for (int jt = 0; jt < KH / 16; ++jt) {
                    const int o = (t * KH + 16 * jt + li) * RF + 16 * kk + 4 * lg;
                    const bf16x4 a_h = *reinterpret_cast<const bf16x4 *>(fh + o);
                    const bf16x4 a_l = *reinterpret_cast<const bf16x4 *>(fl + o);
                    acc[jt] = mfma_parts<SPLIT_BOTH>(a_h, a_l, b_h, b_l, acc[jt]);
                }
            }
        }
        // ---- activation and output layers (FP32)
        const int tl = tr < 0 ? 0 : tr;
        float up = 0.f, qp = 0.f;
        bf16x4 geh[KH / 16], gel[KH / 16], gqh[KH / 16], gql[KH / 16];
#pragma unroll
        for (int jt = 0; jt < KH / 16; ++jt) {
            float ge[4], gqq[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int j = 16 * jt + 4 * lg + e;
                const float hh = tanh_fast(acc[jt][e] - sb0[tl][j]);
                const float wE = sw1E[tl][j], wQ = sw1q[tl][j];  // zero for padded j
                up = fmaf(wE, hh, up);
                qp = fmaf(wQ, hh, qp);
                const float dd = 1.0f - hh * hh;
                ge[e] = tr >= 0 ? dd * wE : 0.0f;
                gqq[e] = tr >= 0 ? dd * wQ : 0.0f;
            }
            split_bf16(ge, geh[jt], gel[jt]);
            split_bf16(gqq, gqh[jt], gql[jt]);
        }
        up += __shfl_xor(up, 16, 64);
        up += __shfl_xor(up, 32, 64);
        qp += __shfl_xor(qp, 16, 64);
        qp += __shfl_xor(qp, 32, 64);
        if (rok && lg == 0) {
            const float u = up - b1E, q = qp - sb1q[tl];
            U[row] = u;
            qraw[row] = q;
            red[0] += u;
            red[1] += q;
        }
        // ---- backward: gU^T = sum_t W0_t^T G_t^T (lane holds gU[row][16 vt + 4 lg + e])
        floatx4 gA[KD / 16], gB[KD / 16];
#pragma unroll
        for (int vt = 0; vt < KD / 16; ++vt) gA[vt] = gB[vt] = floatx4{0.f, 0.f, 0.f, 0.f};
        for (int t = 0; t < T; ++t) {
            if (__ballot(tr == t) == 0) continue;
            const bool mine = tr == t;
#pragma unroll
            for (int jj = 0; jj < KH / 16; ++jj) {
                const bf16x4 beh = mine ? geh[jj] : zero4, bel = mine ? gel[jj] : zero4;
                const bf16x4 bqh = mine ? gqh[jj] : zero4, bql = mine ? gql[jj] : zero4;
#pragma unroll
                for (int vt = 0; vt < KD / 16; ++vt) {
                    const int o = (t * KD + 16 * vt + li) * RB + 16 * jj + 4 * lg;
                    const bf16x4 a_h = *reinterpret_cast<const bf16x4 *>(bh + o);
                    const bf16x4 a_l = BLO ? *reinterpret_cast<const bf16x4 *>(bl + o) : zero4;
                    gA[vt] = mfma_parts<BMASK>(a_h, a_l, beh, bel, gA[vt]);
                    gB[vt] = mfma_parts<BMASK>(a_h, a_l, bqh, bql, gB[vt]);
                }
            }
        }
        if (rok) {
#pragma unroll
            for (int vt = 0; vt < KD / 16; ++vt)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int v = 16 * vt + 4 * lg + e;
                    if (v < ndes) {
                        gU[(size_t)v * N + row] = gA[vt][e];
                        gq[(size_t)v * N + row] = gB[vt][e];
                    }
                }
        }
    }
    block_partials<2>(red, partials);
}

static int pad16(int x) { return (x + 15) / 16 * 16; }

bool mlp_bf16_supported(int ndes, int H) {
    int kd = pad16(ndes), kh = pad16(H);
    return (kd == 32 || kd == 48) && (kh == 32 || kh == 48 || kh == 64);
}

template <int KD, int KH, int BMASK>
static hipError_t run_bf16_form(const Plan &p, int G) {
    // BF16 weight parts of the T species: forward rows hi + lo, backward rows hi (+ lo)
    const int nb = (BMASK & SPLIT_A_LO) ? 2 : 1;
    const size_t lds = sizeof(short) * (size_t)p.T * (2 * KH * (KD + 4) + nb * KD * (KH + 4));
    static bool raised = false;
    if (!raised && lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)k_mlp_bf16<KD, KH, BMASK>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        raised = true;
    }
    hipLaunchKernelGGL((k_mlp_bf16<KD, KH, BMASK>), dim3(G), dim3(256), lds, p.stream, p.N, p.T, p.H, p.ndes, p.ts,
                       p.D, p.theta, p.off_nn, p.per_species, p.off_b1E, p.U, p.qraw, p.gU, p.gq, p.partials);
    return hipGetLastError();
}

template <int KD, int KH>
static hipError_t run_bf16(const Plan &p) {
    // two resident work-groups per compute unit, each wave looping over its tiles: the
    // weight staging is paid once per work-group (measured on the 975,560-atom
    // perovskite: 0.215 ms with 2,048 work-groups, 0.18 ms with two per compute unit,
    // 0.21-0.25 ms with 1, 1.5, 2.5 or 3)
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    const int tiles = (p.N + 15) / 16;
    int G = (tiles + 3) / 4;
    if (G > 2 * cus) G = 2 * cus;
    if (G < 1) G = 1;
    hipError_t e = backward_mask(p.mlp_prec) == SPLIT_BOTH ? run_bf16_form<KD, KH, SPLIT_BOTH>(p, G)
                                                           : run_bf16_form<KD, KH, SPLIT_A_LO>(p, G);
    if (e != hipSuccess) return e;
    return reduce_partials(p, G, 2, S_UNEP, false);
}

hipError_t launch_mlp_bf16(const Plan &p) {
    const int kd = pad16(p.ndes), kh = pad16(p.H);
    if (kd == 32 && kh == 32) return run_bf16<32, 32>(p);
    if (kd == 32 && kh == 48) return run_bf16<32, 48>(p);
    if (kd == 32 && kh == 64) return run_bf16<32, 64>(p);
    if (kd == 48 && kh == 32) return run_bf16<48, 32>(p);
    if (kd == 48 && kh == 48) return run_bf16<48, 48>(p);
    if (kd == 48 && kh == 64) return run_bf16<48, 64>(p);
    return hipErrorInvalidValue;
}

}  // namespace qnep
