// BF16 matrix-core forms of the per-species network (Sec. 2.1 Eq. 1, Sec. 2.2):
//   Z = D W0_t^T, h = tanh(Z - b0_t), U = w1E_t . h - b1E, q = w1q_t . h - b1q_t,
//   dU/dD = [(1 - h^2) w1E_t] W0_t, dq/dD = [(1 - h^2) w1q_t] W0_t.
// One wave computes a tile of 16 consecutive (spatially sorted) atoms with
// v_mfma_f32_16x16x16_bf16 (BF16 inputs, FP32 accumulation).  Atoms of different
// species share a tile: for every species t the A-operand rows of other species are
// zeroed, so sum_t A_t W0_t gives each row its own species' product.  tanh and the
// output layers stay in FP32.
#include "mfma.h"
#include "plan.h"

namespace qnep {

template <int KD, int KH, int NSPLIT>
__global__ __launch_bounds__(256) void k_mlp_bf16(int N, int T, int H, int ndes, const int *__restrict__ ts,
                                                  const float *__restrict__ D, const float *__restrict__ theta,
                                                  int64_t off_nn, int64_t per_species, int64_t off_b1E,
                                                  float *__restrict__ U, float *__restrict__ qraw,
                                                  float *__restrict__ gU, float *__restrict__ gq,
                                                  double *__restrict__ partials) {
    __shared__ float sW0[KH][KD];  // W0_t[j][k] of the species being processed, zero padded
    __shared__ float sb0[MAX_T][KH], sw1E[MAX_T][KH], sw1q[MAX_T][KH], sb1q[MAX_T];
    __shared__ float sG[4][2][16][KH];  // per wave: (1-h^2) w1E and (1-h^2) w1q, rows = atoms
    for (int idx = threadIdx.x; idx < T * KH; idx += blockDim.x) {
        int t = idx / KH, j = idx % KH;
        const float *base = theta + off_nn + t * per_species + (int64_t)H * ndes;
        sb0[t][j] = j < H ? base[j] : 0.0f;
        sw1E[t][j] = j < H ? base[H + j] : 0.0f;
        sw1q[t][j] = j < H ? base[2 * H + j] : 0.0f;
        if (j == 0) sb1q[t] = base[3 * H];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int base = (blockIdx.x * 4 + wave) * 16;
    const int li = lane & 15, lg = lane >> 4;
    const int arow = base + li;  // this lane's A-operand row
    const int at = arow < N ? ts[arow] : -1;
    float dv[KD / 16][4];
#pragma unroll
    for (int kk = 0; kk < KD / 16; ++kk)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int k = 16 * kk + 4 * lg + e;
            dv[kk][e] = (arow < N && k < ndes) ? D[(size_t)k * N + arow] : 0.0f;
        }
    // ---- forward: Z = sum_t A_t W0_t^T
    floatx4 acc[KH / 16];
#pragma unroll
    for (int nt = 0; nt < KH / 16; ++nt) acc[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < T; ++t) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < KH * KD; idx += blockDim.x) {
            int j = idx / KD, k = idx % KD;
            sW0[j][k] = (j < H && k < ndes) ? theta[off_nn + t * per_species + (int64_t)j * ndes + k] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KD / 16; ++kk) {
            float a[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) a[e] = (at == t) ? dv[kk][e] : 0.0f;
#pragma unroll
            for (int nt = 0; nt < KH / 16; ++nt) {
                float b[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) b[e] = sW0[16 * nt + li][16 * kk + 4 * lg + e];
                acc[nt] = mfma_split<NSPLIT>(a, b, acc[nt]);
            }
        }
    }
    // ---- activation and output layers (FP32); D layout: row 4 lg + e, column 16 nt + li
    float up[4] = {0.f, 0.f, 0.f, 0.f}, qp[4] = {0.f, 0.f, 0.f, 0.f};
    int rt[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        int row = base + 4 * lg + e;
        rt[e] = row < N ? ts[row] : 0;
    }
#pragma unroll
    for (int nt = 0; nt < KH / 16; ++nt) {
        const int j = 16 * nt + li;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int t = rt[e];
            float h = tanhf(acc[nt][e] - sb0[t][j]);
            float wE = sw1E[t][j], wQ = sw1q[t][j];  // zero for padded j
            up[e] = fmaf(wE, h, up[e]);
            qp[e] = fmaf(wQ, h, qp[e]);
            float dh = 1.0f - h * h;
            sG[wave][0][4 * lg + e][j] = wE * dh;
            sG[wave][1][4 * lg + e][j] = wQ * dh;
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {
            up[e] += __shfl_xor(up[e], o, 64);
            qp[e] += __shfl_xor(qp[e], o, 64);
        }
    double red[2] = {0.0, 0.0};
    if (li == 0) {
        const float b1E = theta[off_b1E];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int row = base + 4 * lg + e;
            if (row < N) {
                float u = up[e] - b1E, q = qp[e] - sb1q[rt[e]];
                U[row] = u;
                qraw[row] = q;
                red[0] += u;
                red[1] += q;
            }
        }
    }
    // ---- backward: gU = sum_t G_t W0_t (rows of other species zeroed)
    floatx4 aE[KD / 16], aQ[KD / 16];
#pragma unroll
    for (int vt = 0; vt < KD / 16; ++vt) {
        aE[vt] = floatx4{0.f, 0.f, 0.f, 0.f};
        aQ[vt] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    for (int t = 0; t < T; ++t) {
        __syncthreads();  // also orders the sG writes above before their reads
        for (int idx = threadIdx.x; idx < KH * KD; idx += blockDim.x) {
            int j = idx / KD, k = idx % KD;
            sW0[j][k] = (j < H && k < ndes) ? theta[off_nn + t * per_species + (int64_t)j * ndes + k] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < KH / 16; ++jj) {
            float ge[4], gqv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int j = 16 * jj + 4 * lg + e;
                ge[e] = (at == t) ? sG[wave][0][li][j] : 0.0f;
                gqv[e] = (at == t) ? sG[wave][1][li][j] : 0.0f;
            }
#pragma unroll
            for (int vt = 0; vt < KD / 16; ++vt) {
                float b[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) b[e] = sW0[16 * jj + 4 * lg + e][16 * vt + li];
                aE[vt] = mfma_split<NSPLIT>(ge, b, aE[vt]);
                aQ[vt] = mfma_split<NSPLIT>(gqv, b, aQ[vt]);
            }
        }
    }
#pragma unroll
    for (int vt = 0; vt < KD / 16; ++vt) {
        const int v = 16 * vt + li;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int row = base + 4 * lg + e;
            if (row < N && v < ndes) {
                gU[(size_t)v * N + row] = aE[vt][e];
                gq[(size_t)v * N + row] = aQ[vt][e];
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

template <int KD, int KH>
static hipError_t run_bf16(const Plan &p) {
    const int tiles = (p.N + 15) / 16;
    const int G = (tiles + 3) / 4;
    if (p.mlp_prec == QNEP_MLP_BF16X3)
        hipLaunchKernelGGL((k_mlp_bf16<KD, KH, 3>), dim3(G), dim3(256), 0, p.stream, p.N, p.T, p.H, p.ndes, p.ts,
                           p.D, p.theta, p.off_nn, p.per_species, p.off_b1E, p.U, p.qraw, p.gU, p.gq, p.partials);
    else
        hipLaunchKernelGGL((k_mlp_bf16<KD, KH, 1>), dim3(G), dim3(256), 0, p.stream, p.N, p.T, p.H, p.ndes, p.ts, p.D,
                       p.theta, p.off_nn, p.per_species, p.off_b1E, p.U, p.qraw, p.gU, p.gq, p.partials);
    hipError_t e = hipGetLastError();
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
