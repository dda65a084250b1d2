// Reverse mode of the qNEP evaluation for L = gE E + gP . P (the adjoint behind the
// autograd function).  The forward pass is recomputed into the workspace first.
//
//  lambda_i = dL/dq_i  = gE (phi_i - mean phi) + s gP . (r_i - mean r)
//             (exact through the neutrality correction of Eq. 33 and P of Eq. 26)
//  Gamma_i  = dL/dD_i  = gE dU_i/dD + lambda_i dq_i/dD
//  delta_i  = dL/dz_i  = (1 - h^2) (gE w1E + lambda_i w1q)         (z = W0 D - b0, Eq. 1)
//  dL/dW0_t = sum_{i in t} delta_i (x) D_i,  dL/db0_t = -sum delta_i,
//  dL/dw1E_t = gE sum h_i, dL/dw1q_t = sum lambda_i h_i, dL/db1q_t = -sum lambda_i,
//  dL/db1E = -gE N,  dL/ds = -gE Q/(s^2 N) sum_i phi_i + gP . sum_i (q_i - mean q) r_i,
//  dL/dcR[ti][t][n][k] = sum_{i in ti} Gamma_in B_i[t][k]   (B: per-species radial basis sums),
//  dL/dcA[ti][t][n][k] = sum_{i in ti} sum_{j in t} f_k(r_ij) sum_lm 2 Gamma_i,nl A_nlm Y_lm(r_ij),
//  dL/dr_i = -gE F_i + sum_a gP_a Z_i[a][:]   (periodic Born charges, Eq. 28),
//  dL/dh = gE h^{-T} (sum_i F_i (x) r_i - W)^T  (strain identity with W = -dE/d(strain)).
// Parameter sums over atoms are species-masked outer products reduced per chunk of
// atoms in FP32 and across chunks in FP64.
#include <algorithm>

#include "mfma.h"
#include "nep_math.h"
#include "plan.h"

namespace qnep {

// FP64 sums over atoms: sum r (3), sum q_raw r (3), sum F (x) r (9, F_a r_b)
__global__ __launch_bounds__(256) void k_bw_sums(int N, const int *__restrict__ perm, const float *__restrict__ pos,
                                                 const float *__restrict__ qraw, const float *__restrict__ Fout,
                                                 double *__restrict__ partials) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double v[15];
#pragma unroll
    for (int k = 0; k < 15; ++k) v[k] = 0.0;
    if (i < N) {
        const int o = perm[i];
        const double r[3] = {pos[o], pos[(size_t)N + o], pos[(size_t)2 * N + o]};
        const double F[3] = {Fout[o], Fout[(size_t)N + o], Fout[(size_t)2 * N + o]};
        const double q = qraw[i];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a] = r[a];
            v[3 + a] = q * r[a];
#pragma unroll
            for (int b = 0; b < 3; ++b) v[6 + 3 * a + b] = F[a] * r[b];
        }
    }
    block_partials<15>(v, partials);
}

// per-atom adjoints: Xvec = [-delta (H), gE h (H), lambda h (H), -lambda], delta, Gamma
template <int NDES>
__global__ __launch_bounds__(256) void k_bw_atoms(int N, int T, int H, const int *__restrict__ ts,
                                                  const float *__restrict__ D, const float *__restrict__ gU,
                                                  const float *__restrict__ gq, const float *__restrict__ phi,
                                                  const double *__restrict__ scalars, const double *__restrict__ bws,
                                                  const float *__restrict__ theta, int64_t off_nn,
                                                  int64_t per_species, int64_t off_s, const int *__restrict__ perm,
                                                  const float *__restrict__ pos, double gE, double gP0, double gP1,
                                                  double gP2, float *__restrict__ Xvec, float *__restrict__ delta,
                                                  float *__restrict__ Gam) {
    extern __shared__ float wts[];
    const int total = (int)(T * per_species);
    for (int k = threadIdx.x; k < total; k += blockDim.x) wts[k] = theta[off_nn + k];
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int t = ts[i];
    const float *W0 = wts + (size_t)t * per_species;
    const float *b0 = W0 + H * NDES;
    const float *w1E = b0 + H;
    const float *w1q = w1E + H;
    const double s = theta[off_s];
    const int o = perm[i];
    const double rb[3] = {bws[0] / N, bws[1] / N, bws[2] / N};
    const double dr = gP0 * ((double)pos[o] - rb[0]) + gP1 * ((double)pos[(size_t)N + o] - rb[1]) +
                      gP2 * ((double)pos[(size_t)2 * N + o] - rb[2]);
    const float lam = (float)(gE * ((double)phi[i] - scalars[S_PHIBAR]) + s * dr);
    const float ge = (float)gE;
    float d[NDES];
#pragma unroll
    for (int v = 0; v < NDES; ++v) {
        d[v] = D[(size_t)v * N + i];
        Gam[(size_t)v * N + i] = fmaf(lam, gq[(size_t)v * N + i], ge * gU[(size_t)v * N + i]);
    }
    for (int mu = 0; mu < H; ++mu) {
        const float *row = W0 + mu * NDES;
        float z = -b0[mu];
#pragma unroll
        for (int v = 0; v < NDES; ++v) z = fmaf(row[v], d[v], z);
        const float h = tanhf(z);
        const float dl = (1.0f - h * h) * fmaf(lam, w1q[mu], ge * w1E[mu]);
        delta[(size_t)mu * N + i] = dl;
        Xvec[(size_t)mu * N + i] = -dl;
        Xvec[(size_t)(H + mu) * N + i] = ge * h;
        Xvec[(size_t)(2 * H + mu) * N + i] = lam * h;
    }
    Xvec[(size_t)(3 * H) * N + i] = -lam;
}

// per-atom angular coefficient adjoint Gc[tp][n][k] = sum_{j in A(i), tj = tp} f_k(r_ij) P_n(j),
// P_n = sum_lm 2 Gamma_i,nl A_nlm Y_lm(r_ij); one pass per neighbour species
template <int T, int NR, int NA, int NB>
__global__ __launch_bounds__(256) void k_bw_angular(int N, const float4 *__restrict__ xyzt, Cell c, float rcA,
                                                    const uint32_t *__restrict__ listA, const int *__restrict__ cntA,
                                                    int capA, const float *__restrict__ Amom,
                                                    const float *__restrict__ Gam, float *__restrict__ Gc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float4 pi = xyzt[i];
    float At[NA][LM];
#pragma unroll
    for (int n = 0; n < NA; ++n) {
        float G[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) G[l] = 2.0f * Gam[(size_t)(NR + l * NA + n) * N + i];
#pragma unroll
        for (int q = 0; q < LM; ++q) {
            const int l = q < 3 ? 0 : (q < 8 ? 1 : (q < 15 ? 2 : 3));
            At[n][q] = G[l] * Amom[(size_t)(n * LM + q) * N + i];
        }
    }
    const int nA = cntA[i];
    for (int tp = 0; tp < T; ++tp) {
        float acc[NA][NB];
#pragma unroll
        for (int n = 0; n < NA; ++n)
#pragma unroll
            for (int k = 0; k < NB; ++k) acc[n][k] = 0.f;
        for (int sl = 0; sl < nA; ++sl) {
            const uint32_t e = listA[(size_t)i * capA + sl];
            const float4 pj = xyzt[nb_index(e)];
            if (species_of(pj) != tp) continue;
            const float3 d = pair_displacement(pi, pj, e, c);
            const float r = sqrtf(d.x * d.x + d.y * d.y + d.z * d.z);
            const float ir = 1.0f / r;
            float f[NB], df[NB];
            cheb_basis<NB>(r, rcA, f, df);
            float Y[LM];
            harmonics(d.x * ir, d.y * ir, d.z * ir, Y);
#pragma unroll
            for (int n = 0; n < NA; ++n) {
                float Pn = 0.f;
#pragma unroll
                for (int q = 0; q < LM; ++q) Pn = fmaf(At[n][q], Y[q], Pn);
#pragma unroll
                for (int k = 0; k < NB; ++k) acc[n][k] = fmaf(Pn, f[k], acc[n][k]);
            }
        }
#pragma unroll
        for (int n = 0; n < NA; ++n)
#pragma unroll
            for (int k = 0; k < NB; ++k) Gc[(size_t)((tp * NA + n) * NB + k) * N + i] = acc[n][k];
    }
}

// Species-masked outer-product sums on the matrix cores (v_mfma_f32_16x16x4f32):
//   partials[blk][t][a][b] = sum over the atoms i of chunk blk with ts_i = t of X[a][i] Y[b][i]
// (Y = null: ones).  Per chunk this is the product X [A x K] Ym [K x T B] with
// Ym[i][t B + b] = Y[b][i] [ts_i = t]; the mask is applied while forming the B operand.
// Each wave owns up to MO_TPW output tiles of 16 x 16; a K tile of MO_KT atoms is staged
// in LDS for the whole work-group.  FP32 accumulation within a chunk, FP64 across chunks.
constexpr int MO_KT = 64, MO_LD = MO_KT + 1, MO_TPW = 8, MO_WAVES = 4;

// rows [0, R) of atoms [b0, b0 + nv) of a [R][N] array into LDS rows of stride MO_LD,
// zero past nv; MO_BATCH loads per thread are issued before their LDS stores (src = null:
// the constant fill)
constexpr int MO_BATCH = 8;
__device__ inline void stage_rows(float *dst, const float *__restrict__ src, int R, int N, int b0, int nv, float fill) {
    for (int base = threadIdx.x; base < R * MO_KT; base += MO_BATCH * 256) {
        float v[MO_BATCH];
#pragma unroll
        for (int j = 0; j < MO_BATCH; ++j) {
            const int idx = base + j * 256, r = idx / MO_KT, u = idx % MO_KT;
            v[j] = (idx < R * MO_KT && u < nv) ? (src ? src[(size_t)r * N + b0 + u] : fill) : 0.f;
        }
#pragma unroll
        for (int j = 0; j < MO_BATCH; ++j) {
            const int idx = base + j * 256;
            if (idx < R * MO_KT) dst[(idx / MO_KT) * MO_LD + idx % MO_KT] = v[j];
        }
    }
}

// Work-group (x, y) takes atom chunk x and output tiles [y tpb, (y + 1) tpb); wave w of it
// takes the tiles y tpb + w + MO_WAVES s, s < TPW.
template <int TPW>
__global__ __launch_bounds__(256) void k_masked_outer(int N, int T, int A, int B, int chunk, int tpb,
                                                      const float *__restrict__ X, const float *__restrict__ Y,
                                                      const int *__restrict__ ts, double *__restrict__ partials) {
    // LDS: X rows 0..A-1 and a zero row A, Y rows 0..B-1 and a zero row B, the species
    // of the staged atoms; padding rows, columns and tiles read the zero rows, so the
    // product loop has no branches
    extern __shared__ float sm[];
    float *sX = sm, *sY = sm + (A + 1) * MO_LD;
    int *st = reinterpret_cast<int *>(sY + (B + 1) * MO_LD);
    const int C = T * B, MC = (C + 15) / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i16 = lane & 15, k4 = lane >> 4;
    const int a0 = blockIdx.x * chunk, a1 = min(N, a0 + chunk);
    const int t_lo = blockIdx.y * tpb, t_hi = t_lo + tpb;
    for (int u = threadIdx.x; u < MO_KT; u += blockDim.x) {
        sX[A * MO_LD + u] = 0.f;
        sY[B * MO_LD + u] = 0.f;
    }
    // per tile: LDS offsets of the A-operand row and the B-operand row of this lane, and
    // the species its column belongs to (-2: padding)
    int xo[TPW], yo[TPW], tc[TPW];
    floatx4 acc[TPW];
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        acc[s] = floatx4{0.f, 0.f, 0.f, 0.f};
        const int tile = t_lo + wave + MO_WAVES * s;
        const bool ok = tile < t_hi;
        const int ra = (tile / MC) * 16 + i16, cc = (tile % MC) * 16 + i16;
        xo[s] = (ok && ra < A ? ra : A) * MO_LD;
        const int t = cc / B;
        const bool okc = ok && cc < C;
        tc[s] = okc ? t : -2;
        yo[s] = (okc ? cc - t * B : B) * MO_LD;
    }
    for (int b0 = a0; b0 < a1; b0 += MO_KT) {
        const int nv = min(MO_KT, a1 - b0);
        stage_rows(sX, X, A, N, b0, nv, 0.f);
        if (Y) stage_rows(sY, Y, B, N, b0, nv, 0.f);
        else stage_rows(sY, (const float *)nullptr, B, N, b0, nv, 1.0f);
        for (int u = threadIdx.x; u < MO_KT; u += blockDim.x) st[u] = u < nv ? ts[b0 + u] : -1;
        __syncthreads();
        for (int kk = 0; kk < MO_KT; kk += 4) {
            const int u = kk + k4;
            const int tu = st[u];
            float av[TPW], bv[TPW];
#pragma unroll
            for (int s = 0; s < TPW; ++s) {
                av[s] = sX[xo[s] + u];
                bv[s] = sY[yo[s] + u];
            }
#pragma unroll
            for (int s = 0; s < TPW; ++s)
                acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], tc[s] == tu ? bv[s] : 0.f, acc[s], 0, 0, 0);
        }
        __syncthreads();
    }
    // D[i][j] sits in lane j + 16 (i / 4), element i % 4
    double *out = partials + (size_t)blockIdx.x * C * A;
    const int tiles = ((A + 15) / 16) * MC;
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        const int tile = t_lo + wave + MO_WAVES * s;
        if (tile >= t_hi || tile >= tiles) continue;
        const int col = (tile % MC) * 16 + i16;
        if (col >= C) continue;
        const int t = col / B, b = col - t * B;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = (tile / MC) * 16 + 4 * k4 + e;
            if (row < A) out[((size_t)t * A + row) * B + b] = acc[s][e];
        }
    }
}

// fixed-order sum over blocks: dst[k] = sum_b partials[b][k]; 16 strided partial sums
// per output, combined in index order
__global__ __launch_bounds__(256) void k_sum_blocks(const double *__restrict__ partials, int nblk, int nv,
                                                    double *__restrict__ dst) {
    __shared__ double red[16][17];
    const int kl = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int k = blockIdx.x * 16 + kl;
    double s = 0.0;
    if (k < nv) {
#pragma unroll 4
        for (int b = g; b < nblk; b += 16) s += partials[(size_t)b * nv + k];
    }
    red[g][kl] = s;
    __syncthreads();
    if (g == 0 && k < nv) {
        double t = 0.0;
        for (int j = 0; j < 16; ++j) t += red[j][kl];
        dst[k] = t;
    }
}

struct BwLayout {
    int T, NR, NA, NBR, NBA, H, ndes;
    int64_t off_cA, off_nn, per_species, off_b1E, off_s, n_theta;
};

// d_theta in the parameter layout from the FP64 staging sums
__global__ void k_bw_theta(BwLayout L, int N, double gE, double gP0, double gP1, double gP2, double qtot,
                           const float *__restrict__ theta, const double *__restrict__ scalars,
                           const double *__restrict__ bws, const double *__restrict__ sW0,
                           const double *__restrict__ sVec, const double *__restrict__ sCR,
                           const double *__restrict__ sCA, float *__restrict__ dtheta) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= L.n_theta) return;
    double v = 0.0;
    const int T = L.T;
    if (idx < L.off_cA) {  // cR[ti][tj][n][k]  <- sCR[ti][n][tj NB + k]
        int r = (int)idx;
        const int k = r % L.NBR;
        r /= L.NBR;
        const int n = r % L.NR;
        r /= L.NR;
        const int tj = r % T, ti = r / T;
        v = sCR[((size_t)ti * L.NR + n) * (T * L.NBR) + tj * L.NBR + k];
    } else if (idx < L.off_nn) {  // cA[ti][tj][n][k]  <- sCA[ti][(tj NA + n) NB + k]
        int r = (int)(idx - L.off_cA);
        const int k = r % L.NBA;
        r /= L.NBA;
        const int n = r % L.NA;
        r /= L.NA;
        const int tj = r % T, ti = r / T;
        v = sCA[(size_t)ti * (T * L.NA * L.NBA) + (tj * L.NA + n) * L.NBA + k];
    } else if (idx < L.off_b1E) {
        const int64_t r = idx - L.off_nn;
        const int t = (int)(r / L.per_species);
        const int q = (int)(r % L.per_species);
        const int H = L.H, nd = L.ndes;
        if (q < H * nd) v = sW0[(size_t)t * H * nd + q];
        else v = sVec[(size_t)t * (3 * H + 1) + (q - H * nd)];  // b0, w1E, w1q, b1q in Xvec order
    } else if (idx == L.off_b1E) {
        v = -gE * N;
    } else {  // s
        const double s = theta[L.off_s];
        const double qbar = scalars[S_SUMQ] / N;
        v = -gE * qtot / (s * s * N) * scalars[S_SUMPHI];
        v += gP0 * (bws[3] - qbar * bws[0]) + gP1 * (bws[4] - qbar * bws[1]) + gP2 * (bws[5] - qbar * bws[2]);
    }
    dtheta[idx] = (float)v;
}

__global__ void k_bw_positions(int N, double gE, double gP0, double gP1, double gP2, const float *__restrict__ Fout,
                               const float *__restrict__ Zout, float *__restrict__ dpos) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= N) return;
    const double gP[3] = {gP0, gP1, gP2};
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        double v = -gE * (double)Fout[(size_t)b * N + o];
#pragma unroll
        for (int a = 0; a < 3; ++a) v += gP[a] * (double)Zout[(size_t)(3 * a + b) * N + o];
        dpos[(size_t)b * N + o] = (float)v;
    }
}

__global__ void k_bw_cell(Cell c, double gE, const double *__restrict__ virial, const double *__restrict__ bws,
                          double *__restrict__ dcell) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double M[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[3 * a + b] = -virial[3 * a + b] + bws[6 + 3 * a + b];
    // G_{a alpha} = sum_beta M[alpha][beta] hinv[beta][a]
    for (int a = 0; a < 3; ++a)
        for (int al = 0; al < 3; ++al) {
            double g = 0.0;
            for (int be = 0; be < 3; ++be) g += M[3 * al + be] * c.hinv[3 * be + a];
            dcell[3 * a + al] = gE * g;
        }
}

template <int T, int NR, int NA, int NB>
static hipError_t run_bw_angular(const Plan &p) {
    const int G = (p.N + 255) / 256;
    hipLaunchKernelGGL((k_bw_angular<T, NR, NA, NB>), dim3(G), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell,
                       (float)p.rcA, p.listA, p.cntA, p.capA, p.Amom, p.bw.Gam, p.bw.Gc);
    return hipGetLastError();
}

#define QNEP_DISPATCH_BW(FN)                                                                               \
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

static hipError_t launch_bw_angular(const Plan &p) { QNEP_DISPATCH_BW(run_bw_angular) }

// atom chunks of the species-masked parameter sums (one FP64 partial row per chunk)
int masked_outer_chunks(int N) { return N <= 0 ? 1 : std::min((N + 127) / 128, 512); }

template <int TPW>
static void launch_masked_outer(const Plan &p, dim3 grid, size_t lds, int A, int B, int chunk, int tpb, const float *X,
                                const float *Y) {
    hipLaunchKernelGGL(k_masked_outer<TPW>, grid, dim3(256), lds, p.stream, p.N, p.T, A, B, chunk, tpb, X, Y, p.ts,
                       p.bw.partials);
}

static hipError_t masked_outer(const Plan &p, int A, int B, const float *X, const float *Y, double *dst) {
    const int nblk = masked_outer_chunks(p.N);
    const int chunk = (p.N + nblk - 1) / nblk;
    const int tiles = ((A + 15) / 16) * ((p.T * B + 15) / 16);
    const int gy = (tiles + MO_WAVES * MO_TPW - 1) / (MO_WAVES * MO_TPW);
    const int tpb = (tiles + gy - 1) / gy;           // tiles per work-group, balanced over y
    const int tpw = (tpb + MO_WAVES - 1) / MO_WAVES;  // tiles per wave, at most MO_TPW
    const int nv = p.T * A * B;
    const size_t lds = sizeof(float) * (size_t)(A + B + 2) * MO_LD + sizeof(int) * MO_KT;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const dim3 grid(nblk, gy);
    switch (tpw) {
        case 1: launch_masked_outer<1>(p, grid, lds, A, B, chunk, tpb, X, Y); break;
        case 2: launch_masked_outer<2>(p, grid, lds, A, B, chunk, tpb, X, Y); break;
        case 3: launch_masked_outer<3>(p, grid, lds, A, B, chunk, tpb, X, Y); break;
        case 4: launch_masked_outer<4>(p, grid, lds, A, B, chunk, tpb, X, Y); break;
        case 5: launch_masked_outer<5>(p, grid, lds, A, B, chunk, tpb, X, Y); break;
        case 6: launch_masked_outer<6>(p, grid, lds, A, B, chunk, tpb, X, Y); break;
        case 7: launch_masked_outer<7>(p, grid, lds, A, B, chunk, tpb, X, Y); break;
        default: launch_masked_outer<8>(p, grid, lds, A, B, chunk, tpb, X, Y); break;
    }
    hipLaunchKernelGGL(k_sum_blocks, dim3((nv + 15) / 16), dim3(256), 0, p.stream, p.bw.partials, nblk, nv, dst);
    return hipGetLastError();
}

hipError_t launch_backward(const Plan &p) {
    const Backward &b = p.bw;
    const int G = (p.N + 255) / 256;
    hipLaunchKernelGGL(k_bw_sums, dim3(G), dim3(256), 0, p.stream, p.N, p.perm, p.pos, p.qraw, b.Fout, p.partials);
    hipError_t e = reduce_partials_to(p, G, 15, b.sums);
    if (e != hipSuccess) return e;
    const size_t lds = sizeof(float) * (size_t)(p.T * p.per_species);
    if (p.ndes == 25)
        hipLaunchKernelGGL(k_bw_atoms<25>, dim3(G), dim3(256), lds, p.stream, p.N, p.T, p.H, p.ts, p.D, p.gU, p.gq,
                           p.phi, p.scalars, b.sums, p.theta, p.off_nn, p.per_species, p.off_s, p.perm, p.pos, b.gE,
                           b.gP[0], b.gP[1], b.gP[2], b.Xvec, b.delta, b.Gam);
    else if (p.ndes == 37)
        hipLaunchKernelGGL(k_bw_atoms<37>, dim3(G), dim3(256), lds, p.stream, p.N, p.T, p.H, p.ts, p.D, p.gU, p.gq,
                           p.phi, p.scalars, b.sums, p.theta, p.off_nn, p.per_species, p.off_s, p.perm, p.pos, b.gE,
                           b.gP[0], b.gP[1], b.gP[2], b.Xvec, b.delta, b.Gam);
    else
        return hipErrorInvalidValue;
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (b.dtheta) {
        e = launch_bw_angular(p);
        if (e != hipSuccess) return e;
        e = masked_outer(p, p.H, p.ndes, b.delta, p.D, b.sW0);
        if (e != hipSuccess) return e;
        e = masked_outer(p, 3 * p.H + 1, 1, b.Xvec, nullptr, b.sVec);
        if (e != hipSuccess) return e;
        e = masked_outer(p, p.NR, p.T * p.NBR, b.Gam, p.Bsum, b.sCR);
        if (e != hipSuccess) return e;
        e = masked_outer(p, p.T * p.NA * p.NBA, 1, b.Gc, nullptr, b.sCA);
        if (e != hipSuccess) return e;
        BwLayout L{p.T, p.NR, p.NA, p.NBR, p.NBA, p.H, p.ndes, p.off_cA, p.off_nn, p.per_species, p.off_b1E,
                   p.off_s, p.n_theta};
        hipLaunchKernelGGL(k_bw_theta, dim3((unsigned)((p.n_theta + 255) / 256)), dim3(256), 0, p.stream, L, p.N,
                           b.gE, b.gP[0], b.gP[1], b.gP[2], p.qtot, p.theta, p.scalars, b.sums, b.sW0, b.sVec, b.sCR,
                           b.sCA, b.dtheta);
    }
    if (b.dpos)
        hipLaunchKernelGGL(k_bw_positions, dim3(G), dim3(256), 0, p.stream, p.N, b.gE, b.gP[0], b.gP[1], b.gP[2],
                           b.Fout, b.Zout, b.dpos);
    if (b.dcell)
        hipLaunchKernelGGL(k_bw_cell, dim3(1), dim3(64), 0, p.stream, p.cell, b.gE, b.virial, b.sums, b.dcell);
    return hipGetLastError();
}

}  // namespace qnep
