// PPPM reciprocal part (Sec. 2.6):
//   charge assignment with the order-5 B-spline W (Eq. 35), forward FFT to S(k),
//   optimized influence function G_opt = G [prod sinc^5]^2 / [prod poly(z)]^2 (Eq. 36,
//   with the denominator squared and the z^6 coefficient -17/189, the value of the
//   P = 5 alias sum), energy k_e sum G_opt |S|^2 (Eq. 34) and virial k_e sum G_opt |S|^2 B
//   (B as in Eq. 21), ik differentiation for the static force (Eq. 37) and the
//   potential mesh for the dynamic-charge force (Eq. 38), gathered with the same W.
// Two packed complex inverse transforms, interleaved per mesh point and run through
// the same launches, give (E_z + i phi) and (E_x + i E_y).
#include "fft256.h"
#include "plan.h"

namespace qnep {

// order-5 weights of the mesh points m0 - 2 .. m0 + 2 for dx = u - m0 in [-1/2, 1/2]
__host__ __device__ inline void bspline5(float x, float *w) {
    const float x2 = x * x;
    const float a = 1.0f - 2.0f * x, b = 1.0f + 2.0f * x;
    w[0] = (a * a) * (a * a) * (1.0f / 384.0f);
    w[1] = (19.0f - 44.0f * x + 24.0f * x2 + 16.0f * x2 * x - 16.0f * x2 * x2) * (1.0f / 96.0f);
    w[2] = (115.0f - 120.0f * x2 + 48.0f * x2 * x2) * (1.0f / 192.0f);
    w[3] = (19.0f + 44.0f * x + 24.0f * x2 - 16.0f * x2 * x - 16.0f * x2 * x2) * (1.0f / 96.0f);
    w[4] = (b * b) * (b * b) * (1.0f / 384.0f);
}

struct MeshGeom {
    int n[3];
};

__device__ inline void mesh_stencil(float x, float y, float z, const Cell &c, const MeshGeom &g, int *m0,
                                    float (*w)[5]) {
    double s[3];
    s[0] = (double)x * c.hinv[0] + (double)y * c.hinv[3] + (double)z * c.hinv[6];
    s[1] = (double)x * c.hinv[1] + (double)y * c.hinv[4] + (double)z * c.hinv[7];
    s[2] = (double)x * c.hinv[2] + (double)y * c.hinv[5] + (double)z * c.hinv[8];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double sa = s[a] - floor(s[a]);
        double u = sa * g.n[a];
        double m = floor(u + 0.5);
        m0[a] = (int)m;
        bspline5((float)(u - m), w[a]);
    }
}

// j mod n in [0, n); stencil indices lie within one period of the mesh (n >= 3), which
// takes two comparisons instead of an integer division by a run-time value
__device__ inline int wrap_index(int j, int n) {
    if (j >= -n && j < 2 * n) return j < 0 ? j + n : (j >= n ? j - n : j);
    j %= n;
    return j < 0 ? j + n : j;
}

// float offset of mesh point (j0, j1, j2) in the input of the real-input transform:
// lines j1 = 2p and 2p + 1 interleaved, (x[j0][2p][m], x[j0][2p+1][m]) one complex element
__device__ inline size_t pair_index(int j0, int j1, int j2, const MeshGeom &g) {
    return ((size_t)j0 * g.n[1] + (j1 & ~1)) * g.n[2] + 2 * (size_t)j2 + (j1 & 1);
}

// pairs = 1: rho in the interleaved layout of pair_index
__global__ __launch_bounds__(256) void k_spread(int N, const float4 *__restrict__ xyzt, Cell c, MeshGeom g,
                                                const float *__restrict__ qraw, const double *__restrict__ scalars,
                                                float *__restrict__ rho, int pairs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float q = qraw[i] + (float)scalars[S_DELTA];
    int m0[3];
    float w[3][5];
    const float4 pa = xyzt[i];
    mesh_stencil(pa.x, pa.y, pa.z, c, g, m0, w);
    int j0[5], j1[5], j2[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        j0[t] = wrap_index(m0[0] + t - 2, g.n[0]);
        j1[t] = wrap_index(m0[1] + t - 2, g.n[1]);
        j2[t] = wrap_index(m0[2] + t - 2, g.n[2]);
    }
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        const float qa = q * w[0][a];
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            const float qab = qa * w[1][b];
            if (pairs) {
#pragma unroll
                for (int e = 0; e < 5; ++e) atomicAdd(&rho[pair_index(j0[a], j1[b], j2[e], g)], qab * w[2][e]);
            } else {
                const size_t row = ((size_t)j0[a] * g.n[1] + j1[b]) * g.n[2];
#pragma unroll
                for (int e = 0; e < 5; ++e) atomicAdd(&rho[row + j2[e]], qab * w[2][e]);
            }
        }
    }
}

__global__ void k_real_to_complex(int64_t M, const float *__restrict__ rho, float2 *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) out[i] = make_float2(rho[i], 0.0f);
}

// ---------------------------------------------------------------- brick spread
// Charge assignment without global atomics.  A work-group owns a brick of mesh
// points and collects from the cell list every atom copy whose order-5 stencil can
// reach the brick: the bins (unwrapped, so periodic images are explicit) whose atoms
// have u in [M0 - 5/2, M0 + P + 3/2) in mesh units, read as rows along c split per
// image.  Each copy adds the part of its stencil inside the brick to an LDS tile,
// and the brick is stored once as the FFT input (the real mesh with pairs of lines
// interleaved for the real-input transform, else (rho, 0)): every mesh point is
// written by exactly one work-group.  Positions are taken unwrapped (the sorted
// copies lie in the cell up to rounding), so a copy sits next to the bin it is
// listed in.
constexpr int SB_P = 16;      // largest brick edge (mesh points)
constexpr int SB_ROWS = 256;  // rows of bins per brick (one per thread)
constexpr int SB_SEGS = 512;  // segments (row x image along c) per brick
// Contributions are added to the LDS tile in 64-bit fixed point (to_fixed): the mesh
// does not depend on the order of the additions.

__device__ inline int sb_code(int k0, int k1, int k2) { return (k0 + 128) | (k1 + 128) << 8 | (k2 + 128) << 16; }

// exclusive scan of (x, y) over the 256 threads of a work-group; totals in tx, ty
__device__ inline void sb_exscan2(int &x, int &y, int &tx, int &ty) {
    __shared__ int ws[2][4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int ix = x, iy = y;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int vx = __shfl_up(ix, o, 64), vy = __shfl_up(iy, o, 64);
        if (lane >= o) {
            ix += vx;
            iy += vy;
        }
    }
    if (lane == 63) {
        ws[0][wid] = ix;
        ws[1][wid] = iy;
    }
    __syncthreads();
    int bx = 0, by = 0;
    for (int w = 0; w < wid; ++w) {
        bx += ws[0][w];
        by += ws[1][w];
    }
    tx = ws[0][0] + ws[0][1] + ws[0][2] + ws[0][3];
    ty = ws[1][0] + ws[1][1] + ws[1][2] + ws[1][3];
    x = bx + ix - x;
    y = by + iy - y;
}

__global__ __launch_bounds__(256) void k_spread_bricks(const float4 *__restrict__ xyzt, Cell c, MeshGeom g,
                                                       int nc0, int nc1, int nc2, BrickGeom bg,
                                                       const int *__restrict__ start, const float *__restrict__ qraw,
                                                       const double *__restrict__ scalars, float2 *__restrict__ out,
                                                       int real_out) {
    __shared__ unsigned long long tile[SB_P * SB_P * SB_P];  // fixed point
    __shared__ int sbeg[SB_SEGS], spre[SB_SEGS + 1], scode[SB_SEGS];
    const int nc[3] = {nc0, nc1, nc2};
    const int br = xcd_block();
    const int bi[3] = {br / (bg.nb[1] * bg.nb[2]), (br / bg.nb[2]) % bg.nb[1], br % bg.nb[2]};
    int M0[3], Pa[3], blo[3], bhi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        M0[a] = bi[a] * bg.P[a];
        Pa[a] = min(bg.P[a], g.n[a] - M0[a]);
        blo[a] = (int)floor((M0[a] - 2.51) * nc[a] / g.n[a]);
        bhi[a] = (int)floor((M0[a] + Pa[a] + 1.51) * nc[a] / g.n[a]);
    }
    const int TP = bg.P[0] * bg.P[1] * bg.P[2];
    for (int p = threadIdx.x; p < TP; p += blockDim.x) tile[p] = 0ull;
    // one row of bins (x, y fixed) per thread: count its segments and atoms
    const int ny = bhi[1] - blo[1] + 1, nrows = (bhi[0] - blo[0] + 1) * ny;
    const int r = threadIdx.x;
    const bool has_row = r < nrows;
    int i0 = 0, i1 = 0, rowbase = 0;
    if (has_row) {
        const int u0 = blo[0] + r / ny, u1 = blo[1] + r % ny;
        i0 = floor_div(u0, nc0);
        i1 = floor_div(u1, nc1);
        rowbase = row_rank(u0 - i0 * nc0, u1 - i1 * nc1, nc0, nc1) * nc2;
    }
    const int z0 = floor_div(blo[2], nc2), z1 = floor_div(bhi[2], nc2);
    int nseg = 0, nat = 0;
    for (int i2 = z0; has_row && i2 <= z1; ++i2) {
        const int za = max(blo[2], i2 * nc2) - i2 * nc2, zb = min(bhi[2], i2 * nc2 + nc2 - 1) - i2 * nc2;
        ++nseg;
        nat += start[rowbase + zb + 1] - start[rowbase + za];
    }
    int tseg, tat;
    sb_exscan2(nseg, nat, tseg, tat);  // nseg, nat become this row's offsets
    for (int i2 = z0; has_row && i2 <= z1; ++i2) {
        const int za = max(blo[2], i2 * nc2) - i2 * nc2, zb = min(bhi[2], i2 * nc2 + nc2 - 1) - i2 * nc2;
        const int jb = start[rowbase + za];
        sbeg[nseg] = jb;
        spre[nseg] = nat;
        scode[nseg] = sb_code(i0, i1, i2);
        ++nseg;
        nat += start[rowbase + zb + 1] - jb;
    }
    if (threadIdx.x == 0) spre[tseg] = tat;
    __syncthreads();
    const float delta = (float)scalars[S_DELTA];
    // the 64 lanes of a wave take atoms tcol apart in the list (different rows of
    // bins), so that their stencils rarely add to the same LDS word at once
    const int tcol = (tat + 63) / 64;
    for (int v = threadIdx.x; v < 64 * tcol; v += blockDim.x) {
        const int t = (v & 63) * tcol + (v >> 6);
        if (t >= tat) continue;
        int lo = 0, hi = tseg - 1;  // the last segment whose prefix is <= t (non-empty)
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (spre[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const int j = sbeg[lo] + (t - spre[lo]);
        const int code = scode[lo];
        const int k[3] = {(code & 0xFF) - 128, ((code >> 8) & 0xFF) - 128, ((code >> 16) & 0xFF) - 128};
        const float4 p = xyzt[j];
        const float q = qraw[j] + delta;
        int l[3];
        float w[3][5];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double s = (double)p.x * c.hinv[a] + (double)p.y * c.hinv[3 + a] + (double)p.z * c.hinv[6 + a];
            const double u = (s + k[a]) * g.n[a];
            const double m = floor(u + 0.5);
            bspline5((float)(u - m), w[a]);
            l[a] = (int)m - 2 - M0[a];
        }
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            const int x = l[0] + a;
            if (x < 0 || x >= Pa[0]) continue;
            const float qa = q * w[0][a];
#pragma unroll
            for (int b = 0; b < 5; ++b) {
                const int y = l[1] + b;
                if (y < 0 || y >= Pa[1]) continue;
                const float qab = qa * w[1][b];
                unsigned long long *row = tile + (x * bg.P[1] + y) * bg.P[2];
#pragma unroll
                for (int e = 0; e < 5; ++e) {
                    const int z = l[2] + e;
                    if (z >= 0 && z < Pa[2])
                        atomicAdd(row + z, to_fixed((double)(qab * w[2][e])));
                }
            }
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < TP; p += blockDim.x) {
        const int x = p / (bg.P[1] * bg.P[2]), y = (p / bg.P[2]) % bg.P[1], z = p % bg.P[2];
        if (x < Pa[0] && y < Pa[1] && z < Pa[2]) {
            const size_t idx = ((size_t)(M0[0] + x) * g.n[1] + (M0[1] + y)) * g.n[2] + (M0[2] + z);
            const float v = (float)from_fixed(tile[p]);
            if (real_out) reinterpret_cast<float *>(out)[pair_index(M0[0] + x, M0[1] + y, M0[2] + z, g)] = v;
            else out[idx] = make_float2(v, 0.0f);
        }
    }
}

// Brick shape for the spread, or false when the rows or segments of a brick would
// exceed the per-work-group tables (the caller then uses the atomic spread).
bool spread_bricks(const int *mesh, const int *nc, BrickGeom *bg) {
    for (int P = SB_P; P >= 4; P /= 2) {
        int cnt[3];
        for (int a = 0; a < 3; ++a) {
            bg->P[a] = std::min(P, mesh[a]);
            bg->nb[a] = (mesh[a] + bg->P[a] - 1) / bg->P[a];
            cnt[a] = (int)std::floor((bg->P[a] + 4.02) * nc[a] / mesh[a]) + 2;  // bins spanned, upper bound
        }
        const int rows = cnt[0] * cnt[1];
        const int segs = rows * ((cnt[2] - 1) / nc[2] + 2);
        if (rows <= SB_ROWS && segs <= SB_SEGS) return true;
    }
    return false;
}

__device__ inline float alias_poly5(float z) {
    const float z2 = z * z;
    return 1.0f + z2 * (-5.0f / 3.0f + z2 * (7.0f / 9.0f + z2 * (-17.0f / 189.0f + z2 * (2.0f / 2835.0f))));
}

// per-axis factors of G_opt at x = n / N: sinc^{10}(x) and alias_poly5(sin^2(pi x))^2
__device__ inline void gopt_axis(float x, float &num, float &den) {
    const float sn = sinpif(x);
    const float sc = x == 0.0f ? 1.0f : sn / (3.14159265358979f * x);
    const float sc2 = sc * sc, sc5 = sc2 * sc2 * sc;
    const float d = alias_poly5(sn);
    num = sc5 * sc5;
    den = d * d;
}

// Pointwise in k: energy and virial partials, then the two packed spectra
//   A <- i X (k~_z + 1)  (inverse: E_z + i phi'),  B <- i X k~_x - X k~_y  (inverse: E_x + i E_y)
// with X = S G_opt and k~ the derivative wave vector (zero index at a Nyquist plane).
// A work-group takes whole rows along c (the row's a and b factors once per row).  A
// and B are written interleaved, AB[point] = (A, B).

// the a and b parts of one row (j0, j1) of the mesh in k
struct InflRow {
    float kr[3], ktr[3], f01;
    int nv0, nv1;
};

__device__ inline InflRow infl_row(int j0, int j1, const MeshGeom &g, const Cell &c) {
    InflRow r;
    const int n0 = g.n[0], n1 = g.n[1];
    r.nv0 = 2 * j0 < n0 ? j0 : j0 - n0;
    r.nv1 = 2 * j1 < n1 ? j1 : j1 - n1;
    const int nt0 = ((n0 & 1) == 0 && 2 * r.nv0 == -n0) ? 0 : r.nv0;
    const int nt1 = ((n1 & 1) == 0 && 2 * r.nv1 == -n1) ? 0 : r.nv1;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        r.kr[b] = (float)(2.0 * PI_D * (c.hinv[3 * b] * r.nv0 + c.hinv[3 * b + 1] * r.nv1));
        r.ktr[b] = (float)(2.0 * PI_D * (c.hinv[3 * b] * nt0 + c.hinv[3 * b + 1] * nt1));
    }
    float num0, den0, num1, den1;
    gopt_axis((float)r.nv0 / (float)n0, num0, den0);
    gopt_axis((float)r.nv1 / (float)n1, num1, den1);
    r.f01 = (num0 * num1) / (den0 * den1);
    return r;
}

struct InflConst {
    float gk, ia2, cB0, kz[3];
};

// the point (row, j2) with transform S: adds its energy and virial terms to acc and
// returns its (A, B)
__device__ inline float4 infl_point(const InflRow &r, const InflConst &q, int j2, int n2, const float *fc, float2 S,
                                    float (&acc)[10]) {
    const int nv2 = 2 * j2 < n2 ? j2 : j2 - n2;
    if (r.nv0 == 0 && r.nv1 == 0 && nv2 == 0) return make_float4(0.f, 0.f, 0.f, 0.f);
    const int nt2 = ((n2 & 1) == 0 && 2 * nv2 == -n2) ? 0 : nv2;
    float k[3], kt[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        k[b] = fmaf(q.kz[b], (float)nv2, r.kr[b]);
        kt[b] = fmaf(q.kz[b], (float)nt2, r.ktr[b]);
    }
    const float k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    const float ik2 = 1.0f / k2;
    const float Gopt = q.gk * __expf(-k2 * q.ia2) * ik2 * (r.f01 * fc[j2]);
    const float e = (float)KE * Gopt * (S.x * S.x + S.y * S.y);
    const float cB = q.cB0 + 2.0f * ik2;
    acc[0] += e;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) acc[1 + 3 * a + b] += e * ((a == b ? 1.0f : 0.0f) - cB * k[a] * k[b]);
    const float2 X = make_float2(S.x * Gopt, S.y * Gopt);
    const float2 iX = make_float2(-X.y, X.x);
    return make_float4(iX.x * (kt[2] + 1.0f), iX.y * (kt[2] + 1.0f), iX.x * kt[0] - X.x * kt[1],
                       iX.y * kt[0] - X.y * kt[1]);
}

// constants and the c factor num / den of G_opt per index along c (n2 <= 1024) in fc
__device__ inline InflConst infl_setup(const MeshGeom &g, const Cell &c, float alpha, double vol, float *fc) {
    InflConst q;
    q.gk = (float)(2.0 * PI_D / vol);
    q.ia2 = 1.0f / (4.0f * alpha * alpha);
    q.cB0 = 2.0f * q.ia2;
#pragma unroll
    for (int b = 0; b < 3; ++b) q.kz[b] = (float)(2.0 * PI_D * c.hinv[3 * b + 2]);
    const int n2 = g.n[2];
    const float in2 = 1.0f / (float)n2;
    for (int j2 = threadIdx.x; j2 < n2; j2 += blockDim.x) {
        const int nv2 = 2 * j2 < n2 ? j2 : j2 - n2;
        float num2, den2;
        gopt_axis((float)nv2 * in2, num2, den2);
        fc[j2] = num2 / den2;
    }
    __syncthreads();
    return q;
}

// S from the full complex transform Sk
__global__ __launch_bounds__(256) void k_influence(MeshGeom g, Cell c, float alpha, double vol,
                                                   const float2 *__restrict__ Sk, float4 *__restrict__ AB,
                                                   double *__restrict__ partials) {
    const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
    __shared__ float fc[1024];
    const InflConst q = infl_setup(g, c, alpha, vol, fc);
    float acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};  // over this thread's few points, then FP64
    for (int row = blockIdx.x; row < n0 * n1; row += gridDim.x) {
        const int j0 = row / n1, j1 = row - j0 * n1;
        const InflRow r = infl_row(j0, j1, g, c);
        for (int j2 = threadIdx.x; j2 < n2; j2 += blockDim.x) {
            const size_t idx = (size_t)row * n2 + j2;
            AB[idx] = infl_point(r, q, j2, n2, fc, Sk[idx], acc);
        }
    }
    double red[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) red[k] = acc[k];
    block_partials<10>(red, partials);
}

// S(k0, k1, j2) from the half spectrum T[j0][j1][k2], k2 < H = n2 / 2, of the real-input
// transform (row = the row of (k0, k1), mrow = the row of (-k0, -k1)): T itself for
// 0 < j2 < H, conj T(-k) for j2 > H, and for j2 = 0 and H the two values packed in slot 0,
// (P + conj P') / 2 and (P - conj P') / 2i with P, P' slot 0 of the row and the mirrored row
__device__ inline float2 half_fetch(const float2 *__restrict__ T, int row, int mrow, int j2, int n2) {
    const int H = n2 / 2;
    if (j2 == 0 || j2 == H) {
        const float2 P = T[(size_t)row * H], Pm = T[(size_t)mrow * H];
        return j2 == H ? make_float2(0.5f * (P.y + Pm.y), -0.5f * (P.x - Pm.x))
                       : make_float2(0.5f * (P.x + Pm.x), 0.5f * (P.y - Pm.y));
    }
    if (j2 < H) return T[(size_t)row * H + j2];
    const float2 v = T[(size_t)mrow * H + (n2 - j2)];
    return make_float2(v.x, -v.y);
}

// S from the half spectrum of the real-input transform: every row reads its own slots
// and, for j2 > n2 / 2, those of the mirrored row (each slot is read twice, every output
// point written by its own row)
__global__ __launch_bounds__(256) void k_influence_half(MeshGeom g, Cell c, float alpha, double vol,
                                                        const float2 *__restrict__ T, float4 *__restrict__ AB,
                                                        double *__restrict__ partials) {
    const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
    __shared__ float fc[1024];
    const InflConst q = infl_setup(g, c, alpha, vol, fc);
    float acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int row = blockIdx.x; row < n0 * n1; row += gridDim.x) {
        const int j0 = row / n1, j1 = row - j0 * n1;
        const int mrow = (j0 == 0 ? 0 : n0 - j0) * n1 + (j1 == 0 ? 0 : n1 - j1);
        const InflRow r = infl_row(j0, j1, g, c);
        for (int j2 = threadIdx.x; j2 < n2; j2 += blockDim.x)
            AB[(size_t)row * n2 + j2] = infl_point(r, q, j2, n2, fc, half_fetch(T, row, mrow, j2, n2), acc);
    }
    double red[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) red[k] = acc[k];
    block_partials<10>(red, partials);
}

// The influence function fused with the first inverse pass, along a, for n0 = 256 (the
// mesh is then transformed along b and c): a work-group takes row j1, the 8 points j2 in
// [8 j2b, 8 j2b + 8) along c and every j0, i.e. the 16 interleaved lines (A and B of
// each point) of the transform along a, in the thread layout of the length-256 kernel:
// line cl = lane % 16 holds part cl % 2 of point j2 = 8 j2b + cl / 2, thread t = lane / 16
// holds j0 = t + 16 m.  The two threads of a point evaluate alternate j0 (m of their
// parity) and exchange the part they do not keep, so every point is evaluated once.
// The a and b factors of the 256 rows (j0, j1) are tabulated in LDS.
__global__ __launch_bounds__(256) void k_influence_a256(MeshGeom g, Cell c, float alpha, double vol,
                                                        const float2 *__restrict__ T, float4 *__restrict__ AB,
                                                        double *__restrict__ partials) {
    const int n1 = g.n[1], n2 = g.n[2];
    // the row table and the c factors are read only before the transform's first barrier,
    // after which its exchange area reuses their LDS
    static_assert(256 * sizeof(InflRow) + 1024 * sizeof(float) <= 16 * F256_LS * sizeof(float2), "LDS overlay");
    __shared__ __align__(16) float2 xch[16 * F256_LS];
    __shared__ float2 tw[256];
    InflRow *rtab = reinterpret_cast<InflRow *>(xch);
    float *fc = reinterpret_cast<float *>(rtab + 256);
    // consecutive j2 blocks of a row on one XCD: the two halves of a 128-byte line of the
    // half spectrum are read by neighbouring work-groups
    const int lb = xcd_block(), j1 = lb / (n2 / 8), j2b = lb - j1 * (n2 / 8);
    {
        float sn, cs;
        sincospif((float)threadIdx.x / 128.0f, &sn, &cs);
        tw[threadIdx.x] = make_float2(cs, sn);  // e^{+2 pi i m / 256}
        rtab[threadIdx.x] = infl_row(threadIdx.x, j1, g, c);
    }
    const InflConst q = infl_setup(g, c, alpha, vol, fc);  // ends with a barrier
    const int lane = threadIdx.x, cl = lane & 15, t = lane >> 4, part = cl & 1, j2 = 8 * j2b + (cl >> 1);
    const int mj1 = j1 == 0 ? 0 : n1 - j1;
    float acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    float2 a[16];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int j0 = t + 16 * (2 * k + part);
        const int row = j0 * n1 + j1, mrow = ((256 - j0) & 255) * n1 + mj1;
        const float4 R = infl_point(rtab[j0], q, j2, n2, fc, half_fetch(T, row, mrow, j2, n2), acc);
        const float2 own = part ? make_float2(R.z, R.w) : make_float2(R.x, R.y);
        const float2 other = part ? make_float2(R.x, R.y) : make_float2(R.z, R.w);
        const float2 recv = make_float2(__shfl_xor(other.x, 1, 64), __shfl_xor(other.y, 1, 64));
        a[2 * k] = part ? recv : own;
        a[2 * k + 1] = part ? own : recv;
    }
    line256<1>(a, t, tw, xch + cl * F256_LS);
    const size_t S = (size_t)n1 * n2 * 2, base = ((size_t)j1 * n2 + j2) * 2 + part;
    float2 *d = reinterpret_cast<float2 *>(AB);
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) d[base + (size_t)(t + 16 * k2) * S] = a[k2];
    double red[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) red[k] = acc[k];
    block_partials<10>(red, partials);
}

// the full transform S[j0][j1][j2] from the half spectrum (for the per-atom virial)
__global__ __launch_bounds__(256) void k_expand_half(MeshGeom g, const float2 *__restrict__ T,
                                                     float2 *__restrict__ Sk) {
    const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
    const size_t M = (size_t)n0 * n1 * n2;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < M; idx += (size_t)gridDim.x * blockDim.x) {
        const int j2 = (int)(idx % n2), row = (int)(idx / n2);
        const int j0 = row / n1, j1 = row - j0 * n1;
        const int mrow = (j0 == 0 ? 0 : n0 - j0) * n1 + (j1 == 0 ? 0 : n1 - j1);
        Sk[idx] = half_fetch(T, row, mrow, j2, n2);
    }
}

// Per-atom reciprocal virial (Eq. 39): X B_ab with X = S G_opt and the stress kernel
// B = I - (2/(4 alpha^2) + 2/k^2) k k, for the six components packed two per complex
// spectrum (each X B_ab is Hermitian, so its inverse transform is real):
//   V0 = X B_xx + i X B_yy,  V1 = X B_zz + i X B_xy,  V2 = X B_xz + i X B_yz.
__global__ __launch_bounds__(256) void k_influence_virial(MeshGeom g, Cell c, float alpha, double vol,
                                                          const float2 *Sk, float2 *V) {  // Sk may alias V + 2M
    const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
    const size_t M = (size_t)n0 * n1 * n2;
    const float gk = (float)(2.0 * PI_D / vol), ia2 = 1.0f / (4.0f * alpha * alpha), cB0 = 2.0f * ia2;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < M; idx += (size_t)gridDim.x * blockDim.x) {
        const int j2 = (int)(idx % n2), row = (int)(idx / n2);
        const int j0 = row / n1, j1 = row - j0 * n1;
        const int nv0 = 2 * j0 < n0 ? j0 : j0 - n0, nv1 = 2 * j1 < n1 ? j1 : j1 - n1;
        const int nv2 = 2 * j2 < n2 ? j2 : j2 - n2;
        if (nv0 == 0 && nv1 == 0 && nv2 == 0) {
            V[idx] = V[M + idx] = V[2 * M + idx] = make_float2(0.f, 0.f);
            continue;
        }
        float k[3];
#pragma unroll
        for (int b = 0; b < 3; ++b)
            k[b] = (float)(2.0 * PI_D * (c.hinv[3 * b] * nv0 + c.hinv[3 * b + 1] * nv1 + c.hinv[3 * b + 2] * nv2));
        float num0, den0, num1, den1, num2, den2;
        gopt_axis((float)nv0 / (float)n0, num0, den0);
        gopt_axis((float)nv1 / (float)n1, num1, den1);
        gopt_axis((float)nv2 / (float)n2, num2, den2);
        const float k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        const float ik2 = 1.0f / k2;
        const float Gopt = gk * __expf(-k2 * ia2) * ik2 * ((num0 * num1 * num2) / (den0 * den1 * den2));
        const float2 S = Sk[idx];
        const float2 X = make_float2(S.x * Gopt, S.y * Gopt);
        const float cB = cB0 + 2.0f * ik2;
        const float Bxx = 1.0f - cB * k[0] * k[0], Byy = 1.0f - cB * k[1] * k[1], Bzz = 1.0f - cB * k[2] * k[2];
        const float Bxy = -cB * k[0] * k[1], Bxz = -cB * k[0] * k[2], Byz = -cB * k[1] * k[2];
        // P + i Q with P = X B_p and Q = X B_q: (X.x B_p - X.y B_q, X.y B_p + X.x B_q)
        V[idx] = make_float2(X.x * Bxx - X.y * Byy, X.y * Bxx + X.x * Byy);
        V[M + idx] = make_float2(X.x * Bzz - X.y * Bxy, X.y * Bzz + X.x * Bxy);
        V[2 * M + idx] = make_float2(X.x * Bxz - X.y * Byz, X.y * Bxz + X.x * Byz);
    }
}

// phi^k_i += 2 k_e sum_s W phi'_s,  F^k_i += -2 k_e q'_i sum_s W E_s.
// GA_LANES lanes share one atom: lane a < 5 reads the 25 points of stencil plane a, so
// five shorter chains of loads are in flight per atom instead of one long one
constexpr int GA_LANES = 8;

__global__ __launch_bounds__(256) void k_gather(int N, const float4 *__restrict__ xyzt, Cell c, MeshGeom g,
                                                const float *__restrict__ qraw, const double *__restrict__ scalars,
                                                const float4 *__restrict__ AB, float *__restrict__ phi,
                                                float *__restrict__ Fst) {
    const int gtid = xcd_block() * blockDim.x + threadIdx.x;
    const int i = gtid / GA_LANES, pa_ = gtid % GA_LANES;
    float ph = 0.f, ex = 0.f, ey = 0.f, ez = 0.f;
    if (i < N && pa_ < 5) {
        int m0[3];
        float w[3][5];
        const float4 pa = xyzt[i];
        mesh_stencil(pa.x, pa.y, pa.z, c, g, m0, w);
        float wa = 0.f;  // w[0][pa_] without a dynamic register index
#pragma unroll
        for (int t = 0; t < 5; ++t) wa = pa_ == t ? w[0][t] : wa;
        const int j0 = wrap_index(m0[0] + pa_ - 2, g.n[0]);
        int j1[5], j2[5];
#pragma unroll
        for (int t = 0; t < 5; ++t) {
            j1[t] = wrap_index(m0[1] + t - 2, g.n[1]);
            j2[t] = wrap_index(m0[2] + t - 2, g.n[2]);
        }
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            const float wab = wa * w[1][b];
            const size_t row = ((size_t)j0 * g.n[1] + j1[b]) * g.n[2];
#pragma unroll
            for (int e = 0; e < 5; ++e) {
                const float ww = wab * w[2][e];
                const float4 v = AB[row + j2[e]];  // (E_z, phi', E_x, E_y)
                ez = fmaf(ww, v.x, ez);
                ph = fmaf(ww, v.y, ph);
                ex = fmaf(ww, v.z, ex);
                ey = fmaf(ww, v.w, ey);
            }
        }
    }
#pragma unroll
    for (int o = GA_LANES / 2; o > 0; o >>= 1) {
        ph += __shfl_xor(ph, o, 64);
        ex += __shfl_xor(ex, o, 64);
        ey += __shfl_xor(ey, o, 64);
        ez += __shfl_xor(ez, o, 64);
    }
    if (i < N && pa_ == 0) {
        const float q = qraw[i] + (float)scalars[S_DELTA];
        const float k2 = 2.0f * (float)KE;
        phi[i] += k2 * ph;
        Fst[i] += -k2 * q * ex;
        Fst[(size_t)N + i] += -k2 * q * ey;
        Fst[(size_t)2 * N + i] += -k2 * q * ez;
    }
}

// W^k_i[ab] += k_e q'_i sum_s W(r_i - r_s) v_ab(r_s) from the three inverse-transformed
// packed meshes; GA_LANES lanes per atom, lane a < 5 takes stencil plane a
__global__ __launch_bounds__(256) void k_gather_virial(int N, const float4 *__restrict__ xyzt, Cell c, MeshGeom g,
                                                       const float *__restrict__ qraw,
                                                       const double *__restrict__ scalars,
                                                       const float2 *__restrict__ V, float *__restrict__ Vat) {
    const int gtid = xcd_block() * blockDim.x + threadIdx.x;
    const int i = gtid / GA_LANES, pa_ = gtid % GA_LANES;
    const size_t M = (size_t)g.n[0] * g.n[1] * g.n[2];
    float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // xx yy zz xy xz yz
    if (i < N && pa_ < 5) {
        int m0[3];
        float w[3][5];
        const float4 pa = xyzt[i];
        mesh_stencil(pa.x, pa.y, pa.z, c, g, m0, w);
        float wa = 0.f;
#pragma unroll
        for (int t = 0; t < 5; ++t) wa = pa_ == t ? w[0][t] : wa;
        const int j0 = wrap_index(m0[0] + pa_ - 2, g.n[0]);
        int j1[5], j2[5];
#pragma unroll
        for (int t = 0; t < 5; ++t) {
            j1[t] = wrap_index(m0[1] + t - 2, g.n[1]);
            j2[t] = wrap_index(m0[2] + t - 2, g.n[2]);
        }
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            const float wab = wa * w[1][b];
            const size_t row = ((size_t)j0 * g.n[1] + j1[b]) * g.n[2];
#pragma unroll
            for (int e = 0; e < 5; ++e) {
                const float ww = wab * w[2][e];
                const size_t pt = row + j2[e];
                const float2 a0 = V[pt], a1 = V[M + pt], a2 = V[2 * M + pt];
                v[0] = fmaf(ww, a0.x, v[0]);
                v[1] = fmaf(ww, a0.y, v[1]);
                v[2] = fmaf(ww, a1.x, v[2]);
                v[3] = fmaf(ww, a1.y, v[3]);
                v[4] = fmaf(ww, a2.x, v[4]);
                v[5] = fmaf(ww, a2.y, v[5]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int o = GA_LANES / 2; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    if (i < N && pa_ == 0) {
        const float f = (float)KE * (qraw[i] + (float)scalars[S_DELTA]);
#pragma unroll
        for (int k = 0; k < 6; ++k) Vat[(size_t)k * N + i] += f * v[k];
    }
}

hipError_t fft3d_r2c(float2 *data, const int *mesh, hipStream_t s);
hipError_t fft3d_bc(float2 *data, const int *mesh, int sign, hipStream_t s, int inner);
bool fft_r2c_supported(const int *mesh);

hipError_t launch_pppm(const Plan &p) {
    MeshGeom g{{p.mesh[0], p.mesh[1], p.mesh[2]}};
    const int64_t M = p.mesh_pts;
    const int G = (p.N + 255) / 256;
    const int GM = (int)((M + 255) / 256);
    // a mesh of 256 points along c (even along b) takes the real-input transform and the
    // half spectrum; otherwise the complex transform of (rho, 0)
    const bool half = fft_r2c_supported(p.mesh);
    hipError_t e;
    if (p.bricks) {
        BrickGeom bg;
        for (int a = 0; a < 3; ++a) {
            bg.P[a] = p.brickP[a];
            bg.nb[a] = p.brickNb[a];
        }
        const int nbricks = bg.nb[0] * bg.nb[1] * bg.nb[2];
        hipLaunchKernelGGL(k_spread_bricks, dim3(nbricks), dim3(256), 0, p.stream, p.xyzt, p.cell, g, p.nc[0],
                           p.nc[1], p.nc[2], bg, p.cell_start, p.qraw, p.scalars, p.meshA, half ? 1 : 0);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        stage_mark(p, ST_SPREAD, 1);
    } else if (half) {
        e = fill_zero(p.meshA, sizeof(float) * (size_t)M, p.stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_spread, dim3(G), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell, g, p.qraw, p.scalars,
                           reinterpret_cast<float *>(p.meshA), 1);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        stage_mark(p, ST_SPREAD, 2);
    } else {
        e = fill_zero(p.rho, sizeof(float) * (size_t)M, p.stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_spread, dim3(G), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell, g, p.qraw, p.scalars,
                           p.rho, 0);
        hipLaunchKernelGGL(k_real_to_complex, dim3(GM), dim3(256), 0, p.stream, M, p.rho, p.meshA);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        stage_mark(p, ST_SPREAD, 3);
    }
    e = half ? fft3d_r2c(p.meshA, p.mesh, p.stream) : fft3d(p.meshA, nullptr, p.mesh, -1, p.stream);
    if (e != hipSuccess) return e;
    stage_mark(p, ST_FFT_FWD, 3);  // real input: c with the pair split, b, a
    const int rows = p.mesh[0] * p.mesh[1];
    // n0 = 256: the influence function and the first inverse pass (along a) in one kernel
    const bool fused = half && p.mesh[0] == 256 && p.mesh[2] % 8 == 0;
    int GI;
    if (fused) {
        GI = p.mesh[1] * (p.mesh[2] / 8);
        hipLaunchKernelGGL(k_influence_a256, dim3(GI), dim3(256), 0, p.stream, g, p.cell, (float)p.alpha, p.vol,
                           p.meshA, (float4 *)p.meshAB, p.partials);
    } else if (half) {
        GI = rows < 4096 ? rows : 4096;
        hipLaunchKernelGGL(k_influence_half, dim3(GI), dim3(256), 0, p.stream, g, p.cell, (float)p.alpha, p.vol,
                           p.meshA, (float4 *)p.meshAB, p.partials);
    } else {
        GI = rows < 4096 ? rows : 4096;
        hipLaunchKernelGGL(k_influence, dim3(GI), dim3(256), 0, p.stream, g, p.cell, (float)p.alpha, p.vol, p.meshA,
                           (float4 *)p.meshAB, p.partials);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = reduce_partials(p, GI, 10, S_UK, false);  // S_UK, S_WK[9]
    if (e != hipSuccess) return e;
    stage_mark(p, ST_INFLUENCE, 2);
    // both spectra in the same launches
    e = fused ? fft3d_bc(p.meshAB, p.mesh, +1, p.stream, 2) : fft3d(p.meshAB, nullptr, p.mesh, +1, p.stream, 2);
    if (e != hipSuccess) return e;
    stage_mark(p, ST_FFT_INV, fused ? 2 : 3);
    const int GG = (int)(((int64_t)p.N * GA_LANES + 255) / 256);
    hipLaunchKernelGGL(k_gather, dim3(GG), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell, g, p.qraw,
                       p.scalars, (const float4 *)p.meshAB, p.phi, p.Fst);
    stage_mark(p, ST_GATHER);
    if (p.out.virial_atom) {
        // six more inverse transforms, two per packed complex mesh (Eq. 39); from the half
        // spectrum, S is first expanded into the third of those meshes (each point of it
        // is read before the kernel overwrites it)
        const float2 *Sk = p.meshA;
        if (half) {
            hipLaunchKernelGGL(k_expand_half, dim3(GM < 8192 ? GM : 8192), dim3(256), 0, p.stream, g, p.meshA,
                               p.meshV + 2 * (size_t)M);
            Sk = p.meshV + 2 * (size_t)M;
        }
        hipLaunchKernelGGL(k_influence_virial, dim3(GM < 8192 ? GM : 8192), dim3(256), 0, p.stream, g, p.cell,
                           (float)p.alpha, p.vol, Sk, p.meshV);
        e = hipGetLastError();
        for (int v = 0; v < 3 && e == hipSuccess; ++v) e = fft3d(p.meshV + (size_t)v * M, nullptr, p.mesh, +1, p.stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_gather_virial, dim3(GG), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell, g, p.qraw,
                           p.scalars, p.meshV, p.Vat);
        stage_mark(p, ST_OTHER);
    }
    return hipGetLastError();
}

}  // namespace qnep
