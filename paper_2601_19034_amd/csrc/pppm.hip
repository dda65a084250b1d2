// PPPM reciprocal part (Sec. 2.6):
//   charge assignment with the order-5 B-spline W (Eq. 35), forward FFT to S(k),
//   optimized influence function G_opt = G [prod sinc^5]^2 / [prod poly(z)]^2 (Eq. 36,
//   with the denominator squared and the z^6 coefficient -17/189, the value of the
//   P = 5 alias sum), energy k_e sum G_opt |S|^2 (Eq. 34) and virial k_e sum G_opt |S|^2 B
//   (B as in Eq. 21), ik differentiation for the static force (Eq. 37) and the
//   potential mesh for the dynamic-charge force (Eq. 38), gathered with the same W.
// Two packed complex inverse transforms give (E_x + i E_y) and (E_z + i phi).
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

__device__ inline int wrap_index(int j, int n) {
    j %= n;
    return j < 0 ? j + n : j;
}

__global__ __launch_bounds__(256) void k_spread(int N, const float4 *__restrict__ xyzt, Cell c, MeshGeom g,
                                                const float *__restrict__ qraw, const double *__restrict__ scalars,
                                                float *__restrict__ rho) {
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
            const size_t row = ((size_t)j0[a] * g.n[1] + j1[b]) * g.n[2];
#pragma unroll
            for (int e = 0; e < 5; ++e) atomicAdd(&rho[row + j2[e]], qab * w[2][e]);
        }
    }
}

__global__ void k_real_to_complex(int64_t M, const float *__restrict__ rho, float2 *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) out[i] = make_float2(rho[i], 0.0f);
}

// ---------------------------------------------------------------- tiled spread
// Atomic-free charge assignment.  A brick of B0 x B1 x B2 bins accumulates the
// order-5 stencils of its atoms in an LDS tile (LDS atomics) that spans the mesh
// points those atoms can reach, and stores the tile in its own slot; k_tile_gather
// then forms each mesh point as the sum over the few tiles that cover it.  The
// result is deterministic.  Tile origin along axis a: floor(b B_a N_a / nc_a) - 3.
struct TileGeom {
    int B[3], nb[3], T[3];
};

__device__ inline int tile_origin(int b, int B, int N, int nc) { return (int)(((int64_t)b * B * N) / nc) - 3; }

__global__ __launch_bounds__(256) void k_spread_tiles(const float4 *__restrict__ xyzt, Cell c, MeshGeom g,
                                                      int nc0, int nc1, int nc2, TileGeom tg,
                                                      const int *__restrict__ start, const float *__restrict__ qraw,
                                                      const double *__restrict__ scalars, float *__restrict__ tiles,
                                                      int32_t *__restrict__ flags) {
    extern __shared__ float tile[];
    __shared__ int rowoff[65], rowbeg[64];
    const int nc[3] = {nc0, nc1, nc2};
    const int brick = blockIdx.x;
    const int bi[3] = {brick / (tg.nb[1] * tg.nb[2]), (brick / tg.nb[2]) % tg.nb[1], brick % tg.nb[2]};
    int lo[3], blo[3], bhi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        blo[a] = bi[a] * tg.B[a];
        bhi[a] = min(blo[a] + tg.B[a], nc[a]);
        lo[a] = tile_origin(bi[a], tg.B[a], g.n[a], nc[a]);
    }
    const int TV = tg.T[0] * tg.T[1] * tg.T[2];
    for (int p = threadIdx.x; p < TV; p += blockDim.x) tile[p] = 0.0f;
    const int ny = bhi[1] - blo[1];
    const int nrows = (bhi[0] - blo[0]) * ny;
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int r = 0; r < nrows; ++r) {
            const int x = blo[0] + r / ny, y = blo[1] + r % ny;
            const int base = (x * nc1 + y) * nc2;
            rowbeg[r] = start[base + blo[2]];
            rowoff[r] = acc;
            acc += start[base + bhi[2]] - rowbeg[r];
        }
        rowoff[nrows] = acc;
    }
    __syncthreads();
    const int total = rowoff[nrows];
    const float delta = (float)scalars[S_DELTA];
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        int r = 0;
        while (rowoff[r + 1] <= t) ++r;
        const int j = rowbeg[r] + (t - rowoff[r]);
        const float4 p = xyzt[j];
        const float q = qraw[j] + delta;
        const double s[3] = {(double)p.x * c.hinv[0] + (double)p.y * c.hinv[3] + (double)p.z * c.hinv[6],
                             (double)p.x * c.hinv[1] + (double)p.y * c.hinv[4] + (double)p.z * c.hinv[7],
                             (double)p.x * c.hinv[2] + (double)p.y * c.hinv[5] + (double)p.z * c.hinv[8]};
        int l[3];
        float w[3][5];
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double sa = s[a] - floor(s[a]);
            // keep the atom next to its bin across the periodic seam (rounding at s = 1)
            if (sa < (double)blo[a] / nc[a] - 0.5) sa += 1.0;
            if (sa > (double)bhi[a] / nc[a] + 0.5) sa -= 1.0;
            const double u = sa * g.n[a];
            const double m = floor(u + 0.5);
            bspline5((float)(u - m), w[a]);
            l[a] = (int)m - 2 - lo[a];
            ok = ok && l[a] >= 0 && l[a] + 4 < tg.T[a];
        }
        if (!ok) {
            atomicOr(flags, QNEP_FLAG_INTERNAL);
            continue;
        }
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            const float qa = q * w[0][a];
#pragma unroll
            for (int b = 0; b < 5; ++b) {
                const float qab = qa * w[1][b];
                float *row = tile + ((l[0] + a) * tg.T[1] + (l[1] + b)) * tg.T[2] + l[2];
#pragma unroll
                for (int e = 0; e < 5; ++e) atomicAdd(row + e, qab * w[2][e]);
            }
        }
    }
    __syncthreads();
    float *out = tiles + (size_t)brick * TV;
    for (int p = threadIdx.x; p < TV; p += blockDim.x) out[p] = tile[p];
}

// mesh point m <- sum of the tile entries that map to m (periodically); writes the
// complex FFT input (rho, 0)
__global__ __launch_bounds__(256) void k_tile_gather(MeshGeom g, int nc0, int nc1, int nc2, TileGeom tg,
                                                     const float *__restrict__ tiles, float2 *__restrict__ out) {
    const int64_t M = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t idx = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
    if (idx >= M) return;
    const int nc[3] = {nc0, nc1, nc2};
    const int m[3] = {(int)(idx / ((int64_t)g.n[1] * g.n[2])), (int)((idx / g.n[2]) % g.n[1]), (int)(idx % g.n[2])};
    int cb[3][8], cl[3][8], cn[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cn[a] = 0;
        const int N = g.n[a];
        const int kr = tg.T[a] / N + 1;
        for (int k = -kr; k <= kr; ++k) {
            const int mm = m[a] + k * N;  // unwrapped mesh index
            // tile(b) = [origin(b), origin(b) + T) holds mm only for b in [bmin, bmax]
            const double scale = (double)nc[a] / ((double)tg.B[a] * N);
            const int bmin = (int)floor((double)(mm - tg.T[a] + 5) * scale) - 1;
            const int bmax = (int)floor((double)(mm + 3) * scale) + 1;
            for (int b = bmin; b <= bmax; ++b) {
                if (b < 0 || b >= tg.nb[a]) continue;
                const int l = mm - tile_origin(b, tg.B[a], N, nc[a]);
                if (l >= 0 && l < tg.T[a] && cn[a] < 8) {
                    cb[a][cn[a]] = b;
                    cl[a][cn[a]] = l;
                    ++cn[a];
                }
            }
        }
    }
    const int TV = tg.T[0] * tg.T[1] * tg.T[2];
    float sum = 0.0f;
    for (int x = 0; x < cn[0]; ++x)
        for (int y = 0; y < cn[1]; ++y)
            for (int z = 0; z < cn[2]; ++z) {
                const int brick = (cb[0][x] * tg.nb[1] + cb[1][y]) * tg.nb[2] + cb[2][z];
                sum += tiles[(size_t)brick * TV + ((size_t)cl[0][x] * tg.T[1] + cl[1][y]) * tg.T[2] + cl[2][z]];
            }
    out[idx] = make_float2(sum, 0.0f);
}

__device__ inline float alias_poly5(float z) {
    const float z2 = z * z;
    return 1.0f + z2 * (-5.0f / 3.0f + z2 * (7.0f / 9.0f + z2 * (-17.0f / 189.0f + z2 * (2.0f / 2835.0f))));
}

__device__ inline float sinc_pi(float x) {  // sin(pi x)/(pi x)
    if (x == 0.0f) return 1.0f;
    return sinpif(x) / (3.14159265358979f * x);
}

// Pointwise in k: energy and virial partials, then the two packed spectra
//   A <- i X (k~_z + 1)  (inverse: E_z + i phi'),  B <- i X k~_x - X k~_y  (inverse: E_x + i E_y)
// with X = S G_opt and k~ the derivative wave vector (zero index at a Nyquist plane).
__global__ __launch_bounds__(256) void k_influence(MeshGeom g, Cell c, float alpha, double vol,
                                                   float2 *__restrict__ A, float2 *__restrict__ Bm,
                                                   double *__restrict__ partials) {
    const int64_t M = (int64_t)g.n[0] * g.n[1] * g.n[2];
    double red[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < M;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int j2 = (int)(idx % g.n[2]);
        const int j1 = (int)((idx / g.n[2]) % g.n[1]);
        const int j0 = (int)(idx / ((int64_t)g.n[2] * g.n[1]));
        int nv[3] = {2 * j0 < g.n[0] ? j0 : j0 - g.n[0], 2 * j1 < g.n[1] ? j1 : j1 - g.n[1],
                     2 * j2 < g.n[2] ? j2 : j2 - g.n[2]};
        const float2 S = A[idx];
        if (nv[0] == 0 && nv[1] == 0 && nv[2] == 0) {
            A[idx] = make_float2(0.f, 0.f);
            Bm[idx] = make_float2(0.f, 0.f);
            continue;
        }
        int nt[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) nt[a] = ((g.n[a] & 1) == 0 && 2 * nv[a] == -g.n[a]) ? 0 : nv[a];
        float k[3], kt[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            k[b] = (float)(2.0 * PI_D * (c.hinv[3 * b] * nv[0] + c.hinv[3 * b + 1] * nv[1] + c.hinv[3 * b + 2] * nv[2]));
            kt[b] = (float)(2.0 * PI_D * (c.hinv[3 * b] * nt[0] + c.hinv[3 * b + 1] * nt[1] + c.hinv[3 * b + 2] * nt[2]));
        }
        const float k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        const float G = (float)(2.0 * PI_D / vol) * __expf(-k2 / (4.0f * alpha * alpha)) / k2;
        float num = 1.0f, den = 1.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float x = (float)nv[a] / (float)g.n[a];
            const float sc = sinc_pi(x);
            const float sc2 = sc * sc;
            num *= sc2 * sc2 * sc;
            den *= alias_poly5(sinpif(x));
        }
        const float Gopt = G * (num * num) / (den * den);
        const float e = (float)KE * Gopt * (S.x * S.x + S.y * S.y);
        const float cB = 2.0f / (4.0f * alpha * alpha) + 2.0f / k2;
        red[0] += e;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) red[1 + 3 * a + b] += e * ((a == b ? 1.0f : 0.0f) - cB * k[a] * k[b]);
        const float2 X = make_float2(S.x * Gopt, S.y * Gopt);
        const float2 iX = make_float2(-X.y, X.x);
        A[idx] = make_float2(iX.x * (kt[2] + 1.0f), iX.y * (kt[2] + 1.0f));
        Bm[idx] = make_float2(iX.x * kt[0] - X.x * kt[1], iX.y * kt[0] - X.y * kt[1]);
    }
    block_partials<10>(red, partials);
}

// phi^k_i += 2 k_e sum_s W phi'_s,  F^k_i += -2 k_e q'_i sum_s W E_s
__global__ __launch_bounds__(256) void k_gather(int N, const float4 *__restrict__ xyzt, Cell c, MeshGeom g,
                                                const float *__restrict__ qraw, const double *__restrict__ scalars,
                                                const float2 *__restrict__ A, const float2 *__restrict__ Bm,
                                                float *__restrict__ phi, float *__restrict__ Fst) {
    const int i = xcd_block() * blockDim.x + threadIdx.x;
    if (i >= N) return;
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
    float ph = 0.f, ex = 0.f, ey = 0.f, ez = 0.f;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            const float wab = w[0][a] * w[1][b];
            const size_t row = ((size_t)j0[a] * g.n[1] + j1[b]) * g.n[2];
#pragma unroll
            for (int e = 0; e < 5; ++e) {
                const float ww = wab * w[2][e];
                const float2 va = A[row + j2[e]], vb = Bm[row + j2[e]];
                ez = fmaf(ww, va.x, ez);
                ph = fmaf(ww, va.y, ph);
                ex = fmaf(ww, vb.x, ex);
                ey = fmaf(ww, vb.y, ey);
            }
        }
    }
    const float q = qraw[i] + (float)scalars[S_DELTA];
    const float k2 = 2.0f * (float)KE;
    phi[i] += k2 * ph;
    Fst[i] += -k2 * q * ex;
    Fst[(size_t)N + i] += -k2 * q * ey;
    Fst[(size_t)2 * N + i] += -k2 * q * ez;
}

hipError_t launch_pppm(const Plan &p) {
    MeshGeom g{{p.mesh[0], p.mesh[1], p.mesh[2]}};
    const int64_t M = p.mesh_pts;
    const int G = (p.N + 255) / 256;
    const int GM = (int)((M + 255) / 256);
    hipError_t e;
    if (p.tiles) {
        TileGeom tg;
        for (int a = 0; a < 3; ++a) {
            tg.B[a] = p.tileB[a];
            tg.nb[a] = p.tileNb[a];
            tg.T[a] = p.tileT[a];
        }
        const int nbricks = tg.nb[0] * tg.nb[1] * tg.nb[2];
        const size_t lds = sizeof(float) * (size_t)tg.T[0] * tg.T[1] * tg.T[2];
        hipLaunchKernelGGL(k_spread_tiles, dim3(nbricks), dim3(256), lds, p.stream, p.xyzt, p.cell, g, p.nc[0],
                           p.nc[1], p.nc[2], tg, p.cell_start, p.qraw, p.scalars, p.tiles, p.flags);
        hipLaunchKernelGGL(k_tile_gather, dim3(GM), dim3(256), 0, p.stream, g, p.nc[0], p.nc[1], p.nc[2], tg,
                           p.tiles, p.meshA);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        stage_mark(p, ST_SPREAD, 2);
    } else {
        e = fill_zero(p.rho, sizeof(float) * (size_t)M, p.stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_spread, dim3(G), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell, g, p.qraw, p.scalars,
                           p.rho);
        hipLaunchKernelGGL(k_real_to_complex, dim3(GM), dim3(256), 0, p.stream, M, p.rho, p.meshA);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        stage_mark(p, ST_SPREAD, 3);
    }
    e = fft3d(p.meshA, nullptr, p.mesh, -1, p.stream);
    if (e != hipSuccess) return e;
    stage_mark(p, ST_FFT_FWD, 3);
    const int GI = GM < 2048 ? GM : 2048;
    hipLaunchKernelGGL(k_influence, dim3(GI), dim3(256), 0, p.stream, g, p.cell, (float)p.alpha, p.vol, p.meshA,
                       p.meshB, p.partials);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = reduce_partials(p, GI, 10, S_UK, false);  // S_UK, S_WK[9]
    if (e != hipSuccess) return e;
    stage_mark(p, ST_INFLUENCE, 2);
    e = fft3d(p.meshA, nullptr, p.mesh, +1, p.stream);
    if (e != hipSuccess) return e;
    e = fft3d(p.meshB, nullptr, p.mesh, +1, p.stream);
    if (e != hipSuccess) return e;
    stage_mark(p, ST_FFT_INV, 6);
    hipLaunchKernelGGL(k_gather, dim3(G), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell, g, p.qraw,
                       p.scalars, p.meshA, p.meshB, p.phi, p.Fst);
    stage_mark(p, ST_GATHER);
    return hipGetLastError();
}

}  // namespace qnep
