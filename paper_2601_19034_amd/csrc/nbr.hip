// Spatial binning, deterministic counting sort into cell order, and image-aware
// neighbour lists (radial with its angular sub-list; Coulomb).
//
// The NEP cutoffs (Sec. 2.1) and the real-space cutoff of Sec. 2.2.1 define the
// lists; every (j, n) with |r_j + n.h - r_i| < rc and (j, n) != (i, 0) is listed,
// so cells thinner than 2 rc (several images of one atom) are handled exactly.
#include "plan.h"

namespace qnep {

// ---------------------------------------------------------------- binning
__global__ void k_bin(int N, const float *__restrict__ pos, const int32_t *__restrict__ type, int T, Cell c,
                      int nc0, int nc1, int nc2, int *__restrict__ cid, int *__restrict__ count,
                      int32_t *__restrict__ flags) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double x = pos[i], y = pos[N + i], z = pos[2 * N + i];
    int nc[3] = {nc0, nc1, nc2}, cc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double s = x * c.hinv[a] + y * c.hinv[3 + a] + z * c.hinv[6 + a];
        s -= floor(s);
        int k = (int)(s * nc[a]);
        cc[a] = k < 0 ? 0 : (k >= nc[a] ? nc[a] - 1 : k);
    }
    int lin = (cc[0] * nc1 + cc[1]) * nc2 + cc[2];
    cid[i] = lin;
    atomicAdd(&count[lin], 1);
    int t = type[i];
    if (t < 0 || t >= T) atomicOr(flags, QNEP_FLAG_BAD_SPECIES);
}

// exclusive scan of count[0..n) into start[0..n]; one block of 1024 threads
__global__ void k_scan(int n, const int *__restrict__ count, int *__restrict__ start, int *__restrict__ cursor) {
    __shared__ int buf[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        int i = base + threadIdx.x;
        int v = i < n ? count[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            int t = threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < n) {
            int ex = carry + buf[threadIdx.x] - v;
            start[i] = ex;
            cursor[i] = ex;
        }
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) start[n] = carry;
}

__global__ void k_scatter(int N, const int *__restrict__ cid, int *__restrict__ cursor, int *__restrict__ perm) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int slot = atomicAdd(&cursor[cid[i]], 1);
    perm[slot] = i;
}

// order the atoms of each cell by their input index (makes the sort deterministic)
__global__ void k_cell_sort(int ncell, const int *__restrict__ start, int *__restrict__ perm) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    int b = start[c], e = start[c + 1];
    for (int a = b + 1; a < e; ++a) {
        int v = perm[a], k = a - 1;
        while (k >= b && perm[k] > v) {
            perm[k + 1] = perm[k];
            --k;
        }
        perm[k + 1] = v;
    }
}

// sorted SoA copies; positions are moved into the cell by whole lattice vectors
// only (atoms already inside keep their exact FP32 coordinates)
__global__ void k_gather_sorted(int N, const float *__restrict__ pos, const int32_t *__restrict__ type, int T, Cell c,
                                const int *__restrict__ perm, float *__restrict__ xs, float *__restrict__ ys,
                                float *__restrict__ zs, int *__restrict__ ts) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    int i = perm[s];
    double x = pos[i], y = pos[N + i], z = pos[2 * N + i];
    double n[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) n[a] = floor(x * c.hinv[a] + y * c.hinv[3 + a] + z * c.hinv[6 + a]);
    if (n[0] != 0.0 || n[1] != 0.0 || n[2] != 0.0) {
        x -= n[0] * c.h[0] + n[1] * c.h[3] + n[2] * c.h[6];
        y -= n[0] * c.h[1] + n[1] * c.h[4] + n[2] * c.h[7];
        z -= n[0] * c.h[2] + n[1] * c.h[5] + n[2] * c.h[8];
    }
    xs[s] = (float)x;
    ys[s] = (float)y;
    zs[s] = (float)z;
    // species outside [0, T) were flagged by k_bin; clamp so that no kernel indexes past its tables
    int t = type[i];
    ts[s] = t < 0 ? 0 : (t >= T ? T - 1 : t);
}

// ---------------------------------------------------------------- lists
// One thread per sorted atom walks the (2m+1)^3 stencil of cells, unwrapped so
// that each (cell, image) pair is visited once.  Main list: slot-major
// list[k * N + i].  Optional sub-list (r < rc_sub): atom-major sub[i * cap_sub + k].
template <bool SUB>
__global__ void k_lists(int N, const float *__restrict__ xs, const float *__restrict__ ys,
                        const float *__restrict__ zs, Cell c, int nc0, int nc1, int nc2, int m0, int m1, int m2,
                        const int *__restrict__ start, double rc2, int cap, uint32_t *__restrict__ list,
                        int *__restrict__ cnt, double rs2, int cap_sub, uint32_t *__restrict__ sub,
                        int *__restrict__ cnt_sub, int32_t *__restrict__ flags, int flag_main, int flag_sub) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double xi = xs[i], yi = ys[i], zi = zs[i];
    int ci[3], nc[3] = {nc0, nc1, nc2};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double s = xi * c.hinv[a] + yi * c.hinv[3 + a] + zi * c.hinv[6 + a];
        int k = (int)floor(s * nc[a]);
        ci[a] = k < 0 ? 0 : (k >= nc[a] ? nc[a] - 1 : k);
    }
    int n_main = 0, n_sub = 0;
    for (int d0 = -m0; d0 <= m0; ++d0) {
        int u0 = ci[0] + d0;
        int i0 = (int)floor((double)u0 / nc0);
        int w0 = u0 - i0 * nc0;
        for (int d1 = -m1; d1 <= m1; ++d1) {
            int u1 = ci[1] + d1;
            int i1 = (int)floor((double)u1 / nc1);
            int w1 = u1 - i1 * nc1;
            for (int d2 = -m2; d2 <= m2; ++d2) {
                int u2 = ci[2] + d2;
                int i2 = (int)floor((double)u2 / nc2);
                int w2 = u2 - i2 * nc2;
                double sx = i0 * c.h[0] + i1 * c.h[3] + i2 * c.h[6];
                double sy = i0 * c.h[1] + i1 * c.h[4] + i2 * c.h[7];
                double sz = i0 * c.h[2] + i1 * c.h[5] + i2 * c.h[8];
                bool self_img = (i0 == 0 && i1 == 0 && i2 == 0);
                int lin = (w0 * nc1 + w1) * nc2 + w2;
                int b = start[lin], e = start[lin + 1];
                for (int j = b; j < e; ++j) {
                    if (self_img && j == i) continue;
                    double dx = ((double)xs[j] - xi) + sx;
                    double dy = ((double)ys[j] - yi) + sy;
                    double dz = ((double)zs[j] - zi) + sz;
                    float fx = (float)dx, fy = (float)dy, fz = (float)dz;
                    double r2 = (double)fx * fx + (double)fy * fy + (double)fz * fz;
                    if (r2 < rc2) {
                        uint32_t code = nb_encode(j, i0, i1, i2);
                        if (n_main < cap) list[(size_t)n_main * N + i] = code;
                        ++n_main;
                        if (SUB && r2 < rs2) {
                            if (n_sub < cap_sub) sub[(size_t)i * cap_sub + n_sub] = code;
                            ++n_sub;
                        }
                    }
                }
            }
        }
    }
    if (n_main > cap) {
        atomicOr(flags, flag_main);
        n_main = cap;
    }
    cnt[i] = n_main;
    if (SUB) {
        if (n_sub > cap_sub) {
            atomicOr(flags, flag_sub);
            n_sub = cap_sub;
        }
        cnt_sub[i] = n_sub;
    }
}

hipError_t launch_neighbors(const Plan &p) {
    const int N = p.N;
    const int B = 256;
    const int G = (N + B - 1) / B;
    hipError_t e = fill_zero(p.cell_count, sizeof(int) * (size_t)p.ncell, p.stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin, dim3(G), dim3(B), 0, p.stream, N, p.pos, p.type, p.T, p.cell, p.nc[0], p.nc[1],
                       p.nc[2], p.cid, p.cell_count, p.flags);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, p.stream, p.ncell, p.cell_count, p.cell_start,
                       p.cell_cursor);
    hipLaunchKernelGGL(k_scatter, dim3(G), dim3(B), 0, p.stream, N, p.cid, p.cell_cursor, p.perm);
    hipLaunchKernelGGL(k_cell_sort, dim3((p.ncell + B - 1) / B), dim3(B), 0, p.stream, p.ncell, p.cell_start,
                       p.perm);
    hipLaunchKernelGGL(k_gather_sorted, dim3(G), dim3(B), 0, p.stream, N, p.pos, p.type, p.T, p.cell, p.perm, p.xs,
                       p.ys, p.zs, p.ts);
    stage_mark(p, ST_SORT, 6);
    double rcR2 = p.rcR * p.rcR, rcA2 = p.rcA * p.rcA;
    hipLaunchKernelGGL(k_lists<true>, dim3(G), dim3(B), 0, p.stream, N, p.xs, p.ys, p.zs, p.cell, p.nc[0],
                       p.nc[1], p.nc[2], p.mR[0], p.mR[1], p.mR[2], p.cell_start, rcR2, p.capR, p.listR, p.cntR,
                       rcA2, p.capA, p.listA, p.cntA, p.flags, QNEP_FLAG_RADIAL_OVERFLOW,
                       QNEP_FLAG_ANGULAR_OVERFLOW);
    stage_mark(p, ST_LISTS);
    if (p.mode == 1) {
        double rc2 = p.rc_coul * p.rc_coul;
        hipLaunchKernelGGL(k_lists<false>, dim3(G), dim3(B), 0, p.stream, N, p.xs, p.ys, p.zs, p.cell, p.nc[0],
                           p.nc[1], p.nc[2], p.mC[0], p.mC[1], p.mC[2], p.cell_start, rc2, p.capC, p.listC, p.cntC,
                           0.0, 0, (uint32_t *)nullptr, (int *)nullptr, p.flags, QNEP_FLAG_COULOMB_OVERFLOW, 0);
        stage_mark(p, ST_LISTS_C);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- utilities
__global__ void k_fill_zero(uint32_t *__restrict__ p, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0u;
}

hipError_t fill_zero(void *ptr, size_t bytes, hipStream_t s) {
    size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t *)ptr, n);
    return hipGetLastError();
}

__global__ void k_reduce_partials(const double *__restrict__ partials, int nblk, int nv, double *__restrict__ out,
                                  int accumulate) {
    __shared__ double red[256];
    for (int k = 0; k < nv; ++k) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 256) s += partials[(size_t)b * nv + k];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = accumulate ? out[k] + red[0] : red[0];
        __syncthreads();
    }
}

hipError_t reduce_partials(const Plan &p, int nblk, int nv, int slot, bool accumulate) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, p.stream, p.partials, nblk, nv,
                       p.scalars + slot, accumulate ? 1 : 0);
    return hipGetLastError();
}

}  // namespace qnep
