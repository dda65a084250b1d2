// Spatial binning, deterministic counting sort into cell order, and image-aware
// neighbour lists (radial with its angular sub-list).
//
// The NEP cutoffs (Sec. 2.1) define the lists; every (j, n) with
// |r_j + n.h - r_i| < rc and (j, n) != (i, 0) is listed, so cells thinner than 2 rc
// (several images of one atom) are handled exactly.  Bins are about rc_R / 2 wide;
// a stencil of (2m+1)^3 bins is walked unwrapped so that each (bin, image) pair is
// visited once.  Candidates are screened in FP32 and decided with the FP64
// displacement rounded to FP32 (the same rule every kernel uses).
#include "plan.h"

namespace qnep {

// ---------------------------------------------------------------- binning
__global__ void k_bin(int N, const float *__restrict__ pos, const int32_t *__restrict__ type, int T, Cell c,
                      int nc0, int nc1, int nc2, int iso, int *__restrict__ cid, int *__restrict__ count,
                      int32_t *__restrict__ flags) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double x = pos[i], y = pos[N + i], z = pos[2 * N + i];
    int nc[3] = {nc0, nc1, nc2}, cc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double s = x * c.hinv[a] + y * c.hinv[3 + a] + z * c.hinv[6 + a];
        if (iso && (s < 0.0 || s >= 1.0)) atomicOr(flags, QNEP_FLAG_OUTSIDE);  // an isolated system's box
        s -= floor(s);
        int k = (int)(s * nc[a]);
        cc[a] = k < 0 ? 0 : (k >= nc[a] ? nc[a] - 1 : k);
    }
    int lin = row_rank(cc[0], cc[1], nc0, nc1) * nc2 + cc[2];
    cid[i] = lin;
    atomicAdd(&count[lin], 1);
    int t = type[i];
    if (t < 0 || t >= T) atomicOr(flags, QNEP_FLAG_BAD_SPECIES);
}

// three-phase exclusive scan of count[0..n) into start[0..n] (and cursor = start)
constexpr int SCAN_B = 1024;

__device__ inline int block_scan_inclusive(int v, int *buf) {
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < SCAN_B; o <<= 1) {
        int t = threadIdx.x >= (unsigned)o ? buf[threadIdx.x - o] : 0;
        __syncthreads();
        buf[threadIdx.x] += t;
        __syncthreads();
    }
    return buf[threadIdx.x];
}

__global__ void k_scan_blocks(int n, const int *__restrict__ count, int *__restrict__ start,
                              int *__restrict__ bsum) {
    __shared__ int buf[SCAN_B];
    int i = blockIdx.x * SCAN_B + threadIdx.x;
    int v = i < n ? count[i] : 0;
    int inc = block_scan_inclusive(v, buf);
    if (i < n) start[i] = inc - v;
    if (threadIdx.x == SCAN_B - 1) bsum[blockIdx.x] = inc;
}

__global__ void k_scan_top(int nb, int *__restrict__ bsum, int *__restrict__ total) {
    __shared__ int buf[SCAN_B];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += SCAN_B) {
        int i = base + threadIdx.x;
        int v = i < nb ? bsum[i] : 0;
        int inc = block_scan_inclusive(v, buf);
        if (i < nb) bsum[i] = carry + inc - v;
        __syncthreads();
        if (threadIdx.x == SCAN_B - 1) carry += inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_add(int n, const int *__restrict__ bsum, int *__restrict__ start, int *__restrict__ cursor) {
    int i = blockIdx.x * SCAN_B + threadIdx.x;
    if (i < n) {
        int v = start[i] + bsum[blockIdx.x];
        start[i] = v;
        cursor[i] = v;
    }
}

__global__ void k_scatter(int N, const int *__restrict__ cid, int *__restrict__ cursor, int *__restrict__ perm) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int slot = atomicAdd(&cursor[cid[i]], 1);
    perm[slot] = i;
}

// order the atoms of each bin by their input index (makes the sort deterministic)
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

// sorted packed copies (x, y, z, species bits); positions are moved into the cell by
// whole lattice vectors only (atoms already inside keep their exact FP32 coordinates)
__global__ void k_gather_sorted(int N, const float *__restrict__ pos, const int32_t *__restrict__ type, int T,
                                Cell c, const int *__restrict__ perm, float4 *__restrict__ xyzt,
                                int *__restrict__ ts) {
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
    // species outside [0, T) were flagged by k_bin; clamp so that no kernel indexes past its tables
    int t = type[i];
    t = t < 0 ? 0 : (t >= T ? T - 1 : t);
    xyzt[s] = make_float4((float)x, (float)y, (float)z, __int_as_float(t));
    ts[s] = t;
}

// ---------------------------------------------------------------- lists
// LS_LANES lanes share one sorted atom and walk the segments of its bin stencil
// (trimmed to the list cutoff in orthorhombic cells) with stride LS_LANES.  A
// candidate is screened in FP32 and decided with the FP64-formed displacement
// (ImageShift::exact): r^2 < rc^2 puts it in the main list, r^2 < rs^2 also in the
// sub-list.  The hits of one pass of the lane group are compacted with a ballot in
// lane order, so both lists come out in the fixed walk order.  Lists are atom-major:
// list[i * cap + k] and sub[i * cap_sub + k].
constexpr int LS_LANES = 8;
constexpr uint32_t LS_MASK = (1u << LS_LANES) - 1u;  // one lane group in a ballot
constexpr int LS_APB = 256 / LS_LANES;  // atoms per work-group
constexpr int LS_SEG = 64;              // segments of one atom held in LDS at a time

__global__ __launch_bounds__(256, 6) void k_lists(int N, const float4 *__restrict__ xyzt, Cell c, Stencil st,
                                               const int *__restrict__ start, double rc2, int cap,
                                               uint32_t *__restrict__ list, int *__restrict__ cnt, double rs2,
                                               int cap_sub, uint32_t *__restrict__ sub,
                                               int *__restrict__ cnt_sub, int iso, int32_t *__restrict__ flags) {
    __shared__ int2 seg[LS_APB][LS_SEG];
    __shared__ float4 shf[SEG_NIMG];  // (shift rounded to FP32, the image part of a list entry)
    const int nimg = 2 * st.R + 1;
    for (int k = threadIdx.x; k < nimg * nimg * nimg; k += blockDim.x) {
        int n0, n1, n2;
        image_of(k, st.R, n0, n1, n2);
        const ImageShift sh(c, n0, n1, n2);
        shf[k] = make_float4(sh.fx, sh.fy, sh.fz, __uint_as_float(nb_encode(0, n0, n1, n2)));
    }
    const int a = threadIdx.x / LS_LANES, ln = threadIdx.x % LS_LANES;
    const int i = xcd_block() * LS_APB + a;
    const bool live = i < N;
    const float4 pi = xyzt[live ? i : 0];
    const AtomBin ab = atom_bin(pi, c, st);
    // FP32 distances decide every candidate outside thin shells around the two cutoffs
    // (their error is ~1e-5 relative); inside a shell the FP64 test decides
    const float rc2_hi = (float)(rc2 * (1.0 + 1e-4)), rc2_lo = (float)(rc2 * (1.0 - 1e-4));
    const float rs2_hi = (float)(rs2 * (1.0 + 1e-4)), rs2_lo = (float)(rs2 * (1.0 - 1e-4));
    const int self_img = (st.R * nimg + st.R) * nimg + st.R;
    const int gshift = (threadIdx.x & 63) & ~(LS_LANES - 1);  // first lane of this group in the wave
    const uint32_t below = (1u << ln) - 1u;
    int n_main = 0, n_sub = 0;  // exact in lane 0, which has the most candidates of every chunk
    __syncthreads();  // image table in place
    // an atom's segment table is written and read by the atom's own lanes (one wave)
    for (int r0 = 0; r0 < st.nrows; r0 += st.rows_chunk) {
        wave_lds_sync();  // the previous chunk's walk is done with the table
        const int ns = stencil_segments_kept<LS_LANES, LS_SEG / 2 / LS_LANES>(
            st, c, ab, live, ln, r0, min(st.rows_chunk, st.nrows - r0), start, seg[a]);
        wave_lds_sync();
        SegWalk wk(seg[a], ns, ln);
        while (wk.valid()) {
            const int j = wk.atom(), g = wk.image();
            wk.advance(seg[a], LS_LANES);
            const float4 pj = xyzt[j];
            const float4 sf = shf[g];
            const float fx = (pj.x - pi.x) + sf.x, fy = (pj.y - pi.y) + sf.y, fz = (pj.z - pi.z) + sf.z;
            const float r2f = fx * fx + fy * fy + fz * fz;
            const bool cand = r2f < rc2_hi && !(g == self_img && j == i);
            bool hit = cand && r2f < rc2_lo, hs = cand && r2f < rs2_lo;
            if (cand && ((r2f >= rc2_lo) || (r2f >= rs2_lo && r2f < rs2_hi))) {
                int n0, n1, n2;
                image_of(g, st.R, n0, n1, n2);
                const ImageShift sh(c, n0, n1, n2);
                const double sx = sh.sx, sy = sh.sy, sz = sh.sz;
                const float dx = (float)(((double)pj.x - (double)pi.x) + sx);
                const float dy = (float)(((double)pj.y - (double)pi.y) + sy);
                const float dz = (float)(((double)pj.z - (double)pi.z) + sz);
                const double r2 = (double)dx * dx + (double)dy * dy + (double)dz * dz;
                hit = r2 < rc2;
                hs = r2 < rs2;
            }
            const uint32_t gm = (uint32_t)(__ballot(hit) >> gshift) & LS_MASK;
            const uint32_t gs = (uint32_t)(__ballot(hs) >> gshift) & LS_MASK;
            if (hit) {
                if (iso && g != self_img) atomicOr(flags, QNEP_FLAG_IMAGE);  // an isolated system sees an image
                const uint32_t code = (uint32_t)j | __float_as_uint(sf.w);
                const int k = n_main + __popc(gm & below);
                if (k < cap) list[(size_t)i * cap + k] = code;
                if (hs) {
                    const int ks = n_sub + __popc(gs & below);
                    if (ks < cap_sub) sub[(size_t)i * cap_sub + ks] = code;
                }
            }
            n_main += __popc(gm);
            n_sub += __popc(gs);
        }
        // lanes that ran out of candidates early missed the last passes' counts
        n_main = __shfl(n_main, 0, LS_LANES);
        n_sub = __shfl(n_sub, 0, LS_LANES);
    }
    if (live && ln == 0) {
        if (n_main > cap) {
            atomicOr(flags, QNEP_FLAG_RADIAL_OVERFLOW);
            n_main = cap;
        }
        if (n_sub > cap_sub) {
            atomicOr(flags, QNEP_FLAG_ANGULAR_OVERFLOW);
            n_sub = cap_sub;
        }
        cnt[i] = n_main;
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
                       p.nc[2], p.iso, p.cid, p.cell_count, p.flags);
    const int nsb = (p.ncell + SCAN_B - 1) / SCAN_B;
    hipLaunchKernelGGL(k_scan_blocks, dim3(nsb), dim3(SCAN_B), 0, p.stream, p.ncell, p.cell_count, p.cell_start,
                       p.scan_tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_B), 0, p.stream, nsb, p.scan_tmp, p.cell_start + p.ncell);
    hipLaunchKernelGGL(k_scan_add, dim3(nsb), dim3(SCAN_B), 0, p.stream, p.ncell, p.scan_tmp, p.cell_start,
                       p.cell_cursor);
    hipLaunchKernelGGL(k_scatter, dim3(G), dim3(B), 0, p.stream, N, p.cid, p.cell_cursor, p.perm);
    hipLaunchKernelGGL(k_cell_sort, dim3((p.ncell + B - 1) / B), dim3(B), 0, p.stream, p.ncell, p.cell_start,
                       p.perm);
    hipLaunchKernelGGL(k_gather_sorted, dim3(G), dim3(B), 0, p.stream, N, p.pos, p.type, p.T, p.cell, p.perm,
                       p.xyzt, p.ts);
    stage_mark(p, ST_SORT, 8);
    double rcR2 = p.rcR * p.rcR, rcA2 = p.rcA * p.rcA;
    Stencil st;
    if (!stencil_setup(st, p.nc, p.mR, p.cell.h, p.rcR > p.rcA ? p.rcR : p.rcA, LS_SEG)) return hipErrorInvalidValue;
    const int GL = (N + LS_APB - 1) / LS_APB;
    hipLaunchKernelGGL(k_lists, dim3(GL), dim3(B), 0, p.stream, N, p.xyzt, p.cell, st, p.cell_start, rcR2, p.capR,
                       p.listR, p.cntR, rcA2, p.capA, p.listA, p.cntA, p.iso, p.flags);
    stage_mark(p, ST_LISTS);
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

// Sum over the nblk rows of partials[nblk][nv] (nv <= RP_MAX_NV): up to RP_SLICES
// blocks each sum one contiguous slice of rows, every thread one value of rows read
// coalesced, then a fixed-order tree; with several slices one more block adds the
// slice sums in slice order.  The result depends only on (nblk, nv): deterministic.
constexpr int RP_THREADS = 1024, RP_SLICES = 64, RP_MAX_NV = 16;

int reduce_tmp_doubles() { return RP_SLICES * RP_MAX_NV; }

__global__ __launch_bounds__(RP_THREADS) void k_reduce_slices(const double *__restrict__ partials, int nblk,
                                                               int nv, double *__restrict__ tmp,
                                                               double *__restrict__ out, int accumulate) {
    __shared__ double red[RP_THREADS];
    const int rows = RP_THREADS / nv;  // rows read per pass; at most 128 for nv >= 8
    const int tb = threadIdx.x / nv, k = threadIdx.x - tb * nv;
    const int per = (nblk + gridDim.x - 1) / gridDim.x;
    const int b0 = blockIdx.x * per, b1 = min(nblk, b0 + per);
    double s[4] = {0.0, 0.0, 0.0, 0.0};  // four loads in flight per thread
    if (tb < rows)
        for (int b = b0 + tb; b < b1; b += 4 * rows) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int bu = b + u * rows;
                s[u] += bu < b1 ? partials[(size_t)bu * nv + k] : 0.0;
            }
        }
    red[threadIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
    int o = 1;
    while (2 * o < rows) o <<= 1;  // largest power of two below rows (rows <= 2 o)
    for (; o > 0; o >>= 1) {
        __syncthreads();
        if (tb < o && tb + o < rows) red[threadIdx.x] += red[threadIdx.x + o * nv];
    }
    if (threadIdx.x < nv) {
        if (gridDim.x > 1) {
            tmp[blockIdx.x * nv + threadIdx.x] = red[threadIdx.x];
        } else {  // one slice: this is the sum
            const double v = red[threadIdx.x];
            out[threadIdx.x] = accumulate ? out[threadIdx.x] + v : v;
        }
    }
}

// one wave per value: lane b holds slice b (nslice <= 64), then a fixed butterfly
__global__ __launch_bounds__(64 * RP_MAX_NV) void k_reduce_final(const double *__restrict__ tmp, int nslice,
                                                                 int nv, double *__restrict__ out,
                                                                 int accumulate) {
    const int k = threadIdx.x / 64, b = threadIdx.x % 64;
    if (k >= nv) return;  // whole waves leave together
    double s = b < nslice ? tmp[b * nv + k] : 0.0;
    s = wave_sum(s);
    if (b == 0) out[k] = accumulate ? out[k] + s : s;
}

static hipError_t reduce_into(const Plan &p, int nblk, int nv, double *dst, bool accumulate) {
    if (nv < 1 || nv > RP_MAX_NV) return hipErrorInvalidValue;
    // up to 8192 rows one block suffices and saves the second launch
    const int nslice = nblk <= 8192 ? 1 : std::min(RP_SLICES, nblk / 256);
    hipLaunchKernelGGL(k_reduce_slices, dim3(nslice), dim3(RP_THREADS), 0, p.stream, p.partials, nblk, nv,
                       p.red_tmp, dst, accumulate ? 1 : 0);
    if (nslice > 1)
        hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64 * nv), 0, p.stream, p.red_tmp, nslice, nv, dst,
                           accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t reduce_partials_to(const Plan &p, int nblk, int nv, double *dst) {
    return reduce_into(p, nblk, nv, dst, false);
}

hipError_t reduce_partials(const Plan &p, int nblk, int nv, int slot, bool accumulate) {
    return reduce_into(p, nblk, nv, p.scalars + slot, accumulate);
}

}  // namespace qnep
