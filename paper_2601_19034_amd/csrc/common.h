// Internal definitions shared by the HIP translation units of libqnep.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qnep {

constexpr double KE = 14.399645;      // e^2 / (4 pi eps0) in eV * Angstrom
constexpr double PI_D = 3.14159265358979323846;
constexpr int LM = 24;                // real harmonics (l, m) for l = 1..4
constexpr int MAX_T = 4;              // species compiled in
constexpr int MAX_NEU = 64;           // hidden units
constexpr int RED_THREADS = 256;      // threads of every block that writes FP64 partials
// most lanes per atom among the kernels that write FP64 partials (real space, radial
// forces); the partials buffer holds one row per work-group of the largest grid
constexpr int PARTIALS_LANES_MAX = 16;

// Cell passed by value to kernels: rows of h are the cell vectors a, b, c.
struct Cell {
    double h[9];
    double hinv[9];
};

// A neighbour entry packs the atom index (sorted order) and the periodic image
// n in [-3, 3]^3 of the neighbour:  j | (n1+3) << 23 | (n2+3) << 26 | (n3+3) << 29.
constexpr uint32_t IDX_BITS = 23;
constexpr uint32_t IDX_MASK = (1u << IDX_BITS) - 1u;

__host__ __device__ inline uint32_t nb_encode(int j, int n1, int n2, int n3) {
    return (uint32_t)j | ((uint32_t)(n1 + 3) << 23) | ((uint32_t)(n2 + 3) << 26) | ((uint32_t)(n3 + 3) << 29);
}
__device__ inline int nb_index(uint32_t e) { return (int)(e & IDX_MASK); }
__device__ inline void nb_image(uint32_t e, int &n1, int &n2, int &n3) {
    n1 = (int)((e >> 23) & 7u) - 3;
    n2 = (int)((e >> 26) & 7u) - 3;
    n3 = (int)((e >> 29) & 7u) - 3;
}
// the entry that atom j holds for atom i when e = (j, n) is in i's list: (i, -n)
__device__ inline uint32_t nb_reverse(uint32_t e, int i) {
    uint32_t c1 = (e >> 23) & 7u, c2 = (e >> 26) & 7u, c3 = (e >> 29) & 7u;
    return (uint32_t)i | ((6u - c1) << 23) | ((6u - c2) << 26) | ((6u - c3) << 29);
}

__device__ inline int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Storage rank of the row of bins (a, b) (a row runs along c).  Rows are kept in
// strips ROW_STRIP rows wide along b: strip by strip, then a, then b within the
// strip.  A sweep over the sorted atoms then meets a row's neighbours across a
// (which a neighbour search reaches) a few hundred atoms apart rather than a
// whole a-plane apart, so the data of neighbouring atoms is still cached.
constexpr int ROW_STRIP = 8;
__device__ inline int row_rank(int a, int b, int nc0, int nc1) {
    const int b0 = b / ROW_STRIP * ROW_STRIP, w = min(ROW_STRIP, nc1 - b0);
    return b0 * nc0 + a * w + (b - b0);
}

// bin of a (wrapped) position: floor(s_a n_a) with s = r h^{-1} in FP64, clamped
__device__ inline void bin_of(float4 p, const Cell &c, int nc0, int nc1, int nc2, int *ci) {
    const int nc[3] = {nc0, nc1, nc2};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double s = (double)p.x * c.hinv[a] + (double)p.y * c.hinv[3 + a] + (double)p.z * c.hinv[6 + a];
        int k = (int)floor(s * nc[a]);
        ci[a] = k < 0 ? 0 : (k >= nc[a] ? nc[a] - 1 : k);
    }
}

// Lattice shift n.h of one periodic image, in FP64 and rounded to FP32.
struct ImageShift {
    double sx, sy, sz;
    float fx, fy, fz;
    __device__ ImageShift(const Cell &c, int n1, int n2, int n3) {
        sx = n1 * c.h[0] + n2 * c.h[3] + n3 * c.h[6];
        sy = n1 * c.h[1] + n2 * c.h[4] + n3 * c.h[7];
        sz = n1 * c.h[2] + n2 * c.h[5] + n3 * c.h[8];
        fx = (float)sx;
        fy = (float)sy;
        fz = (float)sz;
    }
    // r_j + n.h - r_i formed in FP64 from the FP32 coordinates and rounded once to
    // FP32.  The difference of two FP32 numbers is exact in FP64 and IEEE rounding is
    // odd-symmetric, so the (j, i, -n) displacement is the exact negation of (i, j, n).
    __device__ float3 exact(float4 pi, float4 pj) const {
        return make_float3((float)(((double)pj.x - (double)pi.x) + sx), (float)(((double)pj.y - (double)pi.y) + sy),
                           (float)(((double)pj.z - (double)pi.z) + sz));
    }
};

// ---------------------------------------------------------------- fixed point
// 64-bit fixed point in units of 2^-40 for sums accumulated by LDS atomics: integer
// additions are exact and associative (the sum does not depend on their order) and
// LDS integer atomics are faster than floating-point ones.  Range +-8.4e6.
constexpr double FIX_SCALE = 1099511627776.0;  // 2^40
__device__ inline unsigned long long to_fixed(double x) {
    return (unsigned long long)__double2ll_rn(x * FIX_SCALE);
}
__device__ inline double from_fixed(unsigned long long v) { return (double)(long long)v * (1.0 / FIX_SCALE); }

// ---------------------------------------------------------------- stencil segments
// The bins within m_a of an atom's bin, read as rows along c: a row is one contiguous
// range of sorted atoms per periodic image along c.  A group of lanes that share one
// atom builds the list of these ranges ("segments") in LDS and then walks their
// concatenation with a stride of the group size, so that every lane of the group gets
// the same number of candidates whatever the row lengths.  In an orthorhombic cell a
// row is first trimmed to the bins that can hold an atom within rtrim (a row whose
// gap to the atom in the ab plane exceeds rtrim is dropped, the others are cut to the
// chord of that sphere along c).  A segment is {first atom, length | image index <<
// SEG_LEN_BITS}; the image index addresses the (2R+1)^3 lattice shifts |n_a| <= R.
constexpr int SEG_LEN_BITS = 23;  // N < 2^23
constexpr uint32_t SEG_LEN_MASK = (1u << SEG_LEN_BITS) - 1u;
constexpr int SEG_RMAX = 3;
constexpr int SEG_NIMG = (2 * SEG_RMAX + 1) * (2 * SEG_RMAX + 1) * (2 * SEG_RMAX + 1);

struct Stencil {
    int nc[3], m[3];
    int R;           // images reached: |n_a| <= R
    int nrows;       // (2 m0 + 1)(2 m1 + 1)
    int rows_chunk;  // rows whose segments always fit one table of `cap` entries
    int trim;        // orthorhombic cell: rows trimmed to the sphere of radius rtrim
    float rtrim2;    // rtrim^2
    float bw0, bw1;  // bin widths along a and b (orthorhombic cell)
    float ibw2;      // bins per unit length along c
};

// Host set-up for a stencil of half-widths m over nc bins, trimmed to the cutoff rc
// (plus a margin far above the FP32 error of positions).  False when the stencil
// reaches images beyond SEG_RMAX.
inline bool stencil_setup(Stencil &st, const int *nc, const int *m, const double *h, double rc, int cap) {
    st.R = 0;
    for (int a = 0; a < 3; ++a) {
        st.nc[a] = nc[a];
        st.m[a] = m[a];
        const int r = (m[a] + nc[a] - 1) / nc[a];
        st.R = r > st.R ? r : st.R;
    }
    if (st.R > SEG_RMAX) return false;
    st.nrows = (2 * m[0] + 1) * (2 * m[1] + 1);
    const int nz = 2 * m[2] / nc[2] + 2;  // most images along c that one row spans
    st.rows_chunk = cap / nz > 1 ? cap / nz : 1;
    st.trim = (h[1] == 0.0 && h[2] == 0.0 && h[3] == 0.0 && h[5] == 0.0 && h[6] == 0.0 && h[7] == 0.0 &&
               h[0] > 0.0 && h[4] > 0.0 && h[8] > 0.0) ? 1 : 0;
    const double rt = rc * (1.0 + 1e-4) + 1e-3;
    st.rtrim2 = (float)(rt * rt);
    st.bw0 = (float)(h[0] / nc[0]);
    st.bw1 = (float)(h[4] / nc[1]);
    st.ibw2 = (float)(nc[2] / h[8]);
    return true;
}

// bin of a position (as bin_of) and the position in bin units (the FP32 rounding of u
// is far inside the trimming margin)
struct AtomBin {
    int ci[3];
    float u[3];
};
__device__ inline AtomBin atom_bin(float4 p, const Cell &c, const Stencil &st) {
    AtomBin b;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double s = (double)p.x * c.hinv[a] + (double)p.y * c.hinv[3 + a] + (double)p.z * c.hinv[6 + a];
        const double u = s * st.nc[a];
        b.u[a] = (float)u;
        const int k = (int)floor(u);
        b.ci[a] = k < 0 ? 0 : (k >= st.nc[a] ? st.nc[a] - 1 : k);
    }
    return b;
}

// floor(a / n) for a in [-SEG_RMAX n, (SEG_RMAX + 1) n), the range of unwrapped bin
// coordinates a stencil reaches: the image of the bin, by comparisons (an integer
// division by a value known only at run time costs dozens of instructions)
__device__ inline int image_index(int a, int n) {
    int k = 0;
#pragma unroll
    for (int t = 1; t <= SEG_RMAX; ++t) k += (int)(a >= t * n) - (int)(a < (1 - t) * n);
    return k;
}

// LDS written by other lanes of the same wave becomes visible to this lane
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// bins [zl, zh] along c (unwrapped) of the stencil row at offsets (d0, d1) in
// [0, 2 m0] x [0, 2 m1] that can hold a neighbour
__device__ inline bool stencil_row(const Stencil &st, const Cell &c, const AtomBin &b, int d0, int d1, int &zl,
                                   int &zh) {
    zl = b.ci[2] - st.m[2];
    zh = b.ci[2] + st.m[2];
    if (!st.trim) return true;
    const float l0 = (float)(b.ci[0] + (d0 - st.m[0])), l1 = (float)(b.ci[1] + (d1 - st.m[1]));
    const float g0 = fmaxf(0.0f, fmaxf(l0 - b.u[0], b.u[0] - l0 - 1.0f)) * st.bw0;
    const float g1 = fmaxf(0.0f, fmaxf(l1 - b.u[1], b.u[1] - l1 - 1.0f)) * st.bw1;
    const float h2 = st.rtrim2 - g0 * g0 - g1 * g1;
    if (h2 <= 0.0f) return false;
    const float hz = sqrtf(h2) * st.ibw2;
    zl = max(zl, (int)floorf(b.u[2] - hz));
    zh = min(zh, (int)floorf(b.u[2] + hz));
    return zl <= zh;
}

// Segments of stencil rows [r0, r0 + rn) of one atom into seg[]: every lane of the
// LANES-lane group calls it (lanes without a live atom pass live = false) and gets
// the segment count.  The caller synchronizes before the table is read.
template <int LANES>
__device__ inline int stencil_segments(const Stencil &st, const Cell &c, const AtomBin &b, bool live, int sub,
                                       int r0, int rn, const int *__restrict__ start, int2 *seg) {
    const int nc0 = st.nc[0], nc1 = st.nc[1], nc2 = st.nc[2], w1n = 2 * st.m[1] + 1;
    const int nimg = 2 * st.R + 1;
    const int rpl = (rn + LANES - 1) / LANES;  // rows per lane, contiguous: the table keeps row order
    const int rb = r0 + sub * rpl, re = min(rb + rpl, r0 + rn);
    const int d0b = rb / w1n, d1b = rb - d0b * w1n;  // row rb at offsets (d0b, d1b); later rows by counting
    int cnt = 0;
    for (int r = rb, d0 = d0b, d1 = d1b; live && r < re; ++r) {
        int zl, zh;
        if (stencil_row(st, c, b, d0, d1, zl, zh)) cnt += image_index(zh, nc2) - image_index(zl, nc2) + 1;
        if (++d1 == w1n) { d1 = 0; ++d0; }
    }
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < LANES; o <<= 1) {
        const int v = __shfl_up(incl, o, LANES);
        if (sub >= o) incl += v;
    }
    int pos = incl - cnt;
    for (int r = rb, d0 = d0b, d1 = d1b; live && r < re; ++r) {
        int zl, zh;
        if (stencil_row(st, c, b, d0, d1, zl, zh)) {
            const int u0 = b.ci[0] + d0 - st.m[0], i0 = image_index(u0, nc0), b0 = u0 - i0 * nc0;
            const int u1 = b.ci[1] + d1 - st.m[1], i1 = image_index(u1, nc1), b1 = u1 - i1 * nc1;
            const int rowbase = row_rank(b0, b1, nc0, nc1) * nc2;
            const int z0 = image_index(zl, nc2), z1 = image_index(zh, nc2);
            for (int i2 = z0; i2 <= z1; ++i2) {
                const int za = max(zl, i2 * nc2) - i2 * nc2, zb = min(zh, i2 * nc2 + nc2 - 1) - i2 * nc2;
                const int jb = start[rowbase + za], je = start[rowbase + zb + 1];
                const uint32_t img = (uint32_t)(((i0 + st.R) * nimg + (i1 + st.R)) * nimg + (i2 + st.R));
                seg[pos++] = make_int2(jb, (int)((uint32_t)(je - jb) | (img << SEG_LEN_BITS)));
            }
        }
        if (++d1 == w1n) { d1 = 0; ++d0; }
    }
    return live ? __shfl(incl, LANES - 1, LANES) : 0;
}

// As stencil_segments, for rn <= RPL LANES (a lane takes at most RPL rows): the trimmed
// range of each row is computed once and kept in registers between the counting pass and
// the pass that writes the table.  Fewer instructions for more registers: the callers
// bound their register count to keep their occupancy (launch bounds).
template <int LANES, int RPL>
__device__ inline int stencil_segments_kept(const Stencil &st, const Cell &c, const AtomBin &b, bool live, int sub,
                                       int r0, int rn, const int *__restrict__ start, int2 *seg) {
    const int nc0 = st.nc[0], nc1 = st.nc[1], nc2 = st.nc[2], w1n = 2 * st.m[1] + 1;
    const int nimg = 2 * st.R + 1;
    const int rpl = (rn + LANES - 1) / LANES;  // rows per lane, contiguous: the table keeps row order
    const int rb = r0 + sub * rpl, re = min(rb + rpl, r0 + rn);
    int zl[RPL], zh[RPL], z0[RPL], z1[RPL];
    bool ok[RPL];
    int cnt = 0;
    {
        int d0 = rb / w1n, d1 = rb - (rb / w1n) * w1n;  // row rb at offsets (d0, d1); later rows by counting
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            ok[q] = live && rb + q < re && stencil_row(st, c, b, d0, d1, zl[q], zh[q]);
            z0[q] = ok[q] ? image_index(zl[q], nc2) : 0;
            z1[q] = ok[q] ? image_index(zh[q], nc2) : -1;
            cnt += z1[q] - z0[q] + 1;
            if (++d1 == w1n) {
                d1 = 0;
                ++d0;
            }
        }
    }
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < LANES; o <<= 1) {
        const int v = __shfl_up(incl, o, LANES);
        if (sub >= o) incl += v;
    }
    int pos = incl - cnt;
    int d0 = rb / w1n, d1 = rb - (rb / w1n) * w1n;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        if (ok[q]) {
            const int u0 = b.ci[0] + d0 - st.m[0], i0 = image_index(u0, nc0), b0 = u0 - i0 * nc0;
            const int u1 = b.ci[1] + d1 - st.m[1], i1 = image_index(u1, nc1), b1 = u1 - i1 * nc1;
            const int rowbase = row_rank(b0, b1, nc0, nc1) * nc2;
            for (int i2 = z0[q]; i2 <= z1[q]; ++i2) {
                const int za = max(zl[q], i2 * nc2) - i2 * nc2, zb = min(zh[q], i2 * nc2 + nc2 - 1) - i2 * nc2;
                const int jb = start[rowbase + za], je = start[rowbase + zb + 1];
                const uint32_t img = (uint32_t)(((i0 + st.R) * nimg + (i1 + st.R)) * nimg + (i2 + st.R));
                seg[pos++] = make_int2(jb, (int)((uint32_t)(je - jb) | (img << SEG_LEN_BITS)));
            }
        }
        if (++d1 == w1n) {
            d1 = 0;
            ++d0;
        }
    }
    return live ? __shfl(incl, LANES - 1, LANES) : 0;
}

// lattice shift n of image index k in [0, (2R+1)^3)
__device__ inline void image_of(int k, int R, int &n0, int &n1, int &n2) {
    const int nimg = 2 * R + 1;
    n0 = k / (nimg * nimg) - R;
    n1 = (k / nimg) % nimg - R;
    n2 = k % nimg - R;
}

// position of one lane in the concatenated segments of its atom: segment s, offset off
struct SegWalk {
    int s, off, ns;
    int2 e;
    __device__ SegWalk(const int2 *seg, int ns_, int start_off) : s(0), off(start_off), ns(ns_) {
        e = ns > 0 ? seg[0] : make_int2(0, 0);
        settle(seg);
    }
    __device__ bool valid() const { return s < ns; }
    __device__ int atom() const { return e.x + off; }
    __device__ int image() const { return (int)((uint32_t)e.y >> SEG_LEN_BITS); }
    __device__ void settle(const int2 *seg) {  // move into the segment that holds offset off
        while (s < ns) {
            const int len = (int)((uint32_t)e.y & SEG_LEN_MASK);
            if (off < len) break;
            off -= len;
            if (++s < ns) e = seg[s];
        }
    }
    __device__ void advance(const int2 *seg, int stride) {
        off += stride;
        settle(seg);
    }
};

// image bits of n = (0, 0, 0)
constexpr uint32_t IMAGE_ZERO = 3u | (3u << 3) | (3u << 6);

// Displacement to the neighbour j (position pj) encoded in e.  Without a lattice
// shift the FP32 difference is the correctly rounded value, i.e. bitwise the FP64
// result rounded once; only pairs across the periodic seam take the FP64 path.
__device__ inline float3 pair_displacement(float4 pi, float4 pj, uint32_t e, const Cell &c) {
    if ((e >> IDX_BITS) == IMAGE_ZERO) return make_float3(pj.x - pi.x, pj.y - pi.y, pj.z - pi.z);
    int n1, n2, n3;
    nb_image(e, n1, n2, n3);
    return ImageShift(c, n1, n2, n3).exact(pi, pj);
}

// displacement to the neighbour encoded in e, from atom i at position pi
__device__ inline float3 displacement(float4 pi, const float4 *__restrict__ xyzt, uint32_t e, const Cell &c) {
    return pair_displacement(pi, xyzt[nb_index(e)], e, c);
}

// erfc(x) for x >= 0 given e = exp(-x^2), by the five-term formula of Abramowitz and
// Stegun (Handbook of Mathematical Functions, 7.1.26), absolute error at most 1.5e-7:
// erfc(x) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) e, t = 1 / (1 + p x).  Where the
// caller needs exp(-x^2) anyway this costs one reciprocal and five FMAs.
__device__ inline float erfc_as(float x, float e) {
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));  // v_rcp_f32, 1 ulp
    float p = 1.061405429f;
    p = fmaf(p, t, -1.453152027f);
    p = fmaf(p, t, 1.421413741f);
    p = fmaf(p, t, -0.284496736f);
    p = fmaf(p, t, 0.254829592f);
    return t * p * e;
}

__device__ inline int species_of(float4 p) { return __float_as_int(p.w); }

// Workgroup b of a 1D grid runs on XCD b % 8 (round-robin placement), and each XCD has
// its own L2.  Kernels that read their neighbours' data use the logical block below,
// which gives every XCD one contiguous range of blocks, i.e. spatially close atoms in
// the bin-sorted order, so that neighbour rows are re-read from that XCD's L2.
constexpr int N_XCD = 8;
__device__ inline int xcd_block() {
    const int b = blockIdx.x, nb = gridDim.x;
    const int x = b % N_XCD, k = b / N_XCD, q = nb / N_XCD, r = nb % N_XCD;
    return x * q + (x < r ? x : r) + k;
}

// ---------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Sums NV per-thread FP64 values over a block of RED_THREADS threads and writes
// them to partials[blockIdx.x * NV + k].  The final sum over blocks is done in a
// fixed order by reduce_partials, so results are run-to-run deterministic.
template <int NV>
__device__ inline void block_partials(double (&v)[NV], double *__restrict__ partials) {
    __shared__ double red[RED_THREADS / 64][NV];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = wave_sum(v[k]);
        if (lane == 0) red[wid][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < RED_THREADS / 64; ++w) s += red[w][threadIdx.x];
        partials[(size_t)blockIdx.x * NV + threadIdx.x] = s;
    }
}

// ---------------------------------------------------------------- scalar slots
// Global FP64 scalars kept in the workspace (indices into Scalars::v).
enum ScalarSlot : int {
    S_UNEP = 0,            // sum_i U_i               } written together
    S_SUMQ = 1,            // sum_i q_raw             }
    S_DELTA = 2,           // shift delta with q'_i = q_i + delta
    S_UREAL = 3,           // real-space energy       } written together
    S_QSQ = 4,             // sum_i q'^2              }
    S_WREAL = 5,           // 9: real-space virial    }
    S_UK = 14,             // reciprocal energy       } written together
    S_WK = 15,             // 9: reciprocal virial    }
    S_SUMPHI = 24,         // sum_i phi_i
    S_PHIBAR = 25,         // mean phi
    S_WNEP = 26,           // 9: many-body virial from the partial forces
    S_POL = 35,            // 3: polarization
    S_CENT = 38,           // 3: centroid of the caller's positions (isolated systems)
    S_COUNT = 41
};

}  // namespace qnep
