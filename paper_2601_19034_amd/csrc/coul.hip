// Electrostatics on the corrected screened charges q' = q + delta:
//  * real space (mode 1, Sec. 2.2.1 Eq. 6; static pair force Eq. 15): per-atom
//    potential phi^r_i = k_e sum_j q'_j erfc(alpha r)/r, static force and virial;
//  * direct Ewald reciprocal part (Sec. 2.2.2 Eqs. 7-9, Sec. 2.3.2 Eqs. 18, 21, 22)
//    over the half set of wave vectors (S(-k) = S(k)*), with phases k.r = 2 pi n.s
//    formed in FP64 turns and reduced to [-1/2, 1/2] before the FP32 sin/cos;
//  * self and background terms (Sec. 2.2.3 Eq. 10) and the mean potential used by
//    the chain rule through the neutrality correction.
#include "plan.h"

namespace qnep {

// ---------------------------------------------------------------- real space
// RS_LANES lanes share one sorted atom i and walk the segments of its bin stencil
// (trimmed to the cutoff sphere in orthorhombic cells) with stride RS_LANES.  A
// candidate is decided by its FP32 displacement; the pair terms are evaluated without
// a branch (a candidate outside the cutoff, or i itself, gets weight zero) and give
// phi^r_i, the static pair force
// F_i = -k_e q'_i sum_j q'_j [erfc(a r)/r + 2a e^{-a^2 r^2}/sqrt(pi)] r_ij / r^2
// and the pair virial (each unordered pair is seen from both atoms with weight 1/2).
constexpr int RS_LANES = 8;
constexpr int RS_APB = 256 / RS_LANES;  // atoms per work-group
constexpr int RS_SEG = 64;              // segments of one atom held in LDS at a time
static_assert(RS_LANES <= PARTIALS_LANES_MAX, "partials buffer sized for PARTIALS_LANES_MAX lanes per atom");

// positions with the corrected charge q' in w: one 16-byte load per candidate
__global__ void k_pack_charges(int N, const float4 *__restrict__ xyzt, const float *__restrict__ qraw,
                               const double *__restrict__ scalars, float4 *__restrict__ xyzq) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float4 p = xyzt[i];
    xyzq[i] = make_float4(p.x, p.y, p.z, qraw[i] + (float)scalars[S_DELTA]);
}

// one candidate j (image shift sh) of atom i; w = 0 discards it
__device__ __forceinline__ void rs_pair(const float4 &pi, const float4 &pj, const float4 &sh, float w, float rc2f,
                                        float alpha, float c2, float (&acc)[10]) {
    // FP32 displacement: exactly antisymmetric in (i, j); across the seam its error
    // (~ulp of the box length) is negligible for this soft pair term
    const float dx = (pj.x - pi.x) + sh.x, dy = (pj.y - pi.y) + sh.y, dz = (pj.z - pi.z) + sh.z;
    const float r2 = dx * dx + dy * dy + dz * dz;
    const bool in = r2 < rc2f && r2 > 0.0f;  // r2 = 0 only for i itself
    const float qj = in ? pj.w * w : 0.0f;
    const float rr = in ? r2 : 1.0f;
    const float ir = __builtin_amdgcn_rsqf(rr);
    const float ar = alpha * (rr * ir);
    const float ex = __expf(-ar * ar);
    const float ec = erfc_as(ar, ex);
    const float eir = ec * ir;
    acc[0] = fmaf(qj, eir, acc[0]);
    const float B = qj * fmaf(c2, ex, eir) * ir * ir;
    const float bx = B * dx, by = B * dy, bz = B * dz;
    acc[1] += bx;
    acc[2] += by;
    acc[3] += bz;
    acc[4] = fmaf(bx, dx, acc[4]);
    acc[5] = fmaf(by, dy, acc[5]);
    acc[6] = fmaf(bz, dz, acc[6]);
    acc[7] = fmaf(bx, dy, acc[7]);
    acc[8] = fmaf(bx, dz, acc[8]);
    acc[9] = fmaf(by, dz, acc[9]);
}

__global__ __launch_bounds__(256, 7) void k_real_space(int N, const float4 *__restrict__ xyzq, Cell c, Stencil st,
                                                    const int *__restrict__ start, double rc2,
                                                    const float *__restrict__ qraw,
                                                    const double *__restrict__ scalars, float alpha,
                                                    float *__restrict__ phi, float *__restrict__ Fst,
                                                    float *__restrict__ Vat, double *__restrict__ partials) {
    __shared__ int2 seg[RS_APB][RS_SEG];
    __shared__ float4 shift_tab[SEG_NIMG];
    const int nimg = 2 * st.R + 1;
    for (int k = threadIdx.x; k < nimg * nimg * nimg; k += blockDim.x) {
        int n0, n1, n2;
        image_of(k, st.R, n0, n1, n2);
        const ImageShift sh(c, n0, n1, n2);
        shift_tab[k] = make_float4(sh.fx, sh.fy, sh.fz, 0.0f);
    }
    const int a = threadIdx.x / RS_LANES, sub = threadIdx.x % RS_LANES;
    const int i = xcd_block() * RS_APB + a;
    const bool live = i < N;
    const float4 pi = xyzq[live ? i : 0];
    const AtomBin ab = atom_bin(pi, c, st);
    const float rc2f = (float)rc2;
    const float c2 = 2.0f * alpha * 0.5641895835477563f;  // 2 alpha / sqrt(pi)
    float acc[10];  // phi, B r (3), B r r (xx yy zz xy xz yz)
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[k] = 0.f;
    __syncthreads();  // lattice shifts in place
    // an atom's segment table is written and read by the atom's own lanes (one wave)
    for (int r0 = 0; r0 < st.nrows; r0 += st.rows_chunk) {  // the same trip count in every lane
        wave_lds_sync();  // the previous chunk's walk is done with the table
        const int ns = stencil_segments_kept<RS_LANES, RS_SEG / 2 / RS_LANES>(
            st, c, ab, live, sub, r0, min(st.rows_chunk, st.nrows - r0), start, seg[a]);
        wave_lds_sync();
        // this lane takes candidates sub, sub + RS_LANES, ... of the concatenation, two
        // per pass with both loads issued before either is used
        SegWalk wk(seg[a], ns, sub);
        while (wk.valid()) {
            const int jA = wk.atom(), gA = wk.image();
            wk.advance(seg[a], RS_LANES);
            const bool hasB = wk.valid();
            const int jB = hasB ? wk.atom() : jA, gB = hasB ? wk.image() : gA;
            if (hasB) wk.advance(seg[a], RS_LANES);
            const float4 pa = xyzq[jA], pb = xyzq[jB];
            const float4 sa = shift_tab[gA], sb = shift_tab[gB];
            rs_pair(pi, pa, sa, 1.0f, rc2f, alpha, c2, acc);
            rs_pair(pi, pb, sb, hasB ? 1.0f : 0.0f, rc2f, alpha, c2, acc);
        }
    }
#pragma unroll
    for (int k = 0; k < 10; ++k)
#pragma unroll
        for (int o = RS_LANES / 2; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o, 64);
    double red[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (live && sub == 0) {
        const float qi = qraw[i] + (float)scalars[S_DELTA];
        const float ke = (float)KE;
        phi[i] = ke * acc[0];
        Fst[i] = -ke * qi * acc[1];
        Fst[(size_t)N + i] = -ke * qi * acc[2];
        Fst[(size_t)2 * N + i] = -ke * qi * acc[3];
        red[0] = 0.5 * (double)qi * (double)(ke * acc[0]);
        red[1] = (double)qi * (double)qi;
        const double hw = 0.5 * KE * (double)qi;
        red[2] = hw * acc[4]; red[3] = hw * acc[7]; red[4] = hw * acc[8];
        red[5] = hw * acc[7]; red[6] = hw * acc[5]; red[7] = hw * acc[9];
        red[8] = hw * acc[8]; red[9] = hw * acc[9]; red[10] = hw * acc[6];
        if (Vat) {  // per atom: half of each pair virial (xx yy zz xy xz yz)
            const float hwf = 0.5f * ke * qi;
            Vat[i] = hwf * acc[4];
            Vat[(size_t)N + i] = hwf * acc[5];
            Vat[(size_t)2 * N + i] = hwf * acc[6];
            Vat[(size_t)3 * N + i] = hwf * acc[7];
            Vat[(size_t)4 * N + i] = hwf * acc[8];
            Vat[(size_t)5 * N + i] = hwf * acc[9];
        }
    }
    block_partials<11>(red, partials);
}

hipError_t launch_real_space(const Plan &p) {
    float *Vat = p.out.virial_atom ? p.Vat : nullptr;
    if (p.mode != 1) {
        hipError_t e = fill_zero(p.phi, sizeof(float) * (size_t)p.N, p.stream);
        if (e == hipSuccess && Vat) e = fill_zero(Vat, sizeof(float) * 6 * (size_t)p.N, p.stream);
        if (e != hipSuccess) return e;
        return fill_zero(p.Fst, sizeof(float) * 3 * (size_t)p.N, p.stream);
    }
    hipLaunchKernelGGL(k_pack_charges, dim3((p.N + 255) / 256), dim3(256), 0, p.stream, p.N, p.xyzt, p.qraw,
                       p.scalars, p.xyzq);
    stage_mark(p, ST_OTHER, 1);
    Stencil st;
    if (!stencil_setup(st, p.nc, p.mC, p.cell.h, p.rc_coul, RS_SEG)) return hipErrorInvalidValue;
    const int G = (p.N + RS_APB - 1) / RS_APB;
    hipLaunchKernelGGL(k_real_space, dim3(G), dim3(256), 0, p.stream, p.N, p.xyzq, p.cell, st, p.cell_start,
                       p.rc_coul * p.rc_coul, p.qraw, p.scalars, (float)p.alpha, p.phi, p.Fst, Vat, p.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    stage_mark(p, ST_REAL, 1);
    return reduce_partials(p, G, 11, S_UREAL, false);  // S_UREAL, S_QSQ, S_WREAL[9]
}

// ---------------------------------------------------------------- isolated systems
// Plain Coulomb sum over all pairs of an isolated system (the real-space sum of Eq. 6
// without the splitting and without images): phi_i = k_e sum_{j != i} q'_j / r_ij, the
// static pair forces and the pair virial, each thread one atom against tiles of all
// atoms staged in LDS.  Writes the same outputs and partials as the real-space kernel.
constexpr int DC_TILE = 256;

__global__ __launch_bounds__(256) void k_direct_coulomb(int N, const float4 *__restrict__ xyzq,
                                                        const float *__restrict__ qraw,
                                                        const double *__restrict__ scalars,
                                                        float *__restrict__ phi, float *__restrict__ Fst,
                                                        float *__restrict__ Vat, double *__restrict__ partials) {
    __shared__ float4 tile[DC_TILE];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < N;
    const float4 pi = xyzq[live ? i : 0];
    float acc[10];  // phi, B r (3), B r r (xx yy zz xy xz yz)
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[k] = 0.f;
    for (int t0 = 0; t0 < N; t0 += DC_TILE) {
        __syncthreads();
        const int j0 = t0 + threadIdx.x;
        tile[threadIdx.x] = j0 < N ? xyzq[j0] : make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        const int m = min(DC_TILE, N - t0);
        for (int u = 0; u < m; ++u) {
            const float4 pj = tile[u];
            const float dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            const bool other = t0 + u != i;
            const float qj = other ? pj.w : 0.0f;
            const float ir = __builtin_amdgcn_rsqf(other ? r2 : 1.0f);
            acc[0] = fmaf(qj, ir, acc[0]);
            const float B = qj * ir * ir * ir;
            const float bx = B * dx, by = B * dy, bz = B * dz;
            acc[1] += bx;
            acc[2] += by;
            acc[3] += bz;
            acc[4] = fmaf(bx, dx, acc[4]);
            acc[5] = fmaf(by, dy, acc[5]);
            acc[6] = fmaf(bz, dz, acc[6]);
            acc[7] = fmaf(bx, dy, acc[7]);
            acc[8] = fmaf(bx, dz, acc[8]);
            acc[9] = fmaf(by, dz, acc[9]);
        }
    }
    double red[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (live) {
        const float qi = qraw[i] + (float)scalars[S_DELTA];
        const float ke = (float)KE;
        phi[i] = ke * acc[0];
        Fst[i] = -ke * qi * acc[1];
        Fst[(size_t)N + i] = -ke * qi * acc[2];
        Fst[(size_t)2 * N + i] = -ke * qi * acc[3];
        red[0] = 0.5 * (double)qi * (double)(ke * acc[0]);
        const double hw = 0.5 * KE * (double)qi;
        red[2] = hw * acc[4]; red[3] = hw * acc[7]; red[4] = hw * acc[8];
        red[5] = hw * acc[7]; red[6] = hw * acc[5]; red[7] = hw * acc[9];
        red[8] = hw * acc[8]; red[9] = hw * acc[9]; red[10] = hw * acc[6];
        if (Vat) {
            const float hwf = 0.5f * ke * qi;
            Vat[i] = hwf * acc[4];
            Vat[(size_t)N + i] = hwf * acc[5];
            Vat[(size_t)2 * N + i] = hwf * acc[6];
            Vat[(size_t)3 * N + i] = hwf * acc[7];
            Vat[(size_t)4 * N + i] = hwf * acc[8];
            Vat[(size_t)5 * N + i] = hwf * acc[9];
        }
    }
    block_partials<11>(red, partials);
}

hipError_t launch_direct_coulomb(const Plan &p) {
    hipLaunchKernelGGL(k_pack_charges, dim3((p.N + 255) / 256), dim3(256), 0, p.stream, p.N, p.xyzt, p.qraw,
                       p.scalars, p.xyzq);
    const int G = (p.N + 255) / 256;
    hipLaunchKernelGGL(k_direct_coulomb, dim3(G), dim3(256), 0, p.stream, p.N, p.xyzq, p.qraw, p.scalars, p.phi,
                       p.Fst, p.out.virial_atom ? p.Vat : nullptr, p.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    stage_mark(p, ST_REAL, 2);
    return reduce_partials(p, G, 11, S_UREAL, false);  // S_UREAL, S_QSQ (zero: no self term), S_WREAL[9]
}

// FP64 partials of the centroid of the caller's positions (Born charges of an isolated system)
__global__ __launch_bounds__(256) void k_centroid(int N, const float *__restrict__ pos, double *__restrict__ partials) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double red[3] = {0.0, 0.0, 0.0};
    if (i < N)
        for (int a = 0; a < 3; ++a) red[a] = (double)pos[(size_t)a * N + i];
    block_partials<3>(red, partials);
}

hipError_t launch_centroid(const Plan &p) {
    const int G = (p.N + 255) / 256;
    hipLaunchKernelGGL(k_centroid, dim3(G), dim3(256), 0, p.stream, p.N, p.pos, p.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_partials(p, G, 3, S_CENT, false);  // sums; the assembly divides by N
}

// ---------------------------------------------------------------- Ewald
// fractional coordinates wrapped to [0, 1) in FP64
__device__ inline void frac_coords(double x, double y, double z, const Cell &c, double &s0, double &s1,
                                   double &s2) {
    s0 = x * c.hinv[0] + y * c.hinv[3] + z * c.hinv[6];
    s1 = x * c.hinv[1] + y * c.hinv[4] + z * c.hinv[7];
    s2 = x * c.hinv[2] + y * c.hinv[5] + z * c.hinv[8];
    s0 -= floor(s0);
    s1 -= floor(s1);
    s2 -= floor(s2);
}

// cos and sin of 2 pi n.s
__device__ inline void phase_cs(int n0, int n1, int n2, double s0, double s1, double s2, float &cs, float &sn) {
    double t = (double)n0 * s0 + (double)n1 * s1 + (double)n2 * s2;
    t -= rint(t);
    sincospif(2.0f * (float)t, &sn, &cs);
}

// ---------------------------------------------------------------- Ewald on the matrix cores
// The half set is stored in rows: for every (n0, n1) the wave vectors with consecutive
// n2 >= 0 inside the cutoff sphere, described by (n0, n1, first n2, count) and the index
// of the row's first wave vector; empty rows are left out.  With the per-atom phase
// factors X_j(n0) = e^{-2 pi i n0 s0_j}, Y_j(n1), Z_j(n2) (s the fractional
// coordinates) the structure factor of a row r and the per-atom sums separate:
//   S(r, n2) = sum_j [q'_j X_j(n0_r) Y_j(n1_r)] Z_j(n2),
//   sum_k w(k) G S e^{i k.r_i} = sum_n2 conj Z_i(n2) sum_r U(r, n2) conj(X_i Y_i)(r),
// U = w G S with w = 1 (potential) and k_x, k_y, k_z (force).  The first is a complex
// (rows x atoms)(atoms x n2) product, the second a (channels, n2) x rows x atoms
// product; both run on v_mfma_f32_16x16x4f32 (FP32 operands and accumulation).  A
// complex product a b takes real steps over K = (two complex terms) x (re, im) with A
// arranged as [[a_re, -a_im], [a_im, a_re]] on the output rows (re, im).
// Lane layout of v_mfma_f32_16x16x4f32 (wave64, lane l): A[i][k] at i = l % 16,
// k = l / 16; B[k][j] at j = l % 16, k = l / 16; D[i][j] at j = l % 16, i = 4 (l / 16) + e.
typedef float floatx4 __attribute__((ext_vector_type(4)));

// One block.  Rows in the order of the (n0, n1) box with n1 slowest.
__global__ void k_kvector_rows(Cell c, int M0, int M1, int M2, double kmax2, int inclusive, double alpha,
                               double vol, int64_t cap, int row_cap, float4 *__restrict__ kv,
                               int4 *__restrict__ kn, int4 *__restrict__ rows, int *__restrict__ rowoff,
                               int *__restrict__ kcount, int *__restrict__ nrows) {
    __shared__ int scan_k[1024], scan_r[1024];
    __shared__ int base_k, base_r;
    if (threadIdx.x == 0) base_k = base_r = 0;
    __syncthreads();
    const int n0w = 2 * M0 + 1, n1w = 2 * M1 + 1;
    const int box = n0w * n1w;
    for (int r0 = 0; r0 < box; r0 += 1024) {
        const int r = r0 + threadIdx.x;
        int a0 = 0, a1 = 0, lo = 0, cnt = 0;
        if (r < box) {
            a1 = r / n0w - M1;
            a0 = r % n0w - M0;
            // half set: n2 > 0, or n2 = 0 with (n1 > 0, or n1 = 0 and n0 > 0)
            const int first = (a1 > 0 || (a1 == 0 && a0 > 0)) ? 0 : 1;
            int hi = -1;
            lo = -1;
            for (int a2 = first; a2 <= M2; ++a2) {  // |k|^2 is convex in n2: one interval
                const double kx = 2.0 * PI_D * (c.hinv[0] * a0 + c.hinv[1] * a1 + c.hinv[2] * a2);
                const double ky = 2.0 * PI_D * (c.hinv[3] * a0 + c.hinv[4] * a1 + c.hinv[5] * a2);
                const double kz = 2.0 * PI_D * (c.hinv[6] * a0 + c.hinv[7] * a1 + c.hinv[8] * a2);
                const double k2 = kx * kx + ky * ky + kz * kz;
                const bool keep = inclusive ? (k2 <= kmax2 * (1.0 + 1e-9)) : (k2 < kmax2 * (1.0 - 1e-9));
                if (keep) {
                    if (lo < 0) lo = a2;
                    hi = a2;
                }
            }
            cnt = lo < 0 ? 0 : hi - lo + 1;
        }
        const int nr = cnt > 0 ? 1 : 0;
        scan_k[threadIdx.x] = cnt;
        scan_r[threadIdx.x] = nr;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int tk = threadIdx.x >= (unsigned)o ? scan_k[threadIdx.x - o] : 0;
            const int tr = threadIdx.x >= (unsigned)o ? scan_r[threadIdx.x - o] : 0;
            __syncthreads();
            scan_k[threadIdx.x] += tk;
            scan_r[threadIdx.x] += tr;
            __syncthreads();
        }
        const int kb = base_k + scan_k[threadIdx.x] - cnt, rb = base_r + scan_r[threadIdx.x] - nr;
        for (int m = 0; m < cnt; ++m) {
            const int64_t pos = (int64_t)kb + m;
            if (pos >= cap) break;
            const int a2 = lo + m;
            const double kx = 2.0 * PI_D * (c.hinv[0] * a0 + c.hinv[1] * a1 + c.hinv[2] * a2);
            const double ky = 2.0 * PI_D * (c.hinv[3] * a0 + c.hinv[4] * a1 + c.hinv[5] * a2);
            const double kz = 2.0 * PI_D * (c.hinv[6] * a0 + c.hinv[7] * a1 + c.hinv[8] * a2);
            const double k2 = kx * kx + ky * ky + kz * kz;
            const double G = 2.0 * PI_D / vol * exp(-k2 / (4.0 * alpha * alpha)) / k2;
            kv[pos] = make_float4((float)kx, (float)ky, (float)kz, (float)G);
            kn[pos] = make_int4(a0, a1, a2, 0);
        }
        if (nr && rb < row_cap) {
            // a row past the wave-vector capacity is emptied (never happens when the
            // host count and this one agree, which they do up to the same tie rule)
            const bool fits = (int64_t)kb + cnt <= cap;
            rows[rb] = make_int4(a0, a1, lo, fits ? cnt : 0);
            rowoff[rb] = fits ? kb : 0;
        }
        __syncthreads();
        if (threadIdx.x == 1023) {
            base_k += scan_k[1023];
            base_r += scan_r[1023];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *kcount = base_k < cap ? base_k : (int)cap;
        *nrows = base_r < row_cap ? base_r : row_cap;
    }
}

__device__ inline float2 turn_phase(double t) {  // e^{-2 pi i t}
    t -= rint(t);
    float sn, cs;
    sincospif(2.0f * (float)t, &sn, &cs);
    return make_float2(cs, -sn);
}

// Phase tables X[n0 + M0][j], Y[n1 + M1][j] (|n| <= M), Z[n2][j] (0 <= n2 < NZP, zero
// past M2), each entry from the FP64 product n s reduced to [-1/2, 1/2].
__global__ __launch_bounds__(256) void k_ewald_tables(int N, const float4 *__restrict__ xyzt, Cell c, int M0,
                                                      int M1, int M2, int NZP, float2 *__restrict__ X,
                                                      float2 *__restrict__ Y, float2 *__restrict__ Z) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const float4 pa = xyzt[j];
    double s0, s1, s2;
    frac_coords(pa.x, pa.y, pa.z, c, s0, s1, s2);
    for (int n = -M0; n <= M0; ++n) X[(size_t)(n + M0) * N + j] = turn_phase((double)n * s0);
    for (int n = -M1; n <= M1; ++n) Y[(size_t)(n + M1) * N + j] = turn_phase((double)n * s1);
    for (int n = 0; n < NZP; ++n) Z[(size_t)n * N + j] = n <= M2 ? turn_phase((double)n * s2) : make_float2(0.f, 0.f);
}

__device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

// Partial structure factors: block (row block of 64, atom chunk, pair of n2 tiles).  Per
// stage of ESK_SUB atoms the block forms P(r, j) = q'_j X_j(n0_r) Y_j(n1_r) for its rows
// and copies Z_j(n2) for its n2 into LDS; each wave then multiplies 16 complex rows (two
// M-tiles of 8 rows x (re, im)) by 32 n2 (two N-tiles), two atoms per step, from LDS.
// Spart[chunk][row][n2][re, im].
constexpr int ESK_WROWS = 16, ESK_BROWS = 4 * ESK_WROWS, ESK_SUB = 64, ESK_LD = ESK_SUB + 1;
__global__ __launch_bounds__(256) void k_ewald_sk_mfma(int N, int chunk, const float *__restrict__ qraw,
                                                       const double *__restrict__ scalars,
                                                       const int4 *__restrict__ rows,
                                                       const int *__restrict__ nrows_p, int row_cap, int NZP,
                                                       int M0, int M1, const float2 *__restrict__ X,
                                                       const float2 *__restrict__ Y, const float2 *__restrict__ Z,
                                                       float *__restrict__ Spart) {
    __shared__ float2 Ps[ESK_BROWS][ESK_LD];
    __shared__ float2 Zs[32][ESK_LD];
    __shared__ int2 rowxy[ESK_BROWS];  // (n0 + M0, n1 + M1), or -1 past the last row
    const int nrows = *nrows_p;
    const int brow0 = blockIdx.x * ESK_BROWS;
    if (brow0 >= nrows) return;  // the whole block
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int jb = blockIdx.y * chunk, je = min(N, jb + chunk);
    const int nt0 = blockIdx.z * 32;  // first n2 of this block
    const float delta = (float)scalars[S_DELTA];
    if (threadIdx.x < ESK_BROWS) {
        const int r = brow0 + threadIdx.x;
        const int4 e = rows[r < nrows ? r : 0];
        rowxy[threadIdx.x] = r < nrows ? make_int2(e.x + M0, e.y + M1) : make_int2(-1, -1);
    }
    const int m = l & 15, kk = l >> 4;
    const int o = m >> 3, rho = m & 7, jj = kk >> 1, p = kk & 1;
    // A = [[P_re, -P_im], [P_im, P_re]]: picks of (P_re, P_im) and a sign
    const bool take_re = (o == p);
    const float sgn = (o == 0 && p == 1) ? -1.0f : 1.0f;
    floatx4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[a][t] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int wr = wave * ESK_WROWS;
    for (int j0 = jb; j0 < je; j0 += ESK_SUB) {
        __syncthreads();  // row table in place / the previous stage consumed
        const int ja = threadIdx.x & (ESK_SUB - 1), j = j0 + ja;
        const bool jok = j < je;
        const int jc = jok ? j : jb;
        const float q = jok ? qraw[jc] + delta : 0.0f;
        for (int r = threadIdx.x / ESK_SUB; r < ESK_BROWS; r += 256 / ESK_SUB) {
            const int2 xy = rowxy[r];
            float2 v = make_float2(0.f, 0.f);
            if (xy.x >= 0) {
                const float2 pr = cmul(X[(size_t)xy.x * N + jc], Y[(size_t)xy.y * N + jc]);
                v = make_float2(q * pr.x, q * pr.y);
            }
            Ps[r][ja] = v;
        }
        for (int n = threadIdx.x / ESK_SUB; n < 32; n += 256 / ESK_SUB) {
            const int n2 = nt0 + n;
            Zs[n][ja] = (jok && n2 < NZP) ? Z[(size_t)n2 * N + jc] : make_float2(0.f, 0.f);
        }
        __syncthreads();
#pragma unroll 4
        for (int s2 = 0; s2 < ESK_SUB; s2 += 2) {
            const float2 pa = Ps[wr + rho][s2 + jj], pb = Ps[wr + 8 + rho][s2 + jj];
            const float2 za = Zs[m][s2 + jj], zb = Zs[16 + m][s2 + jj];
            const float aa = sgn * (take_re ? pa.x : pa.y), ab = sgn * (take_re ? pb.x : pb.y);
            const float ba = p ? za.y : za.x, bb = p ? zb.y : zb.x;
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(aa, ba, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(aa, bb, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ab, ba, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(ab, bb, acc[1][1], 0, 0, 0);
        }
    }
    // D[i][n]: n = l % 16, i = 4 (l / 16) + e: output part i / 8, complex row i % 8
    float *out = Spart + (size_t)blockIdx.y * row_cap * NZP * 2;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int n2 = nt0 + 16 * t + (l & 15);
            if (n2 >= NZP) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 4 * (l >> 4) + e;
                const int row = brow0 + wr + 8 * a + (i & 7);
                if (row < nrows) out[((size_t)row * NZP + n2) * 2 + (i >> 3)] = acc[a][t][e];
            }
        }
}

// S(k) = sum over chunks (FP64) for every (row, n2) of the box; energy 2 k_e G |S|^2
// and virial 2 k_e G |S|^2 B(k) over the half set; Sk in the order of the wave-vector
// list; U[row][c][n2] = w_c G S (w = 1, k_x, k_y, k_z), zero outside the row's range.
__global__ __launch_bounds__(256) void k_ewald_reduce_box(int nchunks, const float *__restrict__ Spart,
                                                          const int4 *__restrict__ rows,
                                                          const int *__restrict__ rowoff,
                                                          const int *__restrict__ nrows_p, int row_cap, int NZP,
                                                          int NZ4, const float4 *__restrict__ kv, double alpha,
                                                          float2 *__restrict__ Sk, float2 *__restrict__ U,
                                                          double *__restrict__ partials) {
    const int nrows = *nrows_p;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int row = (int)(t / NZP), n2 = (int)(t - (int64_t)row * NZP);
    double red[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (row < nrows) {
        double re = 0.0, im = 0.0;
        for (int ch = 0; ch < nchunks; ++ch) {
            const float *v = Spart + (((size_t)ch * row_cap + row) * NZP + n2) * 2;
            re += v[0];
            im += v[1];
        }
        const int4 e = rows[row];
        const bool in = n2 >= e.z && n2 < e.z + e.w;
        float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
        if (in) {
            const int k = rowoff[row] + n2 - e.z;
            q = kv[k];
            Sk[k] = make_float2((float)re, (float)im);
            const double kx = q.x, ky = q.y, kz = q.z, G = q.w;
            const double k2 = kx * kx + ky * ky + kz * kz;
            const double en = 2.0 * KE * G * (re * re + im * im);
            const double cB = 2.0 / (4.0 * alpha * alpha) + 2.0 / k2;
            const double kk[3] = {kx, ky, kz};
            red[0] = en;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) red[1 + 3 * a + b] = en * ((a == b ? 1.0 : 0.0) - cB * kk[a] * kk[b]);
        }
        if (n2 < NZ4) {
            const float gr = q.w * (float)re, gi = q.w * (float)im;  // zero outside the range
            float2 *u = U + (size_t)row * 4 * NZ4 + n2;
            u[0] = make_float2(gr, gi);
            u[NZ4] = make_float2(q.x * gr, q.x * gi);
            u[2 * NZ4] = make_float2(q.y * gr, q.y * gi);
            u[3 * NZ4] = make_float2(q.z * gr, q.z * gi);
        }
    }
    block_partials<10>(red, partials);
}

// Per-atom sums, block (atom block of 128, row chunk).  Per stage of EA_RB rows the block
// copies U of those rows and forms conj(X_i Y_i)(r) of its atoms into LDS; each wave then
// multiplies the outputs V_c(n2) of all (channel, n2) (M-tiles of 8 x (re, im)) for 32
// atoms (two N-tiles), two rows per step, from LDS, and finally forms
// sum_n2 conj Z_i(n2) V_c(n2).  Writes the row chunk's partial potential and force sums
// ephi[chunk][4][N] (summed in order by k_ewald_atoms_finish).  LDS (dynamic):
// U [EA_RB][4 NZ4] | conj(X Y) [EA_RB][128] | rows [EA_RB].
constexpr int EA_MT = 12;  // M-tiles per pass: 4 channels x NZ4 x (re, im) / 16 = NZ4 / 2
constexpr int EA_RB = 16;  // rows per stage
size_t ewald_atoms_lds_bytes(int NZ4) {
    return (size_t)EA_RB * 4 * NZ4 * sizeof(float2) + (size_t)EA_RB * 128 * sizeof(float2) + EA_RB * sizeof(int4);
}
__global__ __launch_bounds__(256) void k_ewald_atoms_mfma(int N, const int4 *__restrict__ rows,
                                                          const int *__restrict__ nrows_p, int rchunk, int NZ4,
                                                          int M0, int M1, const float2 *__restrict__ U,
                                                          const float2 *__restrict__ X, const float2 *__restrict__ Y,
                                                          const float2 *__restrict__ Z, float *__restrict__ ephi) {
    extern __shared__ float2 ea_lds[];
    const int nu = 4 * NZ4;
    float2 *Us = ea_lds;                   // [EA_RB][nu]
    float2 *Bs = Us + EA_RB * nu;          // [EA_RB][128]
    int4 *rs = reinterpret_cast<int4 *>(Bs + EA_RB * 128);
    const int nrows = *nrows_p;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int blk0 = blockIdx.x * 128, atom0 = blk0 + wave * 32;
    const int rb = blockIdx.y * rchunk, re = min(nrows, rb + rchunk);
    const int n = l & 15, kk = l >> 4, rr = kk >> 1, p = kk & 1;
    const int ia = atom0 + n, ib = atom0 + 16 + n;
    const int mtiles = NZ4 / 2;
    float sums[2][4];  // per N-tile atom: potential, force x, y, z
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
        for (int c = 0; c < 4; ++c) sums[w][c] = 0.f;
    // this lane's A element: output index gm = 16 tile + n -> part o = gm & 1 of
    // (channel, n2) = gm >> 1; A = [[U_re, -U_im], [U_im, U_re]]
    const int o = n & 1;
    const bool take_re = (o == p);
    const float sgn = (o == 0 && p == 1) ? -1.0f : 1.0f;
    // this thread's atom in the LDS stage of conj(X Y)
    const int sa = threadIdx.x & 127, sj = blk0 + sa, sjc = sj < N ? sj : 0;
    for (int t0 = 0; t0 < mtiles; t0 += EA_MT) {
        floatx4 acc[EA_MT][2];
#pragma unroll
        for (int t = 0; t < EA_MT; ++t) acc[t][0] = acc[t][1] = floatx4{0.f, 0.f, 0.f, 0.f};
        for (int r0 = rb; r0 < re; r0 += EA_RB) {
            const int nr = min(EA_RB, re - r0);
            __syncthreads();  // the previous stage consumed
            if (threadIdx.x < EA_RB) rs[threadIdx.x] = rows[threadIdx.x < nr ? r0 + threadIdx.x : r0];
            for (int k = threadIdx.x; k < EA_RB * nu; k += 256)
                Us[k] = k < nr * nu ? U[(size_t)r0 * nu + k] : make_float2(0.f, 0.f);
            __syncthreads();  // row table in place
            for (int r = threadIdx.x >> 7; r < EA_RB; r += 2) {
                float2 v = make_float2(0.f, 0.f);
                if (r < nr && sj < N) {
                    const int4 e = rs[r];
                    const float2 c = cmul(X[(size_t)(e.x + M0) * N + sjc], Y[(size_t)(e.y + M1) * N + sjc]);
                    v = make_float2(c.x, -c.y);
                }
                Bs[r * 128 + sa] = v;
            }
            __syncthreads();
            for (int s2 = 0; s2 < nr; s2 += 2) {
                const int r = s2 + rr;  // rows past nr are zero in both operands
                const float2 ca = Bs[r * 128 + wave * 32 + n], cb = Bs[r * 128 + wave * 32 + 16 + n];
                const float ba = p ? ca.y : ca.x, bb = p ? cb.y : cb.x;
                const float2 *ur = Us + r * nu;
#pragma unroll
                for (int t = 0; t < EA_MT; ++t) {
                    if (t0 + t < mtiles) {
                        const float2 u = ur[(16 * (t0 + t) + n) >> 1];
                        const float av = sgn * (take_re ? u.x : u.y);
                        acc[t][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, ba, acc[t][0], 0, 0, 0);
                        acc[t][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bb, acc[t][1], 0, 0, 0);
                    }
                }
            }
        }
        // D[i][n]: i = 4 (l / 16) + e -> gm = 16 tile + i; elements (0, 1) and (2, 3) are
        // (re, im) of V at (channel, n2) = gm >> 1 for atom n of each N-tile
        const int ica = ia < N ? ia : 0, icb = ib < N ? ib : 0;
#pragma unroll
        for (int t = 0; t < EA_MT; ++t) {
            if (t0 + t >= mtiles) continue;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int cn = (16 * (t0 + t) + 4 * kk + 2 * h) >> 1;
                const int ch = cn / NZ4, n2 = cn - ch * NZ4;
#pragma unroll
                for (int w = 0; w < 2; ++w) {
                    const float2 z = Z[(size_t)n2 * N + (w ? icb : ica)];
                    const float vr = acc[t][w][2 * h], vi = acc[t][w][2 * h + 1];
                    // (vr + i vi) conj(z): the real part for the potential, the imaginary for the force
                    const float pr = fmaf(vr, z.x, vi * z.y), pim = fmaf(vi, z.x, -vr * z.y);
                    sums[w][ch] += ch == 0 ? pr : pim;
                }
            }
        }
    }
    // the four lane groups (l / 16) hold different (channel, n2) of the same atoms
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            sums[w][c] += __shfl_xor(sums[w][c], 16, 64);
            sums[w][c] += __shfl_xor(sums[w][c], 32, 64);
        }
    if (kk == 0) {
        float *out = ephi + (size_t)blockIdx.y * 4 * N;
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const int i = w ? ib : ia;
            if (i < N)
#pragma unroll
                for (int c = 0; c < 4; ++c) out[(size_t)c * N + i] = sums[w][c];
        }
    }
}

// phi^k_i = 4 k_e sum_half G Re[S e^{i k.r_i}],  F^k_i = 4 k_e q'_i sum_half k G Im[S e^{i k.r_i}]:
// the row chunks' partial sums in chunk order, added to the real-space values
__global__ __launch_bounds__(256) void k_ewald_atoms_finish(int N, int nchunks, const float *__restrict__ ephi,
                                                            const float *__restrict__ qraw,
                                                            const double *__restrict__ scalars,
                                                            float *__restrict__ phi, float *__restrict__ Fst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    for (int ch = 0; ch < nchunks; ++ch)
#pragma unroll
        for (int c = 0; c < 4; ++c) s[c] += ephi[((size_t)ch * 4 + c) * N + i];
    const float qi = qraw[i] + (float)scalars[S_DELTA];
    const float k4 = 4.0f * (float)KE;
    phi[i] += k4 * s[0];
    Fst[i] += k4 * qi * s[1];
    Fst[(size_t)N + i] += k4 * qi * s[2];
    Fst[(size_t)2 * N + i] += k4 * qi * s[3];
}
// per-atom reciprocal virial (Eq. 20) over the half set: W^k_i = 2 k_e q'_i sum_half G
// Re[S e^{i k.r_i}] B(k), B = I - (2/(4 alpha^2) + 2/k^2) k k; added to Vat
__global__ __launch_bounds__(256) void k_ewald_virial_atoms(int N, const float4 *__restrict__ xyzt, Cell c,
                                                            float alpha, const float *__restrict__ qraw,
                                                            const double *__restrict__ scalars,
                                                            const float4 *__restrict__ kv,
                                                            const int4 *__restrict__ kn,
                                                            const float2 *__restrict__ Sk,
                                                            const int *__restrict__ kcount, float *__restrict__ Vat) {
    __shared__ int4 ln[256];
    __shared__ float4 lk[256];
    __shared__ float2 ls[256];
    const int nk = *kcount;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const float cB0 = 2.0f / (4.0f * alpha * alpha);
    double s0 = 0, s1 = 0, s2 = 0;
    if (i < N) {
        const float4 pa = xyzt[i];
        frac_coords(pa.x, pa.y, pa.z, c, s0, s1, s2);
    }
    float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // xx yy zz xy xz yz
    for (int t0 = 0; t0 < nk; t0 += 256) {
        int k = t0 + threadIdx.x;
        if (k < nk) {
            ln[threadIdx.x] = kn[k];
            lk[threadIdx.x] = kv[k];
            ls[threadIdx.x] = Sk[k];
        }
        __syncthreads();
        const int m = min(256, nk - t0);
        if (i < N) {
            for (int u = 0; u < m; ++u) {
                float cs, sn;
                int4 n = ln[u];
                phase_cs(n.x, n.y, n.z, s0, s1, s2, cs, sn);
                const float2 S = ls[u];
                const float4 q = lk[u];
                const float gre = q.w * (S.x * cs - S.y * sn);
                const float k2 = q.x * q.x + q.y * q.y + q.z * q.z;
                const float cb = gre * (cB0 + 2.0f / k2);
                v[0] = fmaf(-cb * q.x, q.x, v[0] + gre);
                v[1] = fmaf(-cb * q.y, q.y, v[1] + gre);
                v[2] = fmaf(-cb * q.z, q.z, v[2] + gre);
                v[3] = fmaf(-cb * q.x, q.y, v[3]);
                v[4] = fmaf(-cb * q.x, q.z, v[4]);
                v[5] = fmaf(-cb * q.y, q.z, v[5]);
            }
        }
        __syncthreads();
    }
    if (i < N) {
        const float f = 2.0f * (float)KE * (qraw[i] + (float)scalars[S_DELTA]);
#pragma unroll
        for (int k = 0; k < 6; ++k) Vat[(size_t)k * N + i] += f * v[k];
    }
}

hipError_t launch_ewald(const Plan &p) {
    int4 *kn = (int4 *)(p.kvec + p.nk_cap);
    const int M0 = p.nk_box[0], M1 = p.nk_box[1], M2 = p.nk_box[2];
    hipLaunchKernelGGL(k_kvector_rows, dim3(1), dim3(1024), 0, p.stream, p.cell, M0, M1, M2, p.kmax * p.kmax,
                       p.kinc, p.alpha, p.vol, p.nk_cap, p.row_cap, p.kvec, kn, p.krows, p.krowoff, p.kcount,
                       p.knrows);
    const int G = (p.N + 255) / 256;
    hipLaunchKernelGGL(k_ewald_tables, dim3(G), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell, M0, M1, M2, p.NZP,
                       p.ewX, p.ewY, p.ewZ);
    hipLaunchKernelGGL(k_ewald_sk_mfma, dim3((p.row_cap + ESK_BROWS - 1) / ESK_BROWS, p.s_chunks, (p.NZP + 31) / 32),
                       dim3(256), 0, p.stream, p.N, p.s_chunk, p.qraw, p.scalars, p.krows, p.knrows, p.row_cap,
                       p.NZP, M0, M1, p.ewX, p.ewY, p.ewZ, p.Spart);
    const int kb = (int)(((int64_t)p.row_cap * p.NZP + 255) / 256);
    hipLaunchKernelGGL(k_ewald_reduce_box, dim3(kb), dim3(256), 0, p.stream, p.s_chunks, p.Spart, p.krows,
                       p.krowoff, p.knrows, p.row_cap, p.NZP, p.NZ4, p.kvec, p.alpha, p.Sk, p.Ubox, p.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = reduce_partials(p, kb, 10, S_UK, false);  // S_UK, S_WK[9]
    if (e != hipSuccess) return e;
    stage_mark(p, ST_EWALD_SK, 5);
    hipLaunchKernelGGL(k_ewald_atoms_mfma, dim3((p.N + 127) / 128, p.r_chunks), dim3(256),
                       ewald_atoms_lds_bytes(p.NZ4), p.stream, p.N,
                       p.krows, p.knrows, p.r_chunk, p.NZ4, M0, M1, p.Ubox, p.ewX, p.ewY, p.ewZ, p.ephi);
    hipLaunchKernelGGL(k_ewald_atoms_finish, dim3(G), dim3(256), 0, p.stream, p.N, p.r_chunks, p.ephi, p.qraw,
                       p.scalars, p.phi, p.Fst);
    if (p.out.virial_atom)
        hipLaunchKernelGGL(k_ewald_virial_atoms, dim3(G), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell,
                           (float)p.alpha, p.qraw, p.scalars, p.kvec, (const int4 *)kn, p.Sk, p.kcount, p.Vat);
    stage_mark(p, ST_EWALD_ATOMS, p.out.virial_atom ? 3 : 2);
    return hipGetLastError();
}

// ---------------------------------------------------------------- potential centring
// phi_i += self (-2 k_e alpha q'_i / sqrt(pi)) and background terms (mode 1);
// FP64 partials of sum phi for the mean used in chi_i = phi_i - mean(phi).
__global__ __launch_bounds__(256) void k_phi_total(int N, int mode, float alpha, double vol, double qtot,
                                                   const float *__restrict__ qraw,
                                                   const double *__restrict__ scalars,
                                                   const float *__restrict__ theta, int64_t off_s,
                                                   float *__restrict__ phi, double *__restrict__ partials) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double red[1] = {0.0};
    if (i < N) {
        float v = phi[i];
        if (mode == 1) {
            const float qi = qraw[i] + (float)scalars[S_DELTA];
            const double Qs = qtot / (double)theta[off_s];
            v += -2.0f * (float)KE * alpha * 0.5641895835477563f * qi;
            v += (float)(-KE * PI_D * Qs / (vol * (double)alpha * (double)alpha));
            phi[i] = v;
        }
        red[0] = v;
    }
    block_partials<1>(red, partials);
}

__global__ void k_phi_mean(int N, double *__restrict__ scalars) {
    if (threadIdx.x == 0) scalars[S_PHIBAR] = scalars[S_SUMPHI] / (double)N;
}

hipError_t launch_phi_mean(const Plan &p) {
    const int G = (p.N + 255) / 256;
    hipLaunchKernelGGL(k_phi_total, dim3(G), dim3(256), 0, p.stream, p.N, p.iso ? 0 : p.mode, (float)p.alpha, p.vol, p.qtot,
                       p.qraw, p.scalars, p.theta, p.off_s, p.phi, p.partials);
    hipError_t e = reduce_partials(p, G, 1, S_SUMPHI, false);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_phi_mean, dim3(1), dim3(64), 0, p.stream, p.N, p.scalars);
    return hipGetLastError();
}

}  // namespace qnep
