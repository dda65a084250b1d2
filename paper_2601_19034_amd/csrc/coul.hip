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

__global__ __launch_bounds__(256) void k_real_space(int N, const float4 *__restrict__ xyzq, Cell c, Stencil st,
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
        const int ns = stencil_segments<RS_LANES>(st, c, ab, live, sub, r0, min(st.rows_chunk, st.nrows - r0),
                                                  start, seg[a]);
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

// The half set in rows: for every (n0, n1) the wave vectors with consecutive n2 are
// stored consecutively and described by row segments of at most EW_SEG entries,
// (n0, n1, first n2, count) and the index of their first wave vector.  Along a segment
// the phase 2 pi n.s of an atom advances by 2 pi s2 per entry, so it is formed once per
// (segment, atom) and then carried by a complex rotation.  One block.
constexpr int EW_SEG = 32;

__global__ void k_kvector_rows(Cell c, int M0, int M1, int M2, double kmax2, int inclusive, double alpha,
                               double vol, int64_t cap, int64_t seg_cap, float4 *__restrict__ kv,
                               int4 *__restrict__ kn, int4 *__restrict__ segs, int *__restrict__ segoff,
                               int *__restrict__ kcount, int *__restrict__ nseg) {
    __shared__ int scan_k[1024], scan_s[1024];
    __shared__ int base_k, base_s;
    if (threadIdx.x == 0) base_k = base_s = 0;
    __syncthreads();
    const int n0w = 2 * M0 + 1, n1w = 2 * M1 + 1;
    const int rows = n0w * n1w;
    for (int r0 = 0; r0 < rows; r0 += 1024) {
        const int r = r0 + threadIdx.x;
        int a0 = 0, a1 = 0, lo = 0, cnt = 0;
        if (r < rows) {
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
        const int ns = (cnt + EW_SEG - 1) / EW_SEG;
        scan_k[threadIdx.x] = cnt;
        scan_s[threadIdx.x] = ns;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int tk = threadIdx.x >= (unsigned)o ? scan_k[threadIdx.x - o] : 0;
            const int ts = threadIdx.x >= (unsigned)o ? scan_s[threadIdx.x - o] : 0;
            __syncthreads();
            scan_k[threadIdx.x] += tk;
            scan_s[threadIdx.x] += ts;
            __syncthreads();
        }
        const int kb = base_k + scan_k[threadIdx.x] - cnt, sb = base_s + scan_s[threadIdx.x] - ns;
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
        for (int q = 0; q < ns; ++q) {
            const int m0 = q * EW_SEG, len = min(EW_SEG, cnt - m0);
            if (sb + q >= seg_cap) break;
            // a segment past the wave-vector capacity is emptied (never happens when the
            // host count and this one agree, which they do up to the same tie rule)
            const bool fits = (int64_t)kb + m0 + len <= cap;
            segs[sb + q] = make_int4(a0, a1, lo + m0, fits ? len : 0);
            segoff[sb + q] = fits ? kb + m0 : 0;
        }
        __syncthreads();
        if (threadIdx.x == 1023) {
            base_k += scan_k[1023];
            base_s += scan_s[1023];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *kcount = base_k < cap ? base_k : (int)cap;
        *nseg = base_s < seg_cap ? base_s : (int)seg_cap;
    }
}

constexpr int EW_CHUNK = 512;

// partial structure factors by row segments: block (segment block, atom chunk); each
// thread owns one segment and carries every atom's phase along it
__global__ __launch_bounds__(256) void k_structure_factor_rows(int N, const float4 *__restrict__ xyzt, Cell c,
                                                               const float *__restrict__ qraw,
                                                               const double *__restrict__ scalars,
                                                               const int4 *__restrict__ segs,
                                                               const int *__restrict__ segoff,
                                                               const int *__restrict__ nseg, int64_t cap,
                                                               float2 *__restrict__ Spart) {
    __shared__ double sx[256], sy[256], sz[256];
    __shared__ float sq[256];
    __shared__ float2 st[256];  // (cos, sin) of 2 pi s2: the rotation along a segment
    const int ns = *nseg;
    const int sg = blockIdx.x * blockDim.x + threadIdx.x;
    const int4 g = sg < ns ? segs[sg] : make_int4(0, 0, 0, 0);
    const float delta = (float)scalars[S_DELTA];
    float re[EW_SEG], im[EW_SEG];
#pragma unroll
    for (int m = 0; m < EW_SEG; ++m) re[m] = im[m] = 0.f;
    const int a0 = blockIdx.y * EW_CHUNK, a1 = min(N, a0 + EW_CHUNK);
    for (int t0 = a0; t0 < a1; t0 += 256) {
        __syncthreads();
        const int a = t0 + threadIdx.x;
        if (a < a1) {
            const float4 pa = xyzt[a];
            double s0, s1, s2;
            frac_coords(pa.x, pa.y, pa.z, c, s0, s1, s2);
            sx[threadIdx.x] = s0;
            sy[threadIdx.x] = s1;
            sz[threadIdx.x] = s2;
            sq[threadIdx.x] = qraw[a] + delta;
            float cs, sn;
            phase_cs(0, 0, 1, s0, s1, s2, cs, sn);
            st[threadIdx.x] = make_float2(cs, sn);
        }
        __syncthreads();
        const int m = min(256, a1 - t0);
        if (sg < ns) {
            for (int u = 0; u < m; ++u) {
                float cs, sn;
                phase_cs(g.x, g.y, g.z, sx[u], sy[u], sz[u], cs, sn);
                const float q = sq[u];
                const float2 r = st[u];
#pragma unroll
                for (int e = 0; e < EW_SEG; ++e) {
                    if (e < g.w) {
                        re[e] = fmaf(q, cs, re[e]);
                        im[e] = fmaf(-q, sn, im[e]);
                        const float c2 = fmaf(cs, r.x, -sn * r.y);
                        sn = fmaf(sn, r.x, cs * r.y);
                        cs = c2;
                    }
                }
            }
        }
    }
    if (sg < ns) {
        const int k0 = segoff[sg];
#pragma unroll
        for (int e = 0; e < EW_SEG; ++e)
            if (e < g.w) Spart[(size_t)blockIdx.y * cap + k0 + e] = make_float2(re[e], im[e]);
    }
}

// S(k) = sum over chunks (FP64); energy 2 k_e G |S|^2 and virial 2 k_e G |S|^2 B(k)
__global__ __launch_bounds__(256) void k_structure_reduce(int nchunks, const float2 *__restrict__ Spart,
                                                          const float4 *__restrict__ kv,
                                                          const int *__restrict__ kcount, int64_t cap,
                                                          double alpha, float2 *__restrict__ Sk,
                                                          double *__restrict__ partials) {
    const int nk = *kcount;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double red[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (k < nk) {
        double re = 0.0, im = 0.0;
        for (int ch = 0; ch < nchunks; ++ch) {
            float2 v = Spart[(size_t)ch * cap + k];
            re += v.x;
            im += v.y;
        }
        Sk[k] = make_float2((float)re, (float)im);
        float4 q = kv[k];
        double kx = q.x, ky = q.y, kz = q.z, G = q.w;
        double k2 = kx * kx + ky * ky + kz * kz;
        double e = 2.0 * KE * G * (re * re + im * im);
        double cB = 2.0 / (4.0 * alpha * alpha) + 2.0 / k2;
        double kk[3] = {kx, ky, kz};
        red[0] = e;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) red[1 + 3 * a + b] = e * ((a == b ? 1.0 : 0.0) - cB * kk[a] * kk[b]);
    }
    block_partials<10>(red, partials);
}

// phi^k_i = 4 k_e sum_half G Re[S e^{i k.r_i}],  F^k_i = 4 k_e q'_i sum_half k G Im[S e^{i k.r_i}]
// by row segments: the segment and wave-vector data are uniform across the block
// (scalar loads); each atom's phase is formed once per segment and rotated by 2 pi s2
// along it.
__global__ __launch_bounds__(256) void k_ewald_atoms_rows(int N, const float4 *__restrict__ xyzt, Cell c,
                                                          const float *__restrict__ qraw,
                                                          const double *__restrict__ scalars,
                                                          const float4 *__restrict__ kv,
                                                          const int4 *__restrict__ segs,
                                                          const int *__restrict__ segoff,
                                                          const int *__restrict__ nseg,
                                                          const float2 *__restrict__ Sk,
                                                          float *__restrict__ phi, float *__restrict__ Fst) {
    const int ns = *nseg;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double s0 = 0, s1 = 0, s2 = 0;
    if (i < N) {
        const float4 pa = xyzt[i];
        frac_coords(pa.x, pa.y, pa.z, c, s0, s1, s2);
    }
    float rc, rs;
    phase_cs(0, 0, 1, s0, s1, s2, rc, rs);
    float ph = 0.f, fx = 0.f, fy = 0.f, fz = 0.f;
    for (int sg = 0; sg < ns; ++sg) {
        const int4 g = segs[sg];
        const int k0 = segoff[sg];
        float cs, sn;
        phase_cs(g.x, g.y, g.z, s0, s1, s2, cs, sn);
        for (int e = 0; e < g.w; ++e) {
            const float2 S = Sk[k0 + e];
            const float4 q = kv[k0 + e];
            const float re = S.x * cs - S.y * sn;
            const float im = S.x * sn + S.y * cs;
            ph = fmaf(q.w, re, ph);
            const float gi = q.w * im;
            fx = fmaf(q.x, gi, fx);
            fy = fmaf(q.y, gi, fy);
            fz = fmaf(q.z, gi, fz);
            const float c2 = fmaf(cs, rc, -sn * rs);
            sn = fmaf(sn, rc, cs * rs);
            cs = c2;
        }
    }
    if (i < N) {
        const float qi = qraw[i] + (float)scalars[S_DELTA];
        const float k4 = 4.0f * (float)KE;
        phi[i] += k4 * ph;
        Fst[i] += k4 * qi * fx;
        Fst[(size_t)N + i] += k4 * qi * fy;
        Fst[(size_t)2 * N + i] += k4 * qi * fz;
    }
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
    hipLaunchKernelGGL(k_kvector_rows, dim3(1), dim3(1024), 0, p.stream, p.cell, p.nk_box[0], p.nk_box[1],
                       p.nk_box[2], p.kmax * p.kmax, p.kinc, p.alpha, p.vol, p.nk_cap, p.seg_cap, p.kvec, kn,
                       p.ksegs, p.ksegoff, p.kcount, p.knseg);
    const int kb = (int)((p.nk_cap + 255) / 256);
    const int sbk = (int)((p.seg_cap + 255) / 256);
    hipLaunchKernelGGL(k_structure_factor_rows, dim3(sbk, p.s_chunks), dim3(256), 0, p.stream, p.N, p.xyzt,
                       p.cell, p.qraw, p.scalars, p.ksegs, p.ksegoff, p.knseg, p.nk_cap, p.Spart);
    hipLaunchKernelGGL(k_structure_reduce, dim3(kb), dim3(256), 0, p.stream, p.s_chunks, p.Spart, p.kvec,
                       p.kcount, p.nk_cap, p.alpha, p.Sk, p.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = reduce_partials(p, kb, 10, S_UK, false);  // S_UK, S_WK[9]
    if (e != hipSuccess) return e;
    stage_mark(p, ST_EWALD_SK, 4);
    const int G = (p.N + 255) / 256;
    hipLaunchKernelGGL(k_ewald_atoms_rows, dim3(G), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell, p.qraw,
                       p.scalars, p.kvec, p.ksegs, p.ksegoff, p.knseg, p.Sk, p.phi, p.Fst);
    if (p.out.virial_atom)
        hipLaunchKernelGGL(k_ewald_virial_atoms, dim3(G), dim3(256), 0, p.stream, p.N, p.xyzt, p.cell,
                           (float)p.alpha, p.qraw, p.scalars, p.kvec, (const int4 *)kn, p.Sk, p.kcount, p.Vat);
    stage_mark(p, ST_EWALD_ATOMS, p.out.virial_atom ? 2 : 1);
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
