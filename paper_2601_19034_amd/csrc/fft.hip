// In-house 3D complex FFT for the PPPM mesh: one kernel launch per axis, each
// work-group loading a batch of lines into LDS, transforming them with Stockham
// radix-2/3/4/5/8 stages and writing them back in place.  Unnormalized in both
// directions: sign -1 gives sum_m x_m e^{-2 pi i n m / L}, sign +1 the inverse sum.
//
// The twiddles e^{sign 2 pi i m / L} of the line length are tabulated once per
// work-group in LDS; the roots of the small DFTs are compile-time constants.  Lines
// are stored in LDS with a stride of L + 1 elements so that the transposing loads and
// stores of the strided axes (consecutive lanes = consecutive lines) hit distinct banks.
#include "fft256.h"
#include "plan.h"

namespace qnep {

constexpr int FFT_THREADS = 256;
constexpr int FFT_MAX_STAGES = 12;
constexpr int FFT_ELEMS = 2048;  // line elements held per work-group (8 lines of 256: 34 KB of LDS)

struct FftPlan1D {
    int L;
    int nst;
    int radix[FFT_MAX_STAGES];
};

static bool make_plan(int L, FftPlan1D &p) {
    p.L = L;
    p.nst = 0;
    int r = L;
    const int order[5] = {8, 4, 2, 5, 3};
    while (r > 1) {
        bool ok = false;
        for (int f : order) {
            if (r % f == 0) {
                if (p.nst >= FFT_MAX_STAGES) return false;
                p.radix[p.nst++] = f;
                r /= f;
                ok = true;
                break;
            }
        }
        if (!ok) return false;
    }
    return true;
}

bool fft_length_supported(int n) {
    FftPlan1D p;
    return n >= 1 && n <= 1024 && make_plan(n, p);
}


// cos and sin of 2 pi k / R for the small radices
template <int R>
struct Roots;
template <>
struct Roots<2> {
    static constexpr float c[2] = {1.0f, -1.0f}, s[2] = {0.0f, 0.0f};
};
template <>
struct Roots<3> {
    static constexpr float c[3] = {1.0f, -0.5f, -0.5f};
    static constexpr float s[3] = {0.0f, 0.86602540378443865f, -0.86602540378443865f};
};
template <>
struct Roots<4> {
    static constexpr float c[4] = {1.0f, 0.0f, -1.0f, 0.0f}, s[4] = {0.0f, 1.0f, 0.0f, -1.0f};
};
template <>
struct Roots<5> {
    static constexpr float c[5] = {1.0f, 0.30901699437494742f, -0.80901699437494742f, -0.80901699437494742f,
                                   0.30901699437494742f};
    static constexpr float s[5] = {0.0f, 0.95105651629515357f, 0.58778525229247313f, -0.58778525229247313f,
                                   -0.95105651629515357f};
};
template <>
struct Roots<8> {
    static constexpr float c[8] = {1.0f, 0.70710678118654752f, 0.0f, -0.70710678118654752f,
                                   -1.0f, -0.70710678118654752f, 0.0f, 0.70710678118654752f};
    static constexpr float s[8] = {0.0f, 0.70710678118654752f, 1.0f, 0.70710678118654752f,
                                   0.0f, -0.70710678118654752f, -1.0f, -0.70710678118654752f};
};

// small DFT of length R: out_m = sum_r a_r w^{r m}, w = e^{SG 2 pi i / R}, SG = +-1.
// Radices 3 and 5 by the definition with constant roots; 2, 4 and 8 as butterflies
// (8 = two radix-4 transforms of the even and odd inputs joined by w^m).
template <int R, int SG>
struct SmallDft {
    __device__ static void run(float2 (&a)[R]) {
        float2 o[R];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            float2 acc = a[0];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const int idx = (r * m) % R;
                const float2 t = cmul(a[r], make_float2(Roots<R>::c[idx], (float)SG * Roots<R>::s[idx]));
                acc.x += t.x;
                acc.y += t.y;
            }
            o[m] = acc;
        }
#pragma unroll
        for (int m = 0; m < R; ++m) a[m] = o[m];
    }
};
template <int SG>
struct SmallDft<2, SG> {
    __device__ static void run(float2 (&a)[2]) {
        const float2 t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    }
};
template <int SG>
struct SmallDft<4, SG> {
    __device__ static void run(float2 (&a)[4]) {
        float2 o[4];
        dft4<SG>(a[0], a[1], a[2], a[3], o);
#pragma unroll
        for (int m = 0; m < 4; ++m) a[m] = o[m];
    }
};
template <int SG>
struct SmallDft<8, SG> {
    __device__ static void run(float2 (&a)[8]) {
        constexpr float h = 0.70710678118654752f;
        float2 e[4], d[4];
        dft4<SG>(a[0], a[2], a[4], a[6], e);
        dft4<SG>(a[1], a[3], a[5], a[7], d);
        // w^1 d1 = h (x - SG y, SG x + y), w^2 d2 = (SG i) d2, w^3 d3 = h (-x - SG y, SG x - y)
        const float2 w1 = make_float2(h * (d[1].x - (float)SG * d[1].y), h * ((float)SG * d[1].x + d[1].y));
        const float2 w2 = mul_i<SG>(d[2]);
        const float2 w3 = make_float2(h * (-d[3].x - (float)SG * d[3].y), h * ((float)SG * d[3].x - d[3].y));
        a[0] = cadd(e[0], d[0]);
        a[4] = csub(e[0], d[0]);
        a[1] = cadd(e[1], w1);
        a[5] = csub(e[1], w1);
        a[2] = cadd(e[2], w2);
        a[6] = csub(e[2], w2);
        a[3] = cadd(e[3], w3);
        a[7] = csub(e[3], w3);
    }
};

// one Stockham stage over `nlines` lines of stride Lp; tw[m] = e^{SG 2 pi i m / L}
// nbs, nss: log2 of L / R and of Ns when L is a power of two (shifts replace the
// integer divisions), else -1
template <int R, int SG>
__device__ inline void stage(const float2 *__restrict__ src, float2 *__restrict__ dst, const float2 *__restrict__ tw,
                             int L, int Lp, int nlines, int Ns, int nbs, int nss) {
    const int nb = L / R;
    const int tstep = L / (Ns * R);  // twiddle index step: e^{2 pi i r k / (Ns R)} = tw[r k tstep]
    for (int bf = threadIdx.x; bf < nlines * nb; bf += FFT_THREADS) {
        const int line = nbs >= 0 ? bf >> nbs : bf / nb, j = bf - line * nb;
        const int k = nss >= 0 ? (j & (Ns - 1)) : j % Ns;
        const float2 *s = src + line * Lp;
        float2 *d = dst + line * Lp;
        float2 a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = s[j + r * nb];
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) a[r] = cmul(a[r], tw[r * k * tstep]);
        }
        SmallDft<R, SG>::run(a);
        const int base = (j - k) * R + k;  // (j / Ns) Ns R + k
#pragma unroll
        for (int r = 0; r < R; ++r) d[base + r * Ns] = a[r];
    }
}

// Lines of length L along an axis with element stride S.  Line (o, in): element p at
// o * L * S + p * S + in.  S > 1: a block holds B consecutive `in` of one `o`;
// S == 1: B consecutive `o`.
// ls, bs: log2 L and log2 B when they are powers of two, else -1
template <int SG>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_axis(float2 *__restrict__ data, FftPlan1D plan, int S,
                                                           int nouter, int B, int ls, int bs) {
    extern __shared__ float2 lds[];
    const int L = plan.L, Lp = L + 1;
    float2 *tw = lds;
    float2 *buf0 = lds + L, *buf1 = buf0 + Lp * B;
    for (int m = threadIdx.x; m < L; m += FFT_THREADS) {
        float sn, cs;
        sincospif(2.0f * (float)m / (float)L, &sn, &cs);
        tw[m] = make_float2(cs, (float)SG * sn);
    }
    // XCD-aware order: neighbouring batches (which share 128-byte lines on the strided
    // axes) run on the same XCD and meet in its L2
    const int blk = xcd_block();
    int o0, in0, nl;
    if (S > 1) {
        const int groups = (S + B - 1) / B;
        o0 = blk / groups;
        in0 = (blk % groups) * B;
        nl = min(B, S - in0);
    } else {
        o0 = blk * B;
        in0 = 0;
        nl = min(B, nouter - o0);
    }
    // load (consecutive lanes read consecutive addresses in both cases)
    for (int idx = threadIdx.x; idx < L * B; idx += FFT_THREADS) {
        int p, cl;
        if (S > 1) {
            p = bs >= 0 ? idx >> bs : idx / B;
            cl = idx - p * B;
        } else {
            cl = ls >= 0 ? idx >> ls : idx / L;
            p = idx - cl * L;
        }
        if (cl < nl) {
            const size_t g = S > 1 ? ((size_t)o0 * L * S + (size_t)p * S + in0 + cl) : ((size_t)(o0 + cl) * L + p);
            buf0[cl * Lp + p] = data[g];
        }
    }
    __syncthreads();
    float2 *src = buf0, *dst = buf1;
    int Ns = 1, nsl = 0;
    for (int st = 0; st < plan.nst; ++st) {
        const int R = plan.radix[st];
        const int rl = R == 8 ? 3 : (R == 4 ? 2 : 1);  // log2 R (used only when L is a power of two)
        const int nbs = ls >= 0 ? ls - rl : -1, nss = ls >= 0 ? nsl : -1;
        switch (R) {
            case 8: stage<8, SG>(src, dst, tw, L, Lp, nl, Ns, nbs, nss); break;
            case 4: stage<4, SG>(src, dst, tw, L, Lp, nl, Ns, nbs, nss); break;
            case 2: stage<2, SG>(src, dst, tw, L, Lp, nl, Ns, nbs, nss); break;
            case 5: stage<5, SG>(src, dst, tw, L, Lp, nl, Ns, -1, -1); break;
            default: stage<3, SG>(src, dst, tw, L, Lp, nl, Ns, -1, -1); break;
        }
        Ns *= R;
        nsl += rl;
        __syncthreads();
        float2 *t = src;
        src = dst;
        dst = t;
    }
    // store
    for (int idx = threadIdx.x; idx < L * B; idx += FFT_THREADS) {
        int p, cl;
        if (S > 1) {
            p = bs >= 0 ? idx >> bs : idx / B;
            cl = idx - p * B;
        } else {
            cl = ls >= 0 ? idx >> ls : idx / L;
            p = idx - cl * L;
        }
        if (cl < nl) {
            const size_t g = S > 1 ? ((size_t)o0 * L * S + (size_t)p * S + in0 + cl) : ((size_t)(o0 + cl) * L + p);
            data[g] = src[cl * Lp + p];
        }
    }
}

// ---------------------------------------------------------------- length 256
// Four-step transform of lines of 256 = 16 x 16 held in registers: thread t of a line
// holds x[t + 16 m], m < 16, and transforms over m (16-point DFT, radix 4 x 4); the
// results are multiplied by w_256^{t k1}, exchanged through LDS (thread k1 gathers
// the values of all t) and transformed again, giving X[k1 + 16 k2] in thread k1 at
// register k2 -- the load pattern, so loads and stores match.  One LDS exchange
// replaces the three staged passes of the general kernel.  A work-group holds 16
// lines; consecutive lanes read consecutive addresses in every layout:
//   mode 0 (S == 1): lane = 16 line + t;  mode 1 (S a multiple of 16): lane = 16 t + line
//   (16 consecutive `in`);  mode 2 (S = 2, 4, 8): lane = S (t + 16 o) + in (16 / S
//   consecutive `o` with all their `in`).
template <int SG>
__global__ __launch_bounds__(256) void k_fft256(float2 *__restrict__ data, int S, int nouter, int mode) {
    __shared__ float2 tw[256];
    __shared__ float2 xch[16 * F256_LS];
    for (int m = threadIdx.x; m < 256; m += blockDim.x) {
        float sn, cs;
        sincospif((float)m / 128.0f, &sn, &cs);
        tw[m] = make_float2(cs, (float)SG * sn);
    }
    const int lane = threadIdx.x, blk = xcd_block();
    int cl, t;        // line in the work-group and position in the line
    size_t base;      // address of element 0 of the line
    int stride;       // element stride along the line
    bool ok;
    if (mode == 0) {
        cl = lane >> 4;
        t = lane & 15;
        const int o = blk * 16 + cl;
        ok = o < nouter;
        base = (size_t)o * 256;
        stride = 1;
    } else if (mode == 1) {
        cl = lane & 15;
        t = lane >> 4;
        const int groups = S / 16;
        const int o = blk / groups, in = (blk - o * groups) * 16 + cl;
        ok = true;
        base = (size_t)o * 256 * S + in;
        stride = S;
    } else {
        const int in = lane % S, r = lane / S;
        t = r & 15;
        const int ol = r >> 4, o = blk * (16 / S) + ol;
        cl = ol * S + in;
        ok = o < nouter;
        base = (size_t)o * 256 * S + in;
        stride = S;
    }
    float2 a[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) a[m] = ok ? data[base + (size_t)(t + 16 * m) * stride] : make_float2(0.f, 0.f);
    line256<SG>(a, t, tw, xch + cl * F256_LS);
    if (ok) {
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) data[base + (size_t)(t + 16 * k2) * stride] = a[k2];
    }
}

// One axis: nouter groups of S interleaved lines of length L, element t of line s of
// group o at (o L + t) S + s, transformed in place.
static hipError_t fft_lines(float2 *data, int L, int S, int nouter, int sign, hipStream_t s) {
    static size_t lds_allowed = 65536;  // the default limit of dynamic LDS per work-group
    FftPlan1D plan;
    if (!make_plan(L, plan)) return hipErrorInvalidValue;
    if (L == 256 && (S == 1 || S % 16 == 0 || S == 2 || S == 4 || S == 8)) {
        const int mode = S == 1 ? 0 : (S % 16 == 0 ? 1 : 2);
        const int blocks = mode == 0 ? (nouter + 15) / 16
                                     : (mode == 1 ? nouter * (S / 16) : (nouter + 16 / S - 1) / (16 / S));
        if (sign < 0)
            hipLaunchKernelGGL(k_fft256<-1>, dim3(blocks), dim3(256), 0, s, data, S, nouter, mode);
        else
            hipLaunchKernelGGL(k_fft256<1>, dim3(blocks), dim3(256), 0, s, data, S, nouter, mode);
        return hipGetLastError();
    }
    int B = FFT_ELEMS / L;
    if (B < 1) B = 1;
    int blocks;
    if (S > 1) {
        if (B > S) B = S;
        blocks = nouter * ((S + B - 1) / B);
    } else {
        blocks = (nouter + B - 1) / B;
    }
    // twiddle table plus two buffers of B lines of L + 1 elements (at most 139 KB)
    const size_t lds = sizeof(float2) * ((size_t)L + 2 * (size_t)(L + 1) * B);
    if (lds > lds_allowed) {
        hipError_t e =
            hipFuncSetAttribute((const void *)k_fft_axis<-1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_fft_axis<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds);
        if (e != hipSuccess) return e;
        lds_allowed = lds;
    }
    const int ls = (L & (L - 1)) == 0 ? __builtin_ctz(L) : -1;
    const int bs = (B & (B - 1)) == 0 ? __builtin_ctz(B) : -1;
    if (sign < 0)
        hipLaunchKernelGGL(k_fft_axis<-1>, dim3(blocks), dim3(FFT_THREADS), lds, s, data, plan, S, nouter, B, ls, bs);
    else
        hipLaunchKernelGGL(k_fft_axis<1>, dim3(blocks), dim3(FFT_THREADS), lds, s, data, plan, S, nouter, B, ls, bs);
    return hipGetLastError();
}

// `inner` interleaved transforms: element (m0, m1, m2, t) of transform t at
// ((m0 n1 + m1) n2 + m2) inner + t; they go through the same launches
hipError_t fft3d(float2 *data, float2 * /*tmp*/, const int *mesh, int sign, hipStream_t s, int inner) {
    const int64_t M = (int64_t)mesh[0] * mesh[1] * mesh[2] * inner;
    for (int axis = 2; axis >= 0; --axis) {
        const int L = mesh[axis];
        const int S = inner * (axis == 2 ? 1 : (axis == 1 ? mesh[2] : mesh[1] * mesh[2]));
        const int nouter = (int)(M / ((int64_t)L * S));
        hipError_t e = fft_lines(data, L, S, nouter, sign, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The inverse passes along b and c (in that order) of `inner` interleaved transforms;
// the pass along a is done by the caller.
hipError_t fft3d_bc(float2 *data, const int *mesh, int sign, hipStream_t s, int inner) {
    hipError_t e = fft_lines(data, mesh[1], inner * mesh[2], mesh[0], sign, s);
    if (e != hipSuccess) return e;
    return fft_lines(data, mesh[2], inner, mesh[0] * mesh[1], sign, s);
}

// ---------------------------------------------------------------- real input
// Forward transform of a real mesh x[j0][j1][j2] (n1 even, n2 = 256).  Lines j1 = 2p and
// 2p + 1 are given as one complex line z_m = x[j0][2p][m] + i x[j0][2p+1][m] (the pair
// interleaved, complex element (j0 n1 / 2 + p) n2 + m) and transformed together along
// c; the two real lines' spectra are X_k = (Z_k + conj Z_{-k}) / 2 and
// Y_k = (Z_k - conj Z_{-k}) / 2i, of which k = 0 .. H = n2 / 2 are kept, X_0 and X_H
// (real) packed as X_0 + i X_H into slot 0.  The transforms along b and a then run
// over the H slots of every line, so `data` ends as the half spectrum T[j0][j1][k2],
// k2 < H, of S(k) = sum_j x_j e^{-2 pi i k.j / n}:
//   S(k0, k1, k2) = T[k0][k1][k2] for 0 < k2 < H, and with P = T[k0][k1][0],
//   P' = T[-k0][-k1][0]: S(k0, k1, 0) = (P + conj P') / 2, S(k0, k1, H) = (P - conj P') / 2i.
// The pair's n2 complex elements are exactly the two half lines, so this is in place.
//
// The pass along c (n2 = 256) and the pair split: k_fft256<-1> in mode 0 (16 lines per
// work-group, lane = 16 line + t), then each line's spectrum goes through LDS and is
// split into the two real lines' half spectra, X_k and Y_k for k < 128 (X_0 + i X_128
// and Y_0 + i Y_128 in slot 0)
__global__ __launch_bounds__(256) void k_fft256_pairs(float2 *__restrict__ data, int nlines) {
    __shared__ float2 tw[256];
    __shared__ float2 xch[16 * F256_LS];
    {
        float sn, cs;
        sincospif((float)threadIdx.x / 128.0f, &sn, &cs);
        tw[threadIdx.x] = make_float2(cs, -sn);  // e^{-2 pi i m / 256}
    }
    const int cl = threadIdx.x >> 4, t = threadIdx.x & 15;
    const int o = xcd_block() * 16 + cl;
    const bool ok = o < nlines;
    float2 *line = data + (size_t)(ok ? o : 0) * 256;
    float2 a[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) a[m] = ok ? line[t + 16 * m] : make_float2(0.f, 0.f);
    float2 *row = xch + cl * F256_LS;
    line256<-1>(a, t, tw, row);
    __syncthreads();  // every thread is done with the exchange area
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) row[t + 16 * k2] = a[k2];
    __syncthreads();
    if (!ok) return;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = t + 16 * j;
        float2 X, Y;
        if (k == 0) {
            const float2 z0 = row[0], zh = row[128];
            X = make_float2(z0.x, zh.x);
            Y = make_float2(z0.y, zh.y);
        } else {
            const float2 p = row[k], q = row[256 - k];
            X = make_float2(0.5f * (p.x + q.x), 0.5f * (p.y - q.y));
            Y = make_float2(0.5f * (p.y + q.y), -0.5f * (p.x - q.x));
        }
        line[k] = X;
        line[128 + k] = Y;
    }
}

// Meshes of 256 points along c (even along b) only: there the pass along c and the split
// are one kernel; with the general kernel the extra launch cost more than the halved
// bytes saved on 64- and 128-point meshes.
bool fft_r2c_supported(const int *mesh) { return mesh[1] % 2 == 0 && mesh[2] == 256; }

hipError_t fft3d_r2c(float2 *data, const int *mesh, hipStream_t s) {
    const int H = mesh[2] / 2, pairs = mesh[0] * (mesh[1] / 2);  // mesh[2] = 256
    hipLaunchKernelGGL(k_fft256_pairs, dim3((pairs + 15) / 16), dim3(256), 0, s, data, pairs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = fft_lines(data, mesh[1], H, mesh[0], -1, s);
    if (e != hipSuccess) return e;
    return fft_lines(data, mesh[0], mesh[1] * H, 1, -1, s);
}

}  // namespace qnep
