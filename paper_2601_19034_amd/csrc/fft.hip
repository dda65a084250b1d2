// In-house 3D complex FFT for the PPPM mesh: one kernel launch per axis, each
// work-group loading a batch of lines into LDS, transforming them with Stockham
// radix-2/3/4/5/8 stages and writing them back in place.  Unnormalized in both
// directions: sign -1 gives sum_m x_m e^{-2 pi i n m / L}, sign +1 the inverse sum.
#include "plan.h"

namespace qnep {

constexpr int FFT_THREADS = 256;
constexpr int FFT_MAX_STAGES = 12;
constexpr int FFT_ELEMS = 4096;  // line elements held per work-group

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
    return n >= 1 && n <= FFT_ELEMS / 4 && make_plan(n, p);
}

__device__ inline float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// small DFT of length R (R in 2, 3, 4, 5, 8): out_m = sum_r a_r w^{r m}, w = e^{sign 2 pi i / R}
template <int R>
__device__ inline void dft_small(float2 (&a)[R], float sign) {
    float2 o[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
        float2 acc = a[0];
#pragma unroll
        for (int r = 1; r < R; ++r) {
            const int idx = (r * m) % R;
            float sn, cs;
            sincospif(2.0f * (float)idx / (float)R, &sn, &cs);
            float2 w = make_float2(cs, sign * sn);
            float2 t = cmul(a[r], w);
            acc.x += t.x;
            acc.y += t.y;
        }
        o[m] = acc;
    }
#pragma unroll
    for (int m = 0; m < R; ++m) a[m] = o[m];
}

template <int R>
__device__ inline void stage(const float2 *__restrict__ src, float2 *__restrict__ dst, int L, int nlines, int Ns,
                             float sign) {
    const int nb = L / R;
    for (int bf = threadIdx.x; bf < nlines * nb; bf += FFT_THREADS) {
        const int line = bf / nb, j = bf - line * nb;
        const int k = j % Ns;
        const float2 *s = src + line * L;
        float2 *d = dst + line * L;
        float2 a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = s[j + r * nb];
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float sn, cs;
                sincospif(2.0f * (float)(r * k) / (float)(Ns * R), &sn, &cs);
                a[r] = cmul(a[r], make_float2(cs, sign * sn));
            }
        }
        dft_small<R>(a, sign);
        const int base = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) d[base + r * Ns] = a[r];
    }
}

// Lines of length L along an axis with element stride S.  Line (o, in): element p at
// o * L * S + p * S + in.  S > 1: a block holds B consecutive `in` of one `o`;
// S == 1: B consecutive `o`.
__global__ __launch_bounds__(FFT_THREADS) void k_fft_axis(float2 *__restrict__ data, FftPlan1D plan, int S,
                                                           int nouter, int B, float sign) {
    extern __shared__ float2 lds[];
    const int L = plan.L;
    float2 *buf0 = lds, *buf1 = lds + L * B;
    int o0, in0, nl;
    if (S > 1) {
        const int groups = (S + B - 1) / B;
        o0 = blockIdx.x / groups;
        in0 = (blockIdx.x % groups) * B;
        nl = min(B, S - in0);
    } else {
        o0 = blockIdx.x * B;
        in0 = 0;
        nl = min(B, nouter - o0);
    }
    // load
    for (int idx = threadIdx.x; idx < L * B; idx += FFT_THREADS) {
        int p, cl;
        if (S > 1) {
            p = idx / B;
            cl = idx - p * B;
        } else {
            cl = idx / L;
            p = idx - cl * L;
        }
        if (cl < nl) {
            size_t g = S > 1 ? ((size_t)o0 * L * S + (size_t)p * S + in0 + cl) : ((size_t)(o0 + cl) * L + p);
            buf0[cl * L + p] = data[g];
        }
    }
    __syncthreads();
    float2 *src = buf0, *dst = buf1;
    int Ns = 1;
    for (int st = 0; st < plan.nst; ++st) {
        const int R = plan.radix[st];
        switch (R) {
            case 8: stage<8>(src, dst, L, nl, Ns, sign); break;
            case 4: stage<4>(src, dst, L, nl, Ns, sign); break;
            case 2: stage<2>(src, dst, L, nl, Ns, sign); break;
            case 5: stage<5>(src, dst, L, nl, Ns, sign); break;
            default: stage<3>(src, dst, L, nl, Ns, sign); break;
        }
        Ns *= R;
        __syncthreads();
        float2 *t = src;
        src = dst;
        dst = t;
    }
    // store
    for (int idx = threadIdx.x; idx < L * B; idx += FFT_THREADS) {
        int p, cl;
        if (S > 1) {
            p = idx / B;
            cl = idx - p * B;
        } else {
            cl = idx / L;
            p = idx - cl * L;
        }
        if (cl < nl) {
            size_t g = S > 1 ? ((size_t)o0 * L * S + (size_t)p * S + in0 + cl) : ((size_t)(o0 + cl) * L + p);
            data[g] = src[cl * L + p];
        }
    }
}

hipError_t fft3d(float2 *data, float2 * /*tmp*/, const int *mesh, int sign, hipStream_t s) {
    const int64_t M = (int64_t)mesh[0] * mesh[1] * mesh[2];
    for (int axis = 2; axis >= 0; --axis) {
        FftPlan1D plan;
        if (!make_plan(mesh[axis], plan)) return hipErrorInvalidValue;
        const int L = mesh[axis];
        const int S = axis == 2 ? 1 : (axis == 1 ? mesh[2] : mesh[1] * mesh[2]);
        const int nouter = (int)(M / ((int64_t)L * S));
        int B = FFT_ELEMS / L;
        if (B < 1) B = 1;
        int blocks;
        if (S > 1) {
            if (B > S) B = S;
            blocks = nouter * ((S + B - 1) / B);
        } else {
            blocks = (nouter + B - 1) / B;
        }
        const size_t lds = sizeof(float2) * 2 * (size_t)L * B;
        hipLaunchKernelGGL(k_fft_axis, dim3(blocks), dim3(FFT_THREADS), lds, s, data, plan, S, nouter, B,
                           (float)sign);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace qnep
