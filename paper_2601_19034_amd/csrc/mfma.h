// BF16 matrix-core helpers (v_mfma_f32_16x16x16_bf16, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qnep {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ inline short to_bf16(float f) {  // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// Lane layout of the 16x16x16 BF16 MFMA (wave64, lane l):
//   A[i][k]: i = l % 16, k = 4 (l / 16) + e  (element e of the 4-vector)
//   B[k][j]: j = l % 16, k = 4 (l / 16) + e
//   D[i][j]: j = l % 16, i = 4 (l / 16) + e
// NSPLIT = 1: one BF16 product per term.  NSPLIT = 3: operands split x = hi + lo in
// BF16 and hi*hi + hi*lo + lo*hi accumulated (about 16 mantissa bits).
template <int NSPLIT>
__device__ inline floatx4 mfma_split(const float (&a)[4], const float (&b)[4], floatx4 acc) {
    bf16x4 ah, bh;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        ah[e] = to_bf16(a[e]);
        bh[e] = to_bf16(b[e]);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
    if (NSPLIT == 3) {
        bf16x4 al, bl;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            al[e] = to_bf16(a[e] - __uint_as_float((uint32_t)(unsigned short)ah[e] << 16));
            bl[e] = to_bf16(b[e] - __uint_as_float((uint32_t)(unsigned short)bh[e] << 16));
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
    }
    return acc;
}

// x = hi + lo with hi, lo in BF16 (lo = 0 when only hi is used)
__device__ inline void split_bf16(const float (&x)[4], bf16x4 &hi, bf16x4 &lo) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        hi[e] = to_bf16(x[e]);
        lo[e] = to_bf16(x[e] - __uint_as_float((uint32_t)(unsigned short)hi[e] << 16));
    }
}

// products of operands already split into BF16 parts: hi*hi (+ hi*lo + lo*hi)
template <int NSPLIT>
__device__ inline floatx4 mfma_parts(bf16x4 ah, bf16x4 al, bf16x4 bh, bf16x4 bl, floatx4 acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
    if (NSPLIT == 3) {
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
    }
    return acc;
}

// the same with the split chosen at run time (1 or 3 products)
__device__ inline floatx4 mfma_split_rt(const float (&a)[4], const float (&b)[4], floatx4 acc, int nsplit) {
    return nsplit == 3 ? mfma_split<3>(a, b, acc) : mfma_split<1>(a, b, acc);
}

}  // namespace qnep
