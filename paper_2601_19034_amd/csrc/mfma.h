// BF16 matrix-core helpers (v_mfma_f32_16x16x16_bf16, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qnep.h"

namespace qnep {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ inline short to_bf16(float f) {  // round to nearest even (v_cvt_pk_bf16_f32)
    const __bf16 b = (__bf16)f;
    return __builtin_bit_cast(short, b);
}

// tanh x = sign(x) (1 - e) / (1 + e) with e = exp(-2 |x|) = 2^(-2 log2(e) |x|): absolute
// error about 1e-7, far below the rounding of the BF16 network forms that use it
__device__ inline float tanh_fast(float x) {
    const float e = __builtin_amdgcn_exp2f(-2.8853900817779268f * fabsf(x));
    return copysignf((1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e), x);
}

// Lane layout of the 16x16x16 BF16 MFMA (wave64, lane l):
//   A[i][k]: i = l % 16, k = 4 (l / 16) + e  (element e of the 4-vector)
//   B[k][j]: j = l % 16, k = 4 (l / 16) + e
//   D[i][j]: j = l % 16, i = 4 (l / 16) + e
// Operands are split x = hi + lo with hi, lo in BF16 (hi carries 8 mantissa bits,
// hi + lo about 16).  A product of split operands keeps the terms selected by MASK:
// hi*hi always, bit 0 adds A_lo*B_hi, bit 1 adds A_hi*B_lo (lo*lo is below FP32
// accumulation noise and is never formed).
constexpr int SPLIT_A_LO = 1, SPLIT_B_LO = 2, SPLIT_BOTH = 3;

__device__ inline void split_bf16(const float (&x)[4], bf16x4 &hi, bf16x4 &lo) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        hi[e] = to_bf16(x[e]);
        lo[e] = to_bf16(x[e] - __uint_as_float((uint32_t)(unsigned short)hi[e] << 16));
    }
}

template <int MASK>
__device__ inline floatx4 mfma_parts(bf16x4 ah, bf16x4 al, bf16x4 bh, bf16x4 bl, floatx4 acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
    if (MASK & SPLIT_B_LO) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
    if (MASK & SPLIT_A_LO) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
    return acc;
}

// FP32 operands split on the fly; the mask is chosen at run time
__device__ inline floatx4 mfma_split_rt(const float (&a)[4], const float (&b)[4], floatx4 acc, int mask) {
    bf16x4 ah, al, bh, bl;
    split_bf16(a, ah, al);
    split_bf16(b, bh, bl);
    if (mask == SPLIT_BOTH) return mfma_parts<SPLIT_BOTH>(ah, al, bh, bl, acc);
    if (mask == SPLIT_B_LO) return mfma_parts<SPLIT_B_LO>(ah, al, bh, bl, acc);
    if (mask == SPLIT_A_LO) return mfma_parts<SPLIT_A_LO>(ah, al, bh, bl, acc);
    return mfma_parts<0>(ah, al, bh, bl, acc);
}

// Products of the network in each BF16 form (A = weights, B = activations):
//   QNEP_MLP_BF16    forward D W0^T with both operands split, backward G W0 with the
//                    weights split and the activation gradient rounded once to BF16;
//   QNEP_MLP_BF16X3  both products with both operands split.
// Rounding the weights of the backward product instead would make the gradient that of
// a slightly different network, an error that adds up coherently in the virial.
__host__ __device__ constexpr int forward_mask(int) { return SPLIT_BOTH; }
__host__ __device__ constexpr int backward_mask(int prec) { return prec == QNEP_MLP_BF16X3 ? SPLIT_BOTH : SPLIT_A_LO; }

}  // namespace qnep
