// Line operators on the gfx950 matrix cores: bf16 operands, fp32 accumulation.
//
// The tensor-product element operators of the FR procedure act along one reference
// direction at a time: for the lines of one direction they are the product of a small
// (rows x n) coefficient matrix with an (n x lines) matrix of point values. Here 16 lines
// at a time go through one v_mfma_f32_16x16x16_bf16 (M = 16 output rows, K = 16 >= n
// inputs, N = 16 lines), the coefficient and value matrices padded with zeros.
//
// Operand layout of the 16x16x16 instruction for lane l (0..63), j = 0..3:
//   A[i][k]: i = l % 16, k = 4 (l / 16) + j
//   B[k][c]: k = 4 (l / 16) + j, c = l % 16
//   D[i][c]: i = 4 (l / 16) + j, c = l % 16
// so lanes l, l + 16, l + 32, l + 48 all serve line c = l % 16.
#pragma once

#include <hip/hip_runtime.h>

namespace pcpf {
namespace dev {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round to nearest even bf16, as raw bits
__device__ __forceinline__ short bf16_bits(float x) {
    const __bf16 h = static_cast<__bf16>(x);
    return __builtin_bit_cast(short, h);
}

// A operand of a row operator: coef(i, k) for i < NA rows and k < N inputs, zero padded.
template <int NA, int N, typename F>
__device__ __forceinline__ bf16x4 mfma_rows(F coef, int lane) {
    static_assert(NA <= 16 && N <= 16, "operator larger than one 16 x 16 tile");
    const int i = lane & 15, k0 = 4 * (lane >> 4);
    bf16x4 a;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = k0 + j;
        a[j] = (i < NA && k < N) ? bf16_bits(coef(i, k)) : (short)0;
    }
    return a;
}

// D = A U for 16 lines. This lane supplies the values of line c = lane % 16: value k at
// src[base + k * stride] (ok = false: a padding line of zeros); on return it holds rows
// 4 (lane / 16) + j of line c. Every lane of the wave must call it (no divergence).
template <int N>
__device__ __forceinline__ f32x4 mfma_lines(bf16x4 a, const float* src, bool ok, int base,
                                            int stride, int lane) {
    const int k0 = 4 * (lane >> 4);
    bf16x4 b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = k0 + j;
        b[j] = (ok && k < N) ? bf16_bits(src[base + k * stride]) : (short)0;
    }
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, z, 0, 0, 0);
}

}  // namespace dev
}  // namespace pcpf
