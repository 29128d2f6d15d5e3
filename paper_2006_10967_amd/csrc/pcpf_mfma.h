// Line operators on the gfx950 matrix cores: bf16 operands, fp32 accumulation.
//
// The tensor-product element operators of the FR procedure act along one reference
// direction at a time: for the lines of one direction they are the product of a small
// (rows x n) coefficient matrix with an (n x lines) matrix of point values. Here 16 lines
// at a time go through v_mfma_f32_16x16x16_bf16 (M = 16 output rows, K = 16 >= n inputs,
// N = 16 lines), the coefficient and value matrices padded with zeros.
//
// Accuracy: each line's values enter as deviations from the line's mean, the mean's part
// m A 1 added in fp32 from the operator's fp32 row sums (constants and the mean level are
// then exact, and the bf16 rounding acts on the variation along the line only), and both
// operands are split into bf16 pairs, x = x_hi + x_lo with x_lo = bf16(x - x_hi):
//   A u = A_hi d_hi + A_hi d_lo + A_lo d_hi + m A 1   (d = u - m 1),
// three MFMAs per product, each operand then good to about 2^-17 instead of 2^-9.
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

__device__ __forceinline__ float bf16_float(short h) {
    return __builtin_bit_cast(float, (unsigned)(unsigned short)h << 16);
}

// hi / lo bf16 A operands of a row operator and the fp32 sums of this lane's output rows
// 4 (lane / 16) + j (rows i >= NA and inputs k >= N are zero).
struct RowsSplit {
    bf16x4 hi, lo;
    f32x4 rs;
};
template <int NA, int N, typename F>
__device__ __forceinline__ RowsSplit mfma_rows_split(F coef, int lane) {
    static_assert(NA <= 16 && N <= 16, "operator larger than one 16 x 16 tile");
    RowsSplit o;
    const int i = lane & 15, k0 = 4 * (lane >> 4);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = k0 + j;
        const float c = (i < NA && k < N) ? (float)coef(i, k) : 0.f;
        const short h = bf16_bits(c);
        o.hi[j] = h;
        o.lo[j] = bf16_bits(c - bf16_float(h));
        const int r = k0 + j;                  // an output row of this lane
        float sum = 0.f;
        if (r < NA) {
#pragma unroll
            for (int b = 0; b < N; ++b) sum += (float)coef(r, b);
        }
        o.rs[j] = sum;
    }
    return o;
}

// D = A U for 16 lines in the split form above. This lane supplies line c = lane % 16
// (value k at src[base + k * stride]; ok = false: a padding line of zeros) and on return
// holds rows 4 (lane / 16) + j of line c. Every lane of the wave must call it.
template <int N>
__device__ __forceinline__ f32x4 mfma_lines_split(const RowsSplit& a, const float* src, bool ok,
                                                  int base, int stride, int lane) {
    const int k0 = 4 * (lane >> 4);
    float u[N];
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        u[k] = ok ? src[base + k * stride] : 0.f;
        m += u[k];
    }
    m *= 1.f / (float)N;
    bf16x4 dh, dl;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = k0 + j;
        float d = 0.f;
#pragma unroll
        for (int b = 0; b < N; ++b)
            if (b == k) d = u[b] - m;
        const short h = bf16_bits(d);
        dh[j] = h;
        dl[j] = bf16_bits(d - bf16_float(h));
    }
    f32x4 acc = {m * a.rs[0], m * a.rs[1], m * a.rs[2], m * a.rs[3]};
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, dh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, dl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.lo, dh, acc, 0, 0, 0);
    return acc;
}

}  // namespace dev
}  // namespace pcpf
