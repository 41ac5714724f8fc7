// Device functions shared by the pass kernels and the learned-index
// trainer, so that the error bound measured after training is computed with
// exactly the arithmetic the lookups use.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sinet {

// Index of the last arr[i] <= a among arr[0..n), given arr[0] <= a.  The trip
// count depends on n only, so lanes of a wave stay converged.
__device__ __forceinline__ uint32_t upper_last(const uint32_t* arr, uint32_t n, uint32_t a) {
    uint32_t lo = 0;
    while (n > 1) {
        uint32_t half = n >> 1;
        lo = (arr[lo + half] <= a) ? lo + half : lo;
        n -= half;
    }
    return lo;
}

__device__ __forceinline__ int clamp_pos(float pred, uint32_t m) {
    pred = fmaxf(pred, 0.0f);  // also maps NaN to 0
    pred = fminf(pred, (float)(m - 1));
    return (int)rintf(pred);
}

// PLA line of one segment: c + g * (a - knot) in float32, round to nearest,
// one rounding per operation (the error bound is measured with exactly this
// arithmetic).  The operators are written out under the pragma: the
// compiler fuses a product and a sum into one fma wherever contraction is
// left on, including inside __fmul_rn / __fadd_rn, which are plain operators
// in this toolchain.
__device__ __forceinline__ float pla_eval(uint32_t knot, float c, float g, uint32_t a) {
#pragma clang fp contract(off)
    const float d = __uint2float_rn(a - knot);
    const float gd = g * d;
    return c + gd;
}

// PLA prediction with the segment found by a full search over the knots.
__device__ __forceinline__ float pla_predict(const uint32_t* knot, const float* c, const float* g,
                                             uint32_t S, uint32_t a) {
    const uint32_t s = upper_last(knot, S, a);
    return pla_eval(knot[s], c[s], g[s], a);
}

// MLP prediction: m * (b2 + sum_k w2_k relu(w1_k x + b1_k)), x = a / 2^32,
// one rounding per operation (no fma, as in pla_eval), accumulated in k order.
__device__ __forceinline__ float mlp_predict(const float* w, float m_f, uint32_t a) {
#pragma clang fp contract(off)
    const float x = __uint2float_rn(a) * 2.3283064365386963e-10f;
    float f = w[48];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const float wx = w[k] * x;
        const float z = wx + w[16 + k];
        const float t = w[32 + k] * fmaxf(z, 0.0f);
        f = f + t;
    }
    return f * m_f;
}

}  // namespace sinet
