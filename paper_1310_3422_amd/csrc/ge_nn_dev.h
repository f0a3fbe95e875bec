// Device helpers shared by the surrogate network's kernels.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ge {
namespace nn {
namespace dev {

typedef __bf16 bf16;
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTaps = 5;

__device__ __forceinline__ float bf2f(bf16 v) { return (float)v; }
__device__ __forceinline__ bf16 f2bf(float v) { return (bf16)v; }   // round to nearest even

// GELU in its tanh form, gelu(z) = (z/2) (1 + tanh(c (z + a z^3))),
// c = sqrt(2/pi), a = 0.044715, evaluated as z sigma(2w) = z / (1 + e^{-2w}),
// w = c (z + a z^3): one exp2, one reciprocal and four other operations.
// For z -> -inf the exponential overflows to +inf and the reciprocal gives
// 0, so no NaN appears.
constexpr float kGeluE0 = -2.0f * 0.7978845608028654f * 1.4426950408889634f;   // -2c log2(e)
constexpr float kGeluE2 = kGeluE0 * 0.044715f;
constexpr float kGeluD0 = 2.0f * 0.7978845608028654f;                          // 2c
constexpr float kGeluD2 = kGeluD0 * 3.0f * 0.044715f;

// sigma(2w) for the argument z
__device__ __forceinline__ float gelu_sigma(float z)
{
    const float e = __builtin_amdgcn_exp2f(z * fmaf(z * z, kGeluE2, kGeluE0));
    return __builtin_amdgcn_rcpf(1.0f + e);
}
__device__ __forceinline__ float gelu(float z) { return z * gelu_sigma(z); }
// d gelu / dz = s + z s (1 - s) 2w',  s = sigma(2w), 2w' = 2c (1 + 3 a z^2)
__device__ __forceinline__ float gelu_grad(float z)
{
    const float sg = gelu_sigma(z);
    return fmaf(z * sg, (1.0f - sg) * fmaf(z * z, kGeluD2, kGeluD0), sg);
}

// 16-byte copy between global and LDS
__device__ __forceinline__ void copy16(void *dst, const void *src)
{
    *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(src);
}

}  // namespace dev
}  // namespace nn
}  // namespace ge
