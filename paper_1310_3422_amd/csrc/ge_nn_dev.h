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

// Standard normal distribution at z: Phi(z) from the upper tail
// Q(x) = 1 - Phi(x), x = |z|, by Abramowitz and Stegun 26.2.17,
//     Q(x) = phi(x) (b1 t + b2 t^2 + b3 t^3 + b4 t^4 + b5 t^5),  t = 1 / (1 + p x),
// absolute error below 7.5e-8; branch free, and the negative tail comes out
// without the cancellation of 1 + erf.  phi is the density.
struct Normal {
    float cdf, pdf;
};
__device__ __forceinline__ Normal normal_at(float z)
{
    const float x = fabsf(z);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.2316419f, x, 1.0f));
    float poly = fmaf(t, 1.330274429f, -1.821255978f);
    poly = fmaf(t, poly, 1.781477937f);
    poly = fmaf(t, poly, -0.356563782f);
    poly = fmaf(t, poly, 0.319381530f);
    poly *= t;
    const float pdf = 0.398942280401432678f * __expf(-0.5f * x * x);
    const float q = pdf * poly;
    return Normal{z >= 0.f ? 1.0f - q : q, pdf};
}

// GELU(z) = z Phi(z) and its derivative Phi(z) + z phi(z)
__device__ __forceinline__ float gelu(float z) { return z * normal_at(z).cdf; }
__device__ __forceinline__ float gelu_grad(float z)
{
    const Normal nz = normal_at(z);
    return nz.cdf + z * nz.pdf;
}

// 16-byte copy between global and LDS
__device__ __forceinline__ void copy16(void *dst, const void *src)
{
    *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(src);
}

}  // namespace dev
}  // namespace nn
}  // namespace ge
