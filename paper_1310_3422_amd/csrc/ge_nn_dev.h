// Device helpers shared by the surrogate network's kernels.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ge {
namespace nn {
namespace dev {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTaps = 5;

__device__ __forceinline__ float bf2f(bf16 v) { return (float)v; }
__device__ __forceinline__ bf16 f2bf(float v) { return (bf16)v; }   // round to nearest even

__device__ __forceinline__ float gelu(float z)
{
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float z)
{
    const float phi = 0.39894228040143268f * expf(-0.5f * z * z);
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * phi;
}

// 16-byte copy between global and LDS
__device__ __forceinline__ void copy16(void *dst, const void *src)
{
    *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(src);
}

}  // namespace dev
}  // namespace nn
}  // namespace ge
