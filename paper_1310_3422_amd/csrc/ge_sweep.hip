// Tiled, temporally blocked GE sweep of one rod for gfx950 (the kernels are
// in ge_sweep_kernels.h): the persistent form, the tables of built row
// widths, the dispatch of a launch to the file that holds its row width, and
// the conversions of the compensated pair.
#include "ge_sweep_kernels.h"

namespace ge {
namespace {

__global__ void comp_to_fp64_kernel(const float *__restrict__ s, const float *__restrict__ e,
                                    double *__restrict__ x, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        x[i] = (double)s[i] + (double)e[i];
}

__global__ void comp_from_fp64_kernel(const double *__restrict__ x, float *__restrict__ s,
                                      float *__restrict__ e, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const float hi = (float)x[i];
        s[i] = hi;
        e[i] = (float)(x[i] - (double)hi);
    }
}

}  // namespace

int64_t comp_offset(int64_t n);

hipError_t launch_tiles_persistent(int prec, int k, bool src, const TileArgs &a,
                                   hipStream_t stream)
{
#define GE_P(T, KK, C) \
    return src ? launch_persistent<T, KK, C, true>(a, stream) : launch_persistent<T, KK, C, false>(a, stream)
    switch (prec) {
    case kFP64:
        if (k == 16) GE_P(double, 16, false);
        if (k == 32) GE_P(double, 32, false);
        if (k == 64) GE_P(double, 64, false);
        break;
    case kFP32:
        if (k == 16) GE_P(float, 16, false);
        if (k == 32) GE_P(float, 32, false);
        break;
    case kFP32C:
        if (k == 16) GE_P(float, 16, true);
        break;
    }
#undef GE_P
    return hipErrorInvalidValue;
}

bool persistent_supported(int prec, int k)
{
    return (prec == kFP64 && (k == 16 || k == 32 || k == 64)) ||
           (prec == kFP32 && (k == 16 || k == 32)) ||
           (prec == kFP32C && k == 16);
}

bool tile_config_supported(int prec, int k, int nw)
{
    if (nw != 1 && nw != 4)
        return false;
    switch (prec) {
    case kFP64:
        return k == 2 || k == 4 || k == 8 || k == 16 || k == 20 || k == 24 || k == 28 || k == 32 ||
               k == 64;
    case kFP32: return k == 4 || k == 8 || k == 16 || k == 32;
    case kFP32C: return k == 4 || k == 8 || k == 16;
    default: return false;
    }
}

hipError_t launch_tiles(int prec, int k, int nw, bool src, const TileArgs &a,
                        hipStream_t stream, const SideStream *side)
{
    switch (prec) {
    case kFP64:
        if (k <= 20) return launch_tiles_fp64_narrow(k, nw, src, a, stream, side);
        if (k <= 28) return launch_tiles_fp64_mid(k, nw, src, a, stream, side);
        return launch_tiles_fp64_wide(k, nw, src, a, stream, side);
    case kFP32: return launch_tiles_fp32(false, k, nw, src, a, stream, side);
    case kFP32C: return launch_tiles_fp32(true, k, nw, src, a, stream, side);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_comp_to_fp64(const float *pair, double *x, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int64_t off = comp_offset(n);
    hipLaunchKernelGGL(comp_to_fp64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       pair, pair + off, x, n);
    return hipGetLastError();
}

hipError_t launch_comp_from_fp64(const double *x, float *pair, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int64_t off = comp_offset(n);
    hipLaunchKernelGGL(comp_from_fp64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       s, x, pair, pair + off, n);
    return hipGetLastError();
}

}  // namespace ge
