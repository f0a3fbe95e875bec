// Two-dimensional extension of the scheme: u_t = u_xx + u_yy on the unit
// square.  The paper states that the group explicit method extends to two
// dimensions without giving formulas; here every level m applies the
// one-dimensional level m of Section 2 (two-point groups, Eq. (3)/(4), a
// point alone beside a wall by Eq. (1)/(2)) along every row with
// r_x = tau/h_x^2, then along every column with r_y = tau/h_y^2 (first-order
// splitting; each line is paired by the level's global index exactly as a
// single rod is).
//
// A one-dimensional level is explicit: a point's new value depends on old
// values at most two places away along its line.  So one launch advances
// one level of a tile of 16 (FP64) or 32 (FP32) rows by 128 columns: the input tile with two
// points of halo on every side goes from HBM to LDS (coalesced rows), the
// x-level runs on the tile's rows plus two halo rows above and below and
// overwrites the tile in place (after a barrier), and the y-level reads it
// and writes straight back to HBM.  Per level the grid is read and written
// once: 16 bytes per point in FP64, HBM-bound.  Tiles are dealt to the XCDs
// in contiguous runs, so a tile's neighbours (which read the same halo
// lines) mostly run on the same L2 at about the same time.
//
// Walls are constant in time (west, east, south, north); the values beside
// a wall read the wall, which sits in the tile's halo cells.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ge_2d.h"
#include "ge_kernels.h"

namespace ge {
namespace {

constexpr int kTI = 128;            // columns per tile
constexpr int kThreads = 256;
constexpr int kAW = kTI + 4;        // tile row, with the halo

// Rows per tile: 16 in FP64 (21 KB of LDS, more tiles resident per CU: 12%
// faster than 32 rows on a 4096^2 grid, while the extra halo rows hit in
// L2), 32 in FP32 (3% faster than 16).
template <typename T> struct Tile {
    static constexpr int TJ = sizeof(T) == 8 ? 16 : 32;
    static constexpr int AH = TJ + 4;
    static constexpr int LPer = (AH * kAW + kThreads - 1) / kThreads;   // loads per thread
    static constexpr int XPer = AH * kTI / kThreads;                    // x-level values
    static constexpr int YPer = TJ * kTI / kThreads;                    // y-level values
    static_assert(AH * kTI % kThreads == 0 && TJ * kTI % kThreads == 0, "whole rows per block");
};

template <typename T> struct Line {
    T c1, c2, cs;   // (r+r^2)/(1+2r), r^2/(1+2r), r/(1+r)
};

// The one-dimensional level m at point e of a line of n points, from the
// old values u_{e-2} .. u_{e+2} (the wall where the line ends; values past
// a wall are never used).  Second-difference form: D_i = d_i - d_{i-1};
// a pair member takes u + c1 D_e + c2 D_q (q its partner), a point alone
// beside a wall u + cs D_e (constant walls).
template <typename T>
__device__ __forceinline__ T level1d(T um2, T um1, T u0, T up1, T up2, int e, int n, int p,
                                     const Line<T> &c)
{
    const bool left = ((e + p) & 1) == 0;        // pairs (e, e+1) when e + m is even
    const int q = left ? e + 1 : e - 1;
    const T d0 = up1 - u0, dm = u0 - um1;
    const T De = d0 - dm;
    if (q < 0 || q >= n) {
        if constexpr (sizeof(T) == 8) return fma(c.cs, De, u0);
        else return u0 + c.cs * De;
    }
    const T Dq = left ? (up2 - up1) - d0 : dm - (um1 - um2);
    if constexpr (sizeof(T) == 8) return fma(c.c2, Dq, fma(c.c1, De, u0));
    else return u0 + fmaf(c.c2, Dq, c.c1 * De);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void level2d_kernel(const T *__restrict__ in,
                                                           T *__restrict__ out, int nx, int ny,
                                                           int tiles_x, int ntiles, int p,
                                                           Line<T> cx, Line<T> cy, T gw, T ge_,
                                                           T gs, T gn)
{
    using G = Tile<T>;
    constexpr int kTJ = G::TJ, kAH = G::AH, kLPer = G::LPer, kXPer = G::XPer, kYPer = G::YPer;
    __shared__ T A[kAH][kAW];     // the tile with its halo; after the x-level, that level
    const int per = gridDim.x / 8;
    const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;   // XCD-aware
    if (t >= ntiles)
        return;
    const int i0 = (t % tiles_x) * kTI, j0 = (t / tiles_x) * kTJ;
    const int tid = threadIdx.x;
    // HBM -> LDS, every load issued before the first is used; cells past a
    // west/east wall hold the wall
    T v[kLPer];
#pragma unroll
    for (int q = 0; q < kLPer; ++q) {
        const int k = tid + q * kThreads;
        const int r = k / kAW, c = k % kAW;
        const int j = j0 - 2 + r, i = i0 - 2 + c;
        T x = T(0);
        if (k < kAH * kAW && j >= 0 && j < ny) {
            if (i >= 0 && i < nx) x = in[(int64_t)j * nx + i];
            else if (i == -1) x = gw;
            else if (i == nx) x = ge_;
        }
        v[q] = x;
    }
#pragma unroll
    for (int q = 0; q < kLPer; ++q) {
        const int k = tid + q * kThreads;
        if (k < kAH * kAW) A[k / kAW][k % kAW] = v[q];
    }
    __syncthreads();
    // x-level on rows j0-2 .. j0+kTJ+1, held in registers until every
    // thread has read its old values; rows past a south/north wall hold it
    T x[kXPer];
#pragma unroll
    for (int q = 0; q < kXPer; ++q) {
        const int k = tid + q * kThreads;
        const int r = k / kTI, c = k % kTI;
        const int j = j0 - 2 + r, i = i0 + c;
        T y = T(0);
        if (j == -1) y = gs;
        else if (j == ny) y = gn;
        else if (j >= 0 && j < ny && i < nx)
            y = level1d(A[r][c], A[r][c + 1], A[r][c + 2], A[r][c + 3], A[r][c + 4], i, nx, p, cx);
        x[q] = y;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kXPer; ++q) {
        const int k = tid + q * kThreads;
        A[k / kTI][k % kTI + 2] = x[q];
    }
    __syncthreads();
    // y-level on the tile's rows, straight to HBM
#pragma unroll
    for (int q = 0; q < kYPer; ++q) {
        const int k = tid + q * kThreads;
        const int r = k / kTI, c = k % kTI + 2;
        const int j = j0 + r, i = i0 + c - 2;
        if (j < ny && i < nx)
            out[(int64_t)j * nx + i] = level1d(A[r][c], A[r + 1][c], A[r + 2][c], A[r + 3][c],
                                               A[r + 4][c], j, ny, p, cy);
    }
}

template <typename T> Line<T> line_coef(double r)
{
    return Line<T>{(T)((r + r * r) / (1.0 + 2.0 * r)), (T)(r * r / (1.0 + 2.0 * r)),
                   (T)(r / (1.0 + r))};
}

template <typename T>
hipError_t launch_2d_t(const Grid2dArgs &a, hipStream_t stream)
{
    const int64_t tx = (a.nx + kTI - 1) / kTI, ty = (a.ny + Tile<T>::TJ - 1) / Tile<T>::TJ;
    const int64_t ntiles = tx * ty, grid = (ntiles + 7) / 8 * 8;
    const Line<T> cx = line_coef<T>(a.rx), cy = line_coef<T>(a.ry);
    const T *src = static_cast<const T *>(a.u);
    T *dst = static_cast<T *>(a.work);
    for (int64_t s = 0; s < a.nsteps; ++s) {
        hipLaunchKernelGGL((level2d_kernel<T>), dim3((unsigned)grid), dim3(kThreads), 0, stream,
                           src, dst, (int)a.nx, (int)a.ny, (int)tx, (int)ntiles,
                           (int)((a.step0 + s) & 1), cx, cy, (T)a.gw, (T)a.ge, (T)a.gs, (T)a.gn);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        T *t = const_cast<T *>(src);
        src = dst;
        dst = t;
    }
    // after an odd number of levels the result sits in the workspace
    if (a.nsteps % 2 == 1)
        return hipMemcpyAsync(a.u, a.work, (size_t)(a.nx * a.ny) * sizeof(T),
                              hipMemcpyDeviceToDevice, stream);
    return hipSuccess;
}

}  // namespace

hipError_t launch_2d(int prec, const Grid2dArgs &a, hipStream_t stream)
{
    const int64_t tiles = ((a.nx + kTI - 1) / kTI) * ((a.ny + 15) / 16);
    // indices inside a launch are 32-bit: rows and columns below 2^31
    if (a.nx < 1 || a.ny < 1 || a.nx > 0x7fffff00LL || a.ny > 0x7fffff00LL || tiles > 0x7ffffff0LL)
        return hipErrorInvalidValue;
    if (prec == kFP64) return launch_2d_t<double>(a, stream);
    if (prec == kFP32) return launch_2d_t<float>(a, stream);
    return hipErrorInvalidValue;
}

}  // namespace ge
