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
// values at most two places away along its line.  So a launch advances D
// levels (D = 1, 2 or 4) of a strip of columns held in registers, one column
// per lane (see level2d_reg_kernel): the x-level's neighbours come from the
// lanes beside it by DPP shifts, the y-level's from the lane's own rows, and
// the valid lanes and rows shrink by two per side and level (a halo of 2D
// lanes and rows, recomputed).  Per launch the grid is read and written
// once: 16/D bytes per point and level in FP64.  Every point is advanced by
// the same operations whatever D is, so the depth changes no bits.
//
// Walls are constant in time (west, east, south, north); the values beside
// a wall read the wall, which a halo lane or row holds.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ge_2d.h"
#include "ge_kernels.h"
#include "ge_level.h"

namespace ge {
namespace {

constexpr int kThreads = 256;       // four waves, four column strips

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

// Register form.  Lane l of a wave holds column c0 - 2D + l for rows
// r0 - 2D .. r0 + R + 2D - 1 (walls where they fall, zero past them); each
// level takes the x-level's neighbours from the lanes beside it (DPP shifts
// by one and two lanes; the edge lanes are halo) and the y-level's from the
// lane's own registers.  The valid lanes and rows shrink by two per side
// and level; after D levels lanes 2D..63-2D write their column's R rows.
// No LDS and no barrier: every load of a lane is issued at once.
using dev::kWave;

template <typename T>
__device__ __forceinline__ T shr1(T v) { return dev::from_left_open(v); }    // lane l-1
template <typename T>
__device__ __forceinline__ T shl1(T v) { return dev::from_right_open(v); }   // lane l+1

template <int D> struct RegTile {
    static constexpr int R = D == 1 ? 32 : D == 2 ? 24 : 16;   // output rows per wave
    static constexpr int H = 2 * D;                            // halo lanes / rows per side
    static constexpr int N = R + 2 * H;                        // rows held
    static constexpr int COLS = kWave - 2 * H;                 // output columns per wave
};

template <typename T, int D>
__global__ __launch_bounds__(kThreads) void level2d_reg_kernel(const T *__restrict__ in,
                                                               T *__restrict__ out, int nx, int ny,
                                                               int strips, int ntiles, int p0,
                                                               Line<T> cx, Line<T> cy, T gw,
                                                               T ge_, T gs, T gn)
{
    using G = RegTile<D>;
    constexpr int R = G::R, H = G::H, N = G::N;
    const int per = gridDim.x / 8;
    const int b = (blockIdx.x % 8) * per + blockIdx.x / 8;   // XCD-aware
    const int t = b * (kThreads / kWave) + threadIdx.x / kWave;   // this wave's tile
    if (t >= ntiles)
        return;
    const int lane = threadIdx.x % kWave;
    const int i = (t % strips) * G::COLS - H + lane;
    const int jb = (t / strips) * R - H;
    const bool col_in = i >= 0 && i < nx;
    T u[N];
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const int j = jb + q;
        T x = T(0);
        if (j == -1) x = gs;
        else if (j == ny) x = gn;
        else if (j >= 0 && j < ny) {
            if (col_in) x = in[(int64_t)j * nx + i];
            else if (i == -1) x = gw;
            else if (i == nx) x = ge_;
        }
        u[q] = x;
    }
#pragma unroll
    for (int l = 0; l < D; ++l) {
        const int p = (p0 + l) & 1;
        // x-level on rows [2l, N - 2l)
#pragma unroll
        for (int q = 2 * l; q < N - 2 * l; ++q) {
            const T um1 = shr1(u[q]), up1 = shl1(u[q]);
            const T um2 = shr1(um1), up2 = shl1(up1);
            const int j = jb + q;
            if (col_in && j >= 0 && j < ny) u[q] = level1d(um2, um1, u[q], up1, up2, i, nx, p, cx);
        }
        if (l == D - 1)
            break;
        // y-level on rows [2l+2, N-2l-2), from the old values of the column
        T v[N];
#pragma unroll
        for (int q = 2 * l + 2; q < N - 2 * l - 2; ++q) {
            const int j = jb + q;
            v[q] = (col_in && j >= 0 && j < ny)
                       ? level1d(u[q - 2], u[q - 1], u[q], u[q + 1], u[q + 2], j, ny, p, cy)
                       : u[q];
        }
#pragma unroll
        for (int q = 2 * l + 2; q < N - 2 * l - 2; ++q) u[q] = v[q];
    }
    // the last y-level: lanes H .. 63-H, rows H .. H+R-1, straight to HBM
    if (lane < H || lane >= kWave - H || !col_in)
        return;
    const int p = (p0 + D - 1) & 1;
#pragma unroll
    for (int q = H; q < H + R; ++q) {
        const int j = jb + q;
        if (j < ny)
            out[(int64_t)j * nx + i] = level1d(u[q - 2], u[q - 1], u[q], u[q + 1], u[q + 2], j, ny, p,
                                               cy);
    }
}

template <typename T> Line<T> line_coef(double r)
{
    return Line<T>{(T)((r + r * r) / (1.0 + 2.0 * r)), (T)(r * r / (1.0 + 2.0 * r)),
                   (T)(r / (1.0 + r))};
}

template <typename T, int D>
hipError_t launch_reg_levels(const T *src, T *dst, const Grid2dArgs &a, int64_t m,
                             hipStream_t stream)
{
    using G = RegTile<D>;
    const int64_t strips = (a.nx + G::COLS - 1) / G::COLS, rows = (a.ny + G::R - 1) / G::R;
    const int64_t ntiles = strips * rows;
    const int64_t blocks = (ntiles + kThreads / kWave - 1) / (kThreads / kWave);
    const int64_t grid = (blocks + 7) / 8 * 8;
    hipLaunchKernelGGL((level2d_reg_kernel<T, D>), dim3((unsigned)grid), dim3(kThreads), 0, stream,
                       src, dst, (int)a.nx, (int)a.ny, (int)strips, (int)ntiles, (int)(m & 1),
                       line_coef<T>(a.rx), line_coef<T>(a.ry), (T)a.gw, (T)a.ge, (T)a.gs, (T)a.gn);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_2d_t(const Grid2dArgs &a, hipStream_t stream)
{
    const T *src = static_cast<const T *>(a.u);
    T *dst = static_cast<T *>(a.work);
    int64_t launches = 0;
    for (int64_t s = 0; s < a.nsteps;) {
        // D levels per launch while D remain, then single levels
        const int d = a.nsteps - s >= a.depth ? a.depth : 1;
        hipError_t e;
        if (d == 4) e = launch_reg_levels<T, 4>(src, dst, a, a.step0 + s, stream);
        else if (d == 2) e = launch_reg_levels<T, 2>(src, dst, a, a.step0 + s, stream);
        else e = launch_reg_levels<T, 1>(src, dst, a, a.step0 + s, stream);
        if (e != hipSuccess) return e;
        s += d;
        ++launches;
        T *t = const_cast<T *>(src);
        src = dst;
        dst = t;
    }
    // after an odd number of launches the result sits in the workspace
    if (launches % 2 == 1)
        return hipMemcpyAsync(a.u, a.work, (size_t)(a.nx * a.ny) * sizeof(T),
                              hipMemcpyDeviceToDevice, stream);
    return hipSuccess;
}

}  // namespace

hipError_t launch_2d(int prec, const Grid2dArgs &a, hipStream_t stream)
{
    const int64_t tiles = ((a.nx + 47) / 48) * ((a.ny + 15) / 16);   // most tiles, D = 4
    // indices inside a launch are 32-bit: rows and columns below 2^31
    if (a.nx < 1 || a.ny < 1 || a.nx > 0x7fffff00LL || a.ny > 0x7fffff00LL || tiles > 0x7ffffff0LL ||
        (a.depth != 1 && a.depth != 2 && a.depth != 4))
        return hipErrorInvalidValue;
    if (prec == kFP64) return launch_2d_t<double>(a, stream);
    if (prec == kFP32) return launch_2d_t<float>(a, stream);
    return hipErrorInvalidValue;
}

}  // namespace ge
