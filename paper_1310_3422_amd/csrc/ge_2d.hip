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
// levels (D = 1, 2 or 4) of a tile of 128 columns by 16 (FP64) or 32 (FP32)
// rows: the tile with a halo of 2D points on every side goes from HBM to LDS
// (coalesced rows, every load of a thread issued before the first is used);
// each level runs the x-level on the still-valid region (which loses two
// points of width per side), overwriting it in place after a barrier, then
// the y-level likewise (two rows per side); the last y-level writes the tile
// straight to HBM.  Per launch the grid is read and written once: 16/D bytes
// per point and level in FP64.  Tiles are dealt to the XCDs in contiguous
// runs, so neighbours that re-read a tile's halo lines mostly run on the
// same L2 at about the same time.  Every point is advanced by the same
// operations whatever D is, so the depth changes no bits.
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

// Rows per tile: 16 in FP64 (less LDS, more tiles resident per CU: 12%
// faster than 32 rows at D = 1 on a 4096^2 grid, while the extra halo rows
// hit in L2), 32 in FP32 (3% faster than 16).
template <typename T, int D> struct Tile {
    static constexpr int TJ = sizeof(T) == 8 ? 16 : 32;
    static constexpr int H = 2 * D;                  // halo per side
    static constexpr int AW = kTI + 2 * H, AH = TJ + 2 * H;
    static constexpr int LPer = (AH * AW + kThreads - 1) / kThreads;              // loads
    static constexpr int XPer = (AH * (AW - 4) + kThreads - 1) / kThreads;        // x cells
    static constexpr int YPer = ((AH - 4) * (AW - 4) + kThreads - 1) / kThreads;  // y cells
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

template <typename T, int D>
__global__ __launch_bounds__(kThreads) void level2d_kernel(const T *__restrict__ in,
                                                           T *__restrict__ out, int nx, int ny,
                                                           int tiles_x, int ntiles, int p0,
                                                           Line<T> cx, Line<T> cy, T gw, T ge_,
                                                           T gs, T gn)
{
    using G = Tile<T, D>;
    constexpr int TJ = G::TJ, H = G::H, AW = G::AW, AH = G::AH;
    __shared__ T A[AH][AW];       // the tile and its halo, advanced in place
    const int per = gridDim.x / 8;
    const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;   // XCD-aware
    if (t >= ntiles)
        return;
    const int jb = (t / tiles_x) * TJ - H, ib = (t % tiles_x) * kTI - H;   // cell (0, 0)
    const int tid = threadIdx.x;
    // HBM -> LDS; cells on a wall hold it, cells past one are never read
    T v[G::LPer];
#pragma unroll
    for (int q = 0; q < G::LPer; ++q) {
        const int k = tid + q * kThreads;
        const int j = jb + k / AW, i = ib + k % AW;
        T x = T(0);
        if (k < AH * AW) {
            if (j == -1) x = gs;
            else if (j == ny) x = gn;
            else if (j >= 0 && j < ny) {
                if (i >= 0 && i < nx) x = in[(int64_t)j * nx + i];
                else if (i == -1) x = gw;
                else if (i == nx) x = ge_;
            }
        }
        v[q] = x;
    }
#pragma unroll
    for (int q = 0; q < G::LPer; ++q) {
        const int k = tid + q * kThreads;
        if (k < AH * AW) A[k / AW][k % AW] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int l = 0; l < D; ++l) {
        const int p = (p0 + l) & 1;
        // valid before this level: rows [2l, AH-2l), columns [2l, AW-2l)
        const int w = AW - 4 * l - 4;                 // columns [2l+2, AW-2l-2)
        const int hx = AH - 4 * l, hy = AH - 4 * l - 4;
        // x-level on every valid row; new values held in registers until
        // every thread has read its old ones
        T xv[G::XPer];
#pragma unroll
        for (int q = 0; q < G::XPer; ++q) {
            const int k = tid + q * kThreads;
            T y = T(0);
            if (k < w * hx) {
                const int r = 2 * l + k / w, c = 2 * l + 2 + k % w;
                const int j = jb + r, i = ib + c;
                y = A[r][c];
                if (j >= 0 && j < ny && i >= 0 && i < nx)
                    y = level1d(A[r][c - 2], A[r][c - 1], y, A[r][c + 1], A[r][c + 2], i, nx, p, cx);
            }
            xv[q] = y;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < G::XPer; ++q) {
            const int k = tid + q * kThreads;
            if (k < w * hx) A[2 * l + k / w][2 * l + 2 + k % w] = xv[q];
        }
        __syncthreads();
        if (l == D - 1) {
            // the last y-level covers exactly the tile: straight to HBM
#pragma unroll
            for (int q = 0; q < G::YPer; ++q) {
                const int k = tid + q * kThreads;
                if (k < w * hy) {
                    const int r = 2 * l + 2 + k / w, c = 2 * l + 2 + k % w;
                    const int j = jb + r, i = ib + c;
                    if (j < ny && i < nx)
                        out[(int64_t)j * nx + i] = level1d(A[r - 2][c], A[r - 1][c], A[r][c],
                                                           A[r + 1][c], A[r + 2][c], j, ny, p, cy);
                }
            }
        } else {
            T yv[G::YPer];
#pragma unroll
            for (int q = 0; q < G::YPer; ++q) {
                const int k = tid + q * kThreads;
                T y = T(0);
                if (k < w * hy) {
                    const int r = 2 * l + 2 + k / w, c = 2 * l + 2 + k % w;
                    const int j = jb + r, i = ib + c;
                    y = A[r][c];
                    if (j >= 0 && j < ny && i >= 0 && i < nx)
                        y = level1d(A[r - 2][c], A[r - 1][c], y, A[r + 1][c], A[r + 2][c], j, ny, p,
                                    cy);
                }
                yv[q] = y;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < G::YPer; ++q) {
                const int k = tid + q * kThreads;
                if (k < w * hy) A[2 * l + 2 + k / w][2 * l + 2 + k % w] = yv[q];
            }
            __syncthreads();
        }
    }
}

template <typename T> Line<T> line_coef(double r)
{
    return Line<T>{(T)((r + r * r) / (1.0 + 2.0 * r)), (T)(r * r / (1.0 + 2.0 * r)),
                   (T)(r / (1.0 + r))};
}

template <typename T, int D>
hipError_t launch_levels(const T *src, T *dst, const Grid2dArgs &a, int64_t m, hipStream_t stream)
{
    const int64_t tx = (a.nx + kTI - 1) / kTI, ty = (a.ny + Tile<T, D>::TJ - 1) / Tile<T, D>::TJ;
    const int64_t ntiles = tx * ty, grid = (ntiles + 7) / 8 * 8;
    hipLaunchKernelGGL((level2d_kernel<T, D>), dim3((unsigned)grid), dim3(kThreads), 0, stream, src,
                       dst, (int)a.nx, (int)a.ny, (int)tx, (int)ntiles, (int)(m & 1),
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
        if (d == 4) e = launch_levels<T, 4>(src, dst, a, a.step0 + s, stream);
        else if (d == 2) e = launch_levels<T, 2>(src, dst, a, a.step0 + s, stream);
        else e = launch_levels<T, 1>(src, dst, a, a.step0 + s, stream);
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
    const int64_t tiles = ((a.nx + kTI - 1) / kTI) * ((a.ny + 15) / 16);
    // indices inside a launch are 32-bit: rows and columns below 2^31
    if (a.nx < 1 || a.ny < 1 || a.nx > 0x7fffff00LL || a.ny > 0x7fffff00LL || tiles > 0x7ffffff0LL ||
        (a.depth != 1 && a.depth != 2 && a.depth != 4))
        return hipErrorInvalidValue;
    if (prec == kFP64) return launch_2d_t<double>(a, stream);
    if (prec == kFP32) return launch_2d_t<float>(a, stream);
    return hipErrorInvalidValue;
}

}  // namespace ge
