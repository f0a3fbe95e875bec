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
// levels (D = 1, 2 or 4) of a tile held in registers: lane l holds two
// neighbouring columns (an even one and the next) for N rows.  A row's
// x-level takes its neighbours from the lanes beside it by DPP shifts -- at
// levels of even index a lane's two points are a pair, at odd ones each
// pairs with a point of the neighbouring lane -- and a column's y-level from
// the lane's own rows, where the parity of every row is known at compile
// time.  The valid lanes and rows shrink by one lane (two columns) and two
// rows per side and level (a recomputed halo).  Per launch the grid is read
// and written once: 16/D bytes per point and level in FP64.  Every point is
// advanced by the same operations whatever D is and wherever its tile lies,
// so the depth changes no bits.
//
// Walls are constant in time (west, east, south, north); the values beside
// a wall read the wall, which a halo lane or row holds.  Tiles whose halo
// reaches a wall take a second code path (per-lane column tests, per-row
// tests); the others test nothing.
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

// A pair member's new value u + c1 D_e + c2 D_q, a lone point's (beside a
// wall) u + cs D_e; D = second difference, D_e = d_e - d_{e-1}.
template <typename T>
__device__ __forceinline__ T pair_upd(T u, T De, T Dq, const Line<T> &c)
{
    if constexpr (sizeof(T) == 8) return fma(c.c2, Dq, fma(c.c1, De, u));
    else return u + fmaf(c.c2, Dq, c.c1 * De);
}
template <typename T>
__device__ __forceinline__ T lone_upd(T u, T De, const Line<T> &c)
{
    if constexpr (sizeof(T) == 8) return fma(c.cs, De, u);
    else return u + c.cs * De;
}

using dev::kWave;

template <typename T>
__device__ __forceinline__ T shr1(T v) { return dev::from_left_open(v); }    // lane l-1
template <typename T>
__device__ __forceinline__ T shl1(T v) { return dev::from_right_open(v); }   // lane l+1

template <int D> struct RegTile {
    static constexpr int H = 2 * D;                            // halo rows per side
    static constexpr int R = D == 4 ? 20 : 24;                 // output rows per wave
    static constexpr int N = R + 2 * H;                        // rows held
    static constexpr int LANES = kWave - 2 * D;                // output lanes (D halo lanes a side)
    static constexpr int COLS = 2 * LANES;                     // output columns per wave
};

// What a lane's two columns are, for tiles that reach the west or east wall
// (x0 + 2 lane and the next; only points inside the grid change, and a point
// whose partner lies outside the grid is alone beside the wall).
struct ColFlags {
    bool a_in, b_in;       // the columns lie inside the grid
    bool a_lone0;          // even levels: a's partner b is the east ghost
    bool a_lone1, b_lone1; // odd levels: a is column 0; b's partner is the east ghost
};

// The x-level of one row: a, b the lane's two points (old values in, new
// out).  P: the level's parity; XW: the tile reaches a west or east wall.
template <typename T, int P, bool XW>
__device__ __forceinline__ void xlevel(T &a, T &b, const ColFlags &f, const Line<T> &c)
{
    const T l1 = shr1(b);            // column 2l - 1
    const T r1 = shl1(a);            // column 2l + 2
    const T dm = a - l1, d0 = b - a, dp = r1 - b;
    const T Da = d0 - dm, Db = dp - d0;
    T na, nb;
    if constexpr (P == 0) {
        // pairs (2l, 2l+1)
        na = pair_upd(a, Da, Db, c);
        nb = pair_upd(b, Db, Da, c);
        if constexpr (XW) {
            if (f.a_lone0) na = lone_upd(a, Da, c);
        }
    } else {
        // pairs (2l-1, 2l) and (2l+1, 2l+2): the partners' second
        // differences come from the lanes beside
        const T Dl = shr1(Db);       // D of column 2l - 1
        const T Dr = shl1(Da);       // D of column 2l + 2
        na = pair_upd(a, Da, Dl, c);
        nb = pair_upd(b, Db, Dr, c);
        if constexpr (XW) {
            if (f.a_lone1) na = lone_upd(a, Da, c);
            if (f.b_lone1) nb = lone_upd(b, Db, c);
        }
    }
    if constexpr (XW) {
        if (!f.a_in) na = a;
        if (!f.b_in) nb = b;
    }
    a = na;
    b = nb;
}

// The y-level of one column, rows [LO, HI) of u (old values of rows LO-2 ..
// HI+1 used), in place.  Row q is grid row jb + q, and jb is even, so the
// pairing of row q follows q: pairs (q, q+1) with q + P even.  The second
// differences roll along the column (each from old values, computed before
// the row below it is overwritten).  XW: the column may lie outside the grid
// (cin false: it keeps its values).  YW: the tile reaches the south or north
// wall: rows outside the grid keep their values, and a row whose partner
// lies outside is alone beside the wall.
template <typename T, int N, int LO, int HI, int P, bool XW, bool YW>
__device__ __forceinline__ void ylevel(T (&u)[N], bool cin, int jb, int ny, const Line<T> &c)
{
    static_assert(LO >= 2 && HI + 2 <= N, "rows read");
    T Dp = (u[LO] - u[LO - 1]) - (u[LO - 1] - u[LO - 2]);   // row LO - 1
    T Dc = (u[LO + 1] - u[LO]) - (u[LO] - u[LO - 1]);       // row LO
#pragma unroll
    for (int q = LO; q < HI; ++q) {
        const T Dn = (u[q + 2] - u[q + 1]) - (u[q + 1] - u[q]);   // row q + 1
        const bool left = ((q + P) & 1) == 0;                       // compile-time
        T v = pair_upd(u[q], Dc, left ? Dn : Dp, c);
        if constexpr (YW) {
            const int j = jb + q, jq = left ? j + 1 : j - 1;
            if (jq < 0 || jq >= ny) v = lone_upd(u[q], Dc, c);
            if (j < 0 || j >= ny) v = u[q];
        }
        if constexpr (XW) {
            if (!cin) v = u[q];
        }
        u[q] = v;
        Dp = Dc;
        Dc = Dn;
    }
}

template <typename T, int D, int L, int P, bool XW, bool YW>
__device__ __forceinline__ void tile_levels(T (&ua)[RegTile<D>::N], T (&ub)[RegTile<D>::N],
                                            const ColFlags &f, int jb, int ny, const Line<T> &cx,
                                            const Line<T> &cy)
{
    constexpr int N = RegTile<D>::N;
    // x-level on rows [2L, N - 2L)
#pragma unroll
    for (int q = 2 * L; q < N - 2 * L; ++q) {
        if constexpr (YW) {
            const int j = jb + q;
            if (j < 0 || j >= ny) continue;   // wave-uniform
        }
        xlevel<T, P, XW>(ua[q], ub[q], f, cx);
    }
    if constexpr (L + 1 < D) {
        ylevel<T, N, 2 * L + 2, N - 2 * L - 2, P, XW, YW>(ua, f.a_in, jb, ny, cy);
        ylevel<T, N, 2 * L + 2, N - 2 * L - 2, P, XW, YW>(ub, f.b_in, jb, ny, cy);
        tile_levels<T, D, L + 1, 1 - P, XW, YW>(ua, ub, f, jb, ny, cx, cy);
    }
}

// One wave's tile: levels m .. m+D-1 (P = m mod 2) of lanes' column pairs
// x0 + 2 lane, rows jb .. jb+N-1; writes the core (lanes D .. 63-D, rows
// H .. H+R-1) of the last level to `out`.
template <typename T, int D, int P, bool XW, bool YW>
__device__ __forceinline__ void tile2d(const T *__restrict__ in, T *__restrict__ out, int nx,
                                       int ny, int x0, int jb, const Line<T> &cx,
                                       const Line<T> &cy, T gw, T ge_, T gs, T gn)
{
    using G = RegTile<D>;
    constexpr int N = G::N, H = G::H, R = G::R;
    const int lane = threadIdx.x % kWave;
    const int ia = x0 + 2 * lane, ib = ia + 1;
    ColFlags f;
    f.a_in = ia >= 0 && ia < nx;
    f.b_in = ib >= 0 && ib < nx;
    f.a_lone0 = ib >= nx;
    f.a_lone1 = ia == 0;
    f.b_lone1 = ib + 1 >= nx;
    T ua[N], ub[N];
    auto ghost = [&](int i) { return i == -1 ? gw : i == nx ? ge_ : T(0); };
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const int j = jb + q;                 // wave-uniform
        T xa = T(0), xb = T(0);
        if (j == -1) {
            xa = xb = gs;
        } else if (j == ny) {
            xa = xb = gn;
        } else if (!YW || (j >= 0 && j < ny)) {
            const T *row = in + (int64_t)j * nx;
            if (!XW || f.a_in) xa = row[ia];
            else xa = ghost(ia);
            if (!XW || f.b_in) xb = row[ib];
            else xb = ghost(ib);
        }
        ua[q] = xa;
        ub[q] = xb;
    }
    tile_levels<T, D, 0, P, XW, YW>(ua, ub, f, jb, ny, cx, cy);
    // the last y-level, the core straight to HBM
    constexpr int PL = (P + D - 1) & 1;
    ylevel<T, N, H, H + R, PL, XW, YW>(ua, f.a_in, jb, ny, cy);
    ylevel<T, N, H, H + R, PL, XW, YW>(ub, f.b_in, jb, ny, cy);
    if (lane < D || lane >= kWave - D)
        return;
#pragma unroll
    for (int q = H; q < H + R; ++q) {
        const int j = jb + q;
        if (j >= ny) break;                   // wave-uniform
        T *row = out + (int64_t)j * nx;
        if (!XW || f.a_in) row[ia] = ua[q];
        if (!XW || f.b_in) row[ib] = ub[q];
    }
}

template <typename T, int D, int P>
__global__ __launch_bounds__(kThreads) void level2d_reg_kernel(const T *__restrict__ in,
                                                               T *__restrict__ out, int nx, int ny,
                                                               int strips, int ntiles,
                                                               Line<T> cx, Line<T> cy, T gw,
                                                               T ge_, T gs, T gn)
{
    using G = RegTile<D>;
    const int per = gridDim.x / 8;
    const int b = (blockIdx.x % 8) * per + blockIdx.x / 8;   // XCD-aware
    // this wave's tile (wave-uniform: row addresses stay in scalar registers)
    const int t = b * (kThreads / kWave) + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (t >= ntiles)
        return;
    const int x0 = (t % strips) * G::COLS - 2 * D;
    const int jb = (t / strips) * G::R - G::H;
    // the tile's halo reaches a wall (a ghost column or row is read)
    const bool xw = x0 < 0 || x0 + 2 * kWave > nx;
    const bool yw = jb < 0 || jb + G::N > ny;
    if (xw) {
        if (yw) tile2d<T, D, P, true, true>(in, out, nx, ny, x0, jb, cx, cy, gw, ge_, gs, gn);
        else tile2d<T, D, P, true, false>(in, out, nx, ny, x0, jb, cx, cy, gw, ge_, gs, gn);
    } else {
        if (yw) tile2d<T, D, P, false, true>(in, out, nx, ny, x0, jb, cx, cy, gw, ge_, gs, gn);
        else tile2d<T, D, P, false, false>(in, out, nx, ny, x0, jb, cx, cy, gw, ge_, gs, gn);
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
    if (m & 1)
        hipLaunchKernelGGL((level2d_reg_kernel<T, D, 1>), dim3((unsigned)grid), dim3(kThreads), 0,
                           stream, src, dst, (int)a.nx, (int)a.ny, (int)strips, (int)ntiles,
                           line_coef<T>(a.rx), line_coef<T>(a.ry), (T)a.gw, (T)a.ge, (T)a.gs,
                           (T)a.gn);
    else
        hipLaunchKernelGGL((level2d_reg_kernel<T, D, 0>), dim3((unsigned)grid), dim3(kThreads), 0,
                           stream, src, dst, (int)a.nx, (int)a.ny, (int)strips, (int)ntiles,
                           line_coef<T>(a.rx), line_coef<T>(a.ry), (T)a.gw, (T)a.ge, (T)a.gs,
                           (T)a.gn);
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
    const int64_t tiles = ((a.nx + 111) / 112) * ((a.ny + 19) / 20);   // most tiles, D = 4
    // indices inside a launch are 32-bit: rows and columns below 2^31
    if (a.nx < 1 || a.ny < 1 || a.nx > 0x7fffff00LL || a.ny > 0x7fffff00LL || tiles > 0x7ffffff0LL ||
        (a.depth != 1 && a.depth != 2 && a.depth != 4))
        return hipErrorInvalidValue;
    if (prec == kFP64) return launch_2d_t<double>(a, stream);
    if (prec == kFP32) return launch_2d_t<float>(a, stream);
    return hipErrorInvalidValue;
}

}  // namespace ge
