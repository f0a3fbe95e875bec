// Tiled, temporally blocked GE sweep of one rod for gfx950: the kernels and
// their launch templates, instantiated by ge_sweep*.hip (the precisions and
// row widths are spread over several files so that they compile in
// parallel).
//
// One workgroup of NW waves owns a window of W = NW*64*K points; lane l of
// wave w holds points (64w + l)K .. (64w + l)K + K-1 of the window in
// registers and the window advances nlev levels there (ge_level.h).  Edge
// values cross waves through LDS, one barrier per level.  A value at level
// m+1 depends on level-m values at most two places away, and after the first
// level the invalid region entering from an open window edge grows by one
// point per level, so a halo of H >= nlev + 1 points each side leaves the
// core exact; halos are recomputed by the neighbouring tiles instead of being
// exchanged, and no data crosses workgroups inside a launch.
#pragma once

#include "ge_kernels.h"
#include "ge_level.h"
#include "ge_tile.h"

namespace ge {
namespace {

using namespace dev;

// First tile whose window reaches the right wall (tiles from there on, and
// tile 0, take the wall path).
__device__ __host__ inline int64_t first_right_wall_tile(const TileArgs &a, int64_t W)
{
    const int64_t need = a.n + a.halo - W;       // t * core >= need
    int64_t t = need <= 0 ? 1 : (need + a.core - 1) / a.core;
    if (t < 1) t = 1;
    return t < a.ntiles ? t : a.ntiles;
}

// The tiles of a launch.  PART 0: every tile, each taking the wall path or
// not.  The wall path (guarded loads, runtime wall positions, the flux, the
// source profile kept for the lone points) needs far more registers than an
// interior tile, and a kernel holds the registers of its widest path in
// every wave; so rods of very many tiles run two kernels per launch: PART 2
// takes tile 0 and the tiles reaching the right wall (one workgroup each),
// PART 1 the interior tiles 1 .. tw-1 at the interior path's occupancy.  The
// wall kernel costs about one tile's time (it runs beside the interior one
// when the caller gives a second stream, else before it), which pays only
// when a CU sweeps hundreds of tiles per launch.
template <typename T, int K, int NW, bool COMP, bool SRC, int PART>
__global__ __launch_bounds__(NW *kWave) void tile_kernel(TileArgs a)
{
    constexpr int64_t W = NW * kWave * K;
    if constexpr (PART == 2) {
        const int64_t tw = first_right_wall_tile(a, W);
        const int64_t t = blockIdx.x == 0 ? 0 : tw + blockIdx.x - 1;
        if (t < a.ntiles)
            run_tile<T, K, NW, COMP, SRC, true>(a, threadIdx.x, t, t == 0 ? 0 : t * a.core - a.halo);
        return;
    }
    // Consecutive tiles go to the same XCD (workgroups are dealt to the 8
    // XCDs round-robin), so neighbouring halos share that XCD's L2.
    const int64_t per = gridDim.x / 8;
    const int64_t i = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if constexpr (PART == 1) {
        const int64_t t = 1 + i;
        if (t < first_right_wall_tile(a, W))
            run_tile<T, K, NW, COMP, SRC, false>(a, threadIdx.x, t, t * a.core - a.halo);
        return;
    }
    const int64_t t = i;
    if (t >= a.ntiles)
        return;
    const int64_t ws = (t == 0) ? 0 : t * a.core - a.halo;
    const bool wall = (ws == 0) || (ws + W >= a.n);
    if (wall)
        run_tile<T, K, NW, COMP, SRC, true>(a, threadIdx.x, t, ws);
    else
        run_tile<T, K, NW, COMP, SRC, false>(a, threadIdx.x, t, ws);
}

// Persistent form for single-wave windows.  The first nint workgroups sweep
// the interior tiles round-robin, each loading its next tile while the
// current one advances, so the loads hide behind the levels; the remaining
// workgroups take one wall tile each, concurrently (a workgroup sweeps about
// ten tiles per launch here, so a separate wall launch would cost about a
// tenth; the prefetch registers exceed the wall path's anyway).
// Consecutive interior tiles are dealt to the same XCD, as in tile_kernel.
template <typename T, int K, bool COMP, bool SRC>
__global__ __launch_bounds__(kWave) void tile_persistent_kernel(TileArgs a, int nint)
{
    constexpr int64_t W = kWave * K;
    const int64_t tw = first_right_wall_tile(a, W);
    const int g = blockIdx.x;
    if (g >= nint) {
        const int64_t t = g == nint ? 0 : tw + (g - nint - 1);
        if (t < a.ntiles && (t == 0 || t >= tw))
            run_tile<T, K, 1, COMP, SRC, true>(a, threadIdx.x, t, t == 0 ? 0 : t * a.core - a.halo);
        return;
    }
    const int per = nint / 8;
    const int gx = (g % 8) * per + g / 8;        // XCD-aware order (nint is a multiple of 8)
    int64_t t = 1 + gx;
    if (t >= tw)
        return;
    // every tile's values reach the sweep registers by a copy from the
    // prefetch registers, so the loads pending during a sweep are only the
    // next tile's and the sweep never waits for them
    T s[K], e[K], b[K], ns[K], ne[K], nb[K];
    load_tile<T, K, COMP, SRC, false>(a, threadIdx.x, t * a.core - a.halo, ns, ne, nb);
    for (;;) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            s[j] = ns[j];
            e[j] = ne[j];
            b[j] = nb[j];
        }
        const int64_t tn = t + nint;
        if (tn < tw)
            load_tile<T, K, COMP, SRC, false>(a, threadIdx.x, tn * a.core - a.halo, ns, ne, nb);
        sweep_tile<T, K, 1, COMP, SRC, false>(a, threadIdx.x, t, t * a.core - a.halo, s, e, b);
        if (tn >= tw)
            break;
        t = tn;
    }
}

template <typename T, int K, bool COMP, bool SRC>
hipError_t launch_persistent(const TileArgs &a, hipStream_t stream)
{
    // resident single-wave workgroups per CU for this kernel, and CUs
    static int per_cu = 0, ncu = 0;
    if (per_cu == 0) {
        int dev = 0, nb = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, tile_persistent_kernel<T, K, COMP, SRC>, kWave, 0) != hipSuccess ||
            nb < 1 || ncu < 1)
            return hipErrorInvalidValue;
        per_cu = nb;
    }
    constexpr int64_t W = kWave * K;
    const int64_t tw = first_right_wall_tile(a, W);
    const int64_t interior = tw - 1;
    const int64_t walls = 1 + (a.ntiles - tw);
    // as many workgroups as stay resident, trimmed so that every one gets
    // the same number of tiles (to one), in multiples of 8
    const int64_t cap = (int64_t)per_cu * ncu;
    const int64_t rounds = interior < 1 ? 1 : (interior + cap - 1) / cap;
    int64_t nint = interior < 1 ? 0 : (interior + rounds - 1) / rounds;
    nint = (nint + 7) / 8 * 8;
    hipLaunchKernelGGL((tile_persistent_kernel<T, K, COMP, SRC>), dim3((unsigned)(nint + walls)),
                       dim3(kWave), 0, stream, a, (int)nint);
    return hipGetLastError();
}

template <typename T, int K, int NW, bool COMP, bool SRC>
hipError_t launch_one(const TileArgs &a, hipStream_t stream, const SideStream *side)
{
    constexpr int64_t W = NW * kWave * K;
    // compute units (split launches only where a CU sweeps 128 tiles or more)
    static int ncu = 0;
    if (ncu == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            ncu < 1)
            ncu = 256;
    }
    const int64_t tw = a.ntiles >= 3 ? first_right_wall_tile(a, W) : 1;
    if (tw - 1 < 128 * (int64_t)ncu) {
        // no interior tile: every tile in one launch
        const int64_t grid = (a.ntiles + 7) / 8 * 8;
        hipLaunchKernelGGL((tile_kernel<T, K, NW, COMP, SRC, 0>), dim3((unsigned)grid),
                           dim3(NW * kWave), 0, stream, a);
        return hipGetLastError();
    }
    // the wall kernel (a few workgroups, each about one tile's time) beside
    // the interior one when a side stream is given, else before it
    const int64_t walls = 1 + (a.ntiles - tw);
    hipError_t e = hipSuccess;
    hipStream_t ws = stream;
    if (side) {
        if ((e = hipEventRecord(side->fork, stream)) != hipSuccess ||
            (e = hipStreamWaitEvent(side->stream, side->fork, 0)) != hipSuccess)
            return e;
        ws = side->stream;
    }
    hipLaunchKernelGGL((tile_kernel<T, K, NW, COMP, SRC, 2>), dim3((unsigned)walls),
                       dim3(NW * kWave), 0, ws, a);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if (side && (e = hipEventRecord(side->join, side->stream)) != hipSuccess)
        return e;
    const int64_t grid = (tw - 1 + 7) / 8 * 8;
    hipLaunchKernelGGL((tile_kernel<T, K, NW, COMP, SRC, 1>), dim3((unsigned)grid),
                       dim3(NW * kWave), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    return side ? hipStreamWaitEvent(stream, side->join, 0) : hipSuccess;
}

template <typename T, int K, int NW, bool COMP>
hipError_t launch_src(bool src, const TileArgs &a, hipStream_t stream, const SideStream *side)
{
    return src ? launch_one<T, K, NW, COMP, true>(a, stream, side)
               : launch_one<T, K, NW, COMP, false>(a, stream, side);
}

template <typename T, int K, bool COMP>
hipError_t launch_nw(int nw, bool src, const TileArgs &a, hipStream_t stream,
                     const SideStream *side)
{
    switch (nw) {
    case 1: return launch_src<T, K, 1, COMP>(src, a, stream, side);
    case 4: return launch_src<T, K, 4, COMP>(src, a, stream, side);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

// One launch of the per-tile kernels for a row width of each file's set.
hipError_t launch_tiles_fp64_narrow(int k, int nw, bool src, const TileArgs &a,
                                    hipStream_t stream, const SideStream *side);
hipError_t launch_tiles_fp64_mid(int k, int nw, bool src, const TileArgs &a,
                                 hipStream_t stream, const SideStream *side);
hipError_t launch_tiles_fp64_wide(int k, int nw, bool src, const TileArgs &a,
                                  hipStream_t stream, const SideStream *side);
hipError_t launch_tiles_fp32(bool comp, int k, int nw, bool src, const TileArgs &a,
                             hipStream_t stream, const SideStream *side);

}  // namespace ge
