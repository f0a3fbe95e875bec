// Internal interface between the C ABI (ge_api.hip) and the sweep kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ge {

enum Prec : int { kFP64 = 0, kFP32 = 1, kFP32C = 2 };

// Status words a launch may raise (host-mapped memory owned by a plan): a
// stored value was NaN or infinite; a wave's wait for a neighbouring wave
// gave up (the launch's results are then not valid).
enum StatusWord : int { kStatusNonfinite = 0, kStatusWaitGaveUp = 1, kStatusWords = 2 };

// One launch of the tiled sweep: every workgroup loads a window of
// W = NW*64*K consecutive points of one rod, advances it `nlev` levels in
// registers and writes back its core of `core` points.
struct TileArgs {
    const void *in;          // level buffer read (s block then e block for FP32C)
    void *out;               // level buffer written (may equal `in` only when ntiles == 1)
    const void *src_b;       // source profile b(x_i) or null
    const double *gl_t;      // wall values g_L(t_m), m = level0 .. level0+nlev, or null
    const double *gr_t;      // likewise g_R
    const double *src_a;     // a(t_m + tau/2), m = level0 .. level0+nlev-1, or null
    double *flux;            // 2 doubles accumulated in FP64, or null
    int64_t n;               // interior points
    int64_t core;            // core points per tile
    int64_t ntiles;
    int64_t level0;          // global index of the first level of this launch
    int64_t estride;         // FP32C: element offset of the e block of `in`
    int64_t estride_out;     // FP32C: element offset of the e block of `out`
    int32_t halo;            // window points each side of the core
    int32_t nlev;            // levels advanced by this launch
    double c1, c2, cs;       // (r+r^2)/(1+2r), r^2/(1+2r), r/(1+r)
    double e1, e2, es;       // tau(1+r)/(1+2r), tau r/(1+2r), tau/(1+r)
    double gl0, gr0;         // constant walls (used when gl_t / gr_t are null)
    double tau, h;           // for the wall-flux diagnostic
    // sub-domain scheme (launch_sdc): core and halo count sub-domain
    // couples (one per lane), nsdc of them in the rod
    int64_t nsdc;
    double ca;               // (1-r)/(1+r)
    // host-mapped status words of the plan (StatusWord in ge_level.h), or
    // null: a launch that stores a NaN or infinite value sets word 0
    int *status;
};

// Supported (precision, points per lane, waves per workgroup) choices.
bool tile_config_supported(int prec, int k, int nw);

// A second stream and two events on which a launch that splits its wall
// tiles from its interior tiles runs the wall kernel beside the interior
// one (forked from and joined back into the launch stream).
struct SideStream {
    hipStream_t stream;
    hipEvent_t fork, join;
};

// Enqueue one launch.  Returns hipSuccess or the launch error.  side: null,
// or a SideStream for the wall kernel of a split launch.
hipError_t launch_tiles(int prec, int k, int nw, bool src, const TileArgs &a,
                        hipStream_t stream, const SideStream *side = nullptr);

// Persistent single-wave form (tile_persistent_kernel): interior tiles
// round-robin with the next tile's load overlapping the current sweep.
bool persistent_supported(int prec, int k);
hipError_t launch_tiles_persistent(int prec, int k, bool src, const TileArgs &a,
                                   hipStream_t stream);

// Sub-domain scheme with sub-domains of k = K/2 nodes, one sub-domain couple
// (K nodes) per lane, windows of nw x 64 couples, nw waves per workgroup
// exchanging edge values through LDS (ge_sdc.hip).
bool sdc_supported(int prec, int k);
bool sdc_waves_supported(int nw);
hipError_t launch_sdc(int prec, int k, int nw, const TileArgs &a, hipStream_t stream);
// Persistent form of the same (needs ntiles >= 3, out != in and at most
// kSdcMaxLevels levels): resident workgroups, the next window copied into
// LDS during the levels.
constexpr int kSdcMaxLevels = 64;
hipError_t launch_sdc_persistent(int prec, int k, int nw, const TileArgs &a, hipStream_t stream);

// Elementwise conversions for the compensated pair.
hipError_t launch_comp_to_fp64(const float *pair, double *x, int64_t n, hipStream_t s);
hipError_t launch_comp_from_fp64(const double *x, float *pair, int64_t n, hipStream_t s);

}  // namespace ge
