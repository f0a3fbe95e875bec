// Tiled, temporally blocked GE sweep of one rod for gfx950.
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
#include "ge_kernels.h"
#include "ge_level.h"

namespace ge {
namespace {

using namespace dev;

// The lane's points of the window starting at ws (and their compensation
// and source profile where the form has them); guarded at a wall.
template <typename T, int K, bool COMP, bool SRC, bool WALL>
__device__ __forceinline__ void load_tile(const TileArgs &a, int64_t ws, T (&s)[K], T (&e)[K],
                                          T (&b)[K])
{
    const int64_t g0 = ws + (int64_t)threadIdx.x * K;
    const T *in_s = static_cast<const T *>(a.in);
    const T *in_e = in_s + a.estride;
    const T *srcb = static_cast<const T *>(a.src_b);
    if constexpr (WALL) {
        load_lane_guarded<T, K>(in_s + g0, g0, a.n, s);
        if constexpr (COMP) load_lane_guarded<T, K>(in_e + g0, g0, a.n, e);
        if constexpr (SRC) load_lane_guarded<T, K>(srcb + g0, g0, a.n, b);
    } else {
        load_lane<T, K>(in_s + g0, s);
        if constexpr (COMP) load_lane<T, K>(in_e + g0, e);
        if constexpr (SRC) load_lane<T, K>(srcb + g0, b);
    }
    if constexpr (!COMP) {
#pragma unroll
        for (int j = 0; j < K; ++j) e[j] = T(0);
    }
}

// Advance the loaded window of tile t (start ws) by the launch's levels and
// store its core.
template <typename T, int K, int NW, bool COMP, bool SRC, bool WALL>
__device__ __forceinline__ void sweep_tile(const TileArgs &a, int64_t t, int64_t ws, T (&s)[K],
                                           T (&e)[K], const T (&b)[K])
{
    constexpr int W = NW * kWave * K;
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    // the wave index is uniform across the wave: let the compiler keep
    // everything derived from it in scalar registers
    const int w = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int64_t n = a.n;
    const int64_t core_lo = t * a.core;
    const int64_t core_hi = min(core_lo + a.core, n);
    const int64_t g0 = ws + (int64_t)tid * K;       // global index of my first point

    T *out_s = static_cast<T *>(a.out);
    T *out_e = out_s + a.estride;

    __shared__ T xs[2][NW][4];
    __shared__ T xe[2][NW][4];
    __shared__ T xb[NW][2];

    // source profile of the neighbours' edge points (fixed for the launch)
    T bl = T(0), br = T(0);
    if constexpr (SRC) {
        bl = from_left(T(0), b[K - 1]);
        br = from_right(T(0), b[0]);
        if constexpr (NW > 1) {
            if (lane == 0) xb[w][0] = b[0];
            if (lane == kWave - 1) xb[w][1] = b[K - 1];
            __syncthreads();
            if (lane == 0 && w > 0) bl = xb[w - 1][1];
            if (lane == kWave - 1 && w < NW - 1) br = xb[w + 1][0];
        }
    }

    // wall geometry (uniform over the workgroup)
    const bool left_wall = WALL && (ws == 0);
    const int64_t qR = n - ws;                     // window position of the right wall node
    const bool ghost_in = WALL && (qR < W);
    const bool ghost_edge = WALL && (qR == W);
    const int kR = (int)(ghost_in ? (qR % K) : 0);
    const int lR = (int)(ghost_in ? (qR / K) : -1);          // thread holding it
    const int64_t qS = qR - 1;                     // window position of point n-1
    const bool has_S = WALL && (qS >= 0) && (qS < W);
    const int kS = (int)(has_S ? (qS % K) : 0);
    const int lS = (int)(has_S ? (qS / K) : -1);
    const bool flux_on = WALL && (a.flux != nullptr);
    const bool own_L = flux_on && left_wall && core_lo == 0;
    const bool own_R = flux_on && has_S && (n - 1 >= core_lo) && (n - 1 < core_hi);
    double accL = 0.0, accR = 0.0;
    if (own_L) accL = a.flux[0];
    if (own_R) accR = a.flux[1];

    const Coef<T> cf = lane_coef(Coef<T>{(T)a.c1, (T)a.c2, (T)a.cs, (T)a.e1, (T)a.e2, (T)a.es});
    FluxTap ft{own_L && tid == 0, accL, a.tau, a.h, 0.0};

    for_levels(a.level0, a.nlev, [&](auto par, int lev) {
        constexpr int p = decltype(par)::value;
        double glo = a.gl0, gln = a.gl0, gro = a.gr0, grn = a.gr0;
        if constexpr (WALL) {
            if (a.gl_t) { glo = a.gl_t[lev]; gln = a.gl_t[lev + 1]; }
            if (a.gr_t) { gro = a.gr_t[lev]; grn = a.gr_t[lev + 1]; }
            if (ghost_in) {
                T gh, gl_;
                split_wall<T, COMP>(gro, gh, gl_);
                put_at<T, K>(s, kR, tid == lR, gh);
                if constexpr (COMP) put_at<T, K>(e, kR, tid == lR, gl_);
            }
        }

        // Values entering the wave at its edges: from the neighbouring waves
        // through LDS, or (at an open window edge) anything -- those points
        // lie in the halo.  They ride in as the DPP fill of lanes 0 and 63.
        T xl = T(0), xl2 = T(0), xr = T(0), xr2 = T(0);
        T yl = T(0), yl2 = T(0), yr = T(0), yr2 = T(0);
        if constexpr (NW > 1) {
            const int pb = lev & 1;
            if (lane == 0) { xs[pb][w][0] = s[0]; xs[pb][w][1] = s[1]; }
            if (lane == kWave - 1) { xs[pb][w][2] = s[K - 2]; xs[pb][w][3] = s[K - 1]; }
            if constexpr (COMP) {
                if (lane == 0) { xe[pb][w][0] = e[0]; xe[pb][w][1] = e[1]; }
                if (lane == kWave - 1) { xe[pb][w][2] = e[K - 2]; xe[pb][w][3] = e[K - 1]; }
            }
            __syncthreads();
            const int wl = w > 0 ? w - 1 : 0, wr = w < NW - 1 ? w + 1 : NW - 1;
            xl = xs[pb][wl][3]; xr = xs[pb][wr][0];
            xl2 = xs[pb][wl][2]; xr2 = xs[pb][wr][1];
            if constexpr (COMP) {
                yl = xe[pb][wl][3]; yr = xe[pb][wr][0];
                yl2 = xe[pb][wl][2]; yr2 = xe[pb][wr][1];
            }
        }
        WallLevel<T> wlv{false, T(0)};
        T gr_hi = T(0), gr_lo = T(0), dgr = T(0);
        bool singR = false;
        if constexpr (WALL) {
            if (left_wall && w == 0) {
                T gh, glw;
                split_wall<T, COMP>(glo, gh, glw);
                xl = gh;
                if constexpr (COMP) yl = glw;
            }
            if (ghost_edge && w == NW - 1) {
                T gh, glw;
                split_wall<T, COMP>(gro, gh, glw);
                xr = gh;
                if constexpr (COMP) yr = glw;
            }
            wlv.dgl = (T)(gln - glo);
            wlv.isL = left_wall && (p == 1) && (tid == 0);
            ft.gln = gln;
            split_wall<T, COMP>(gro, gr_hi, gr_lo);
            dgr = (T)(grn - gro);
            singR = has_S && (((n - 1 + p) & 1) == 0);
        }
        const T an = SRC ? (T)a.src_a[lev] : T(0);
        Lone<T> lone{T(0), T(0)};
        if (WALL && singR)
            lone = right_lone<T, K, COMP, SRC>(s, e, b, kS, xl, yl, gr_hi, gr_lo, dgr, cf, an);
        ge_level<T, K, COMP, SRC, WALL, p, NW == 1 && !WALL>(s, e, b, bl, br, xl, xl2, xr, xr2,
                                                             yl, yl2, yr, yr2, cf, an, wlv, ft);
        if (WALL && singR) {
            put_at<T, K>(s, kS, tid == lS, lone.s);
            if constexpr (COMP) put_at<T, K>(e, kS, tid == lS, lone.e);
        }
        if (WALL && own_R) {
            // wall first difference at the new level, accumulated in FP64
            const double v = (double)get_at<T, K>(s, kS, T(0)) +
                             (COMP ? (double)get_at<T, K>(e, kS, T(0)) : 0.0);
            if (tid == lS) accR = accR + a.tau * (v - grn) / a.h;
        }
    });
    accL = ft.accL;

    if (own_L && tid == 0) a.flux[0] = accL;
    if (own_R && tid == lS) a.flux[1] = accR;

    if constexpr (WALL) {
        store_lane_guarded<T, K>(out_s + g0, g0, core_lo, core_hi, s);
        if constexpr (COMP) store_lane_guarded<T, K>(out_e + g0, g0, core_lo, core_hi, e);
    } else {
        store_lane_chunks<T, K>(out_s + g0, g0, core_lo, core_hi, s);
        if constexpr (COMP) store_lane_chunks<T, K>(out_e + g0, g0, core_lo, core_hi, e);
    }
}

template <typename T, int K, int NW, bool COMP, bool SRC, bool WALL>
__device__ __forceinline__ void run_tile(const TileArgs &a, int64_t t, int64_t ws)
{
    T s[K], e[K], b[K];
    load_tile<T, K, COMP, SRC, WALL>(a, ws, s, e, b);
    sweep_tile<T, K, NW, COMP, SRC, WALL>(a, t, ws, s, e, b);
}

template <typename T, int K, int NW, bool COMP, bool SRC>
__global__ __launch_bounds__(NW *kWave) void tile_kernel(TileArgs a)
{
    // Consecutive tiles go to the same XCD (workgroups are dealt to the 8
    // XCDs round-robin), so neighbouring halos share that XCD's L2.
    const int64_t per = gridDim.x / 8;
    const int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (t >= a.ntiles)
        return;
    const int64_t ws = (t == 0) ? 0 : t * a.core - a.halo;
    constexpr int64_t W = NW * kWave * K;
    const bool wall = (ws == 0) || (ws + W >= a.n);
    if (wall)
        run_tile<T, K, NW, COMP, SRC, true>(a, t, ws);
    else
        run_tile<T, K, NW, COMP, SRC, false>(a, t, ws);
}

// First tile whose window reaches the right wall (tiles from there on, and
// tile 0, take the wall path).
__device__ __host__ inline int64_t first_right_wall_tile(const TileArgs &a, int64_t W)
{
    const int64_t need = a.n + a.halo - W;       // t * core >= need
    int64_t t = need <= 0 ? 1 : (need + a.core - 1) / a.core;
    if (t < 1) t = 1;
    return t < a.ntiles ? t : a.ntiles;
}

// Persistent form for single-wave windows.  The first nint workgroups sweep
// the interior tiles round-robin, each loading its next tile while the
// current one advances, so the loads hide behind the levels; the remaining
// workgroups take one wall tile each.  Consecutive interior tiles are dealt
// to the same XCD, as in tile_kernel.
template <typename T, int K, bool COMP, bool SRC>
__global__ __launch_bounds__(kWave) void tile_persistent_kernel(TileArgs a, int nint)
{
    constexpr int64_t W = kWave * K;
    const int64_t tw = first_right_wall_tile(a, W);
    const int g = blockIdx.x;
    if (g >= nint) {
        const int64_t t = g == nint ? 0 : tw + (g - nint - 1);
        if (t < a.ntiles && (t == 0 || t >= tw))
            run_tile<T, K, 1, COMP, SRC, true>(a, t, t == 0 ? 0 : t * a.core - a.halo);
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
    load_tile<T, K, COMP, SRC, false>(a, t * a.core - a.halo, ns, ne, nb);
    for (;;) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            s[j] = ns[j];
            e[j] = ne[j];
            b[j] = nb[j];
        }
        const int64_t tn = t + nint;
        if (tn < tw)
            load_tile<T, K, COMP, SRC, false>(a, tn * a.core - a.halo, ns, ne, nb);
        sweep_tile<T, K, 1, COMP, SRC, false>(a, t, t * a.core - a.halo, s, e, b);
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
    const int64_t rounds = (interior + cap - 1) / cap;
    int64_t nint = (interior + rounds - 1) / rounds;
    nint = (nint + 7) / 8 * 8;
    hipLaunchKernelGGL((tile_persistent_kernel<T, K, COMP, SRC>), dim3((unsigned)(nint + walls)),
                       dim3(kWave), 0, stream, a, (int)nint);
    return hipGetLastError();
}

template <typename T, int K, int NW, bool COMP, bool SRC>
hipError_t launch_one(const TileArgs &a, hipStream_t stream)
{
    const int64_t grid = (a.ntiles + 7) / 8 * 8;
    hipLaunchKernelGGL((tile_kernel<T, K, NW, COMP, SRC>), dim3((unsigned)grid),
                       dim3(NW * kWave), 0, stream, a);
    return hipGetLastError();
}

template <typename T, int K, int NW, bool COMP>
hipError_t launch_src(bool src, const TileArgs &a, hipStream_t stream)
{
    return src ? launch_one<T, K, NW, COMP, true>(a, stream)
               : launch_one<T, K, NW, COMP, false>(a, stream);
}

template <typename T, int K, bool COMP>
hipError_t launch_nw(int nw, bool src, const TileArgs &a, hipStream_t stream)
{
    switch (nw) {
    case 1: return launch_src<T, K, 1, COMP>(src, a, stream);
    case 4: return launch_src<T, K, 4, COMP>(src, a, stream);
    default: return hipErrorInvalidValue;
    }
}

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
    case kFP64: return k == 2 || k == 4 || k == 8 || k == 16 || k == 32 || k == 64;
    case kFP32: return k == 4 || k == 8 || k == 16 || k == 32;
    case kFP32C: return k == 4 || k == 8 || k == 16;
    default: return false;
    }
}

hipError_t launch_tiles(int prec, int k, int nw, bool src, const TileArgs &a,
                        hipStream_t stream)
{
    switch (prec) {
    case kFP64:
        if (k == 2) return launch_nw<double, 2, false>(nw, src, a, stream);
        if (k == 4) return launch_nw<double, 4, false>(nw, src, a, stream);
        if (k == 8) return launch_nw<double, 8, false>(nw, src, a, stream);
        if (k == 16) return launch_nw<double, 16, false>(nw, src, a, stream);
        if (k == 32) return launch_nw<double, 32, false>(nw, src, a, stream);
        if (k == 64) return launch_nw<double, 64, false>(nw, src, a, stream);
        break;
    case kFP32:
        if (k == 4) return launch_nw<float, 4, false>(nw, src, a, stream);
        if (k == 8) return launch_nw<float, 8, false>(nw, src, a, stream);
        if (k == 16) return launch_nw<float, 16, false>(nw, src, a, stream);
        if (k == 32) return launch_nw<float, 32, false>(nw, src, a, stream);
        break;
    case kFP32C:
        if (k == 4) return launch_nw<float, 4, true>(nw, src, a, stream);
        if (k == 8) return launch_nw<float, 8, true>(nw, src, a, stream);
        if (k == 16) return launch_nw<float, 16, true>(nw, src, a, stream);
        break;
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
