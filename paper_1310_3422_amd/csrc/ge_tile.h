// One window of the tiled GE sweep (Section 2, two-point groups), shared by
// the single-rod kernels (ge_sweep_kernels.h) and the multi-pass tasks of the
// batch kernel (ge_batch.hip).
//
// A window of W = NW*64*K consecutive points starts at ws; thread `tid`
// (0 .. NW*64-1 of the threads sweeping it) holds points ws + tid*K ..
// ws + tid*K + K-1 in registers, the window advances a.nlev levels there
// (ge_level.h) and the core of tile t, [t*core, t*core + core), is stored.
// Edge values cross waves through LDS with one barrier per level (NW > 1);
// a single-wave window (NW = 1) has no barrier, so waves of one workgroup
// may sweep different windows.
#pragma once

#include "ge_kernels.h"
#include "ge_level.h"

namespace ge {
namespace dev {

// The lane's points of the window starting at ws (and their compensation
// and source profile where the form has them); guarded at a wall.
template <typename T, int K, bool COMP, bool SRC, bool WALL>
__device__ __forceinline__ void load_tile(const TileArgs &a, int tid, int64_t ws, T (&s)[K],
                                          T (&e)[K], T (&b)[K])
{
    const int64_t g0 = ws + (int64_t)tid * K;
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
__device__ __forceinline__ void sweep_tile(const TileArgs &a, int tid, int64_t t, int64_t ws,
                                           T (&s)[K], T (&e)[K], const T (&b)[K])
{
    constexpr int W = NW * kWave * K;
    const int lane = tid & (kWave - 1);
    // the wave index is uniform across the wave: let the compiler keep
    // everything derived from it in scalar registers
    const int w = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int64_t n = a.n;
    const int64_t core_lo = t * a.core;
    const int64_t core_hi = min(core_lo + a.core, n);
    const int64_t g0 = ws + (int64_t)tid * K;       // global index of my first point

    T *out_s = static_cast<T *>(a.out);
    T *out_e = out_s + a.estride_out;

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

    // Interior tiles with a source form each point's source weight for both
    // parities once (source_weights); wall tiles keep the profile for the
    // lone points' formulas.  The same bits either way.
    constexpr bool COMB = SRC && !WALL;
    T B0[COMB ? K : 1], B1[COMB ? K : 1];
    if constexpr (COMB) {
        source_weights<T, K, 0>(b, bl, br, cf, B0);
        source_weights<T, K, 1>(b, bl, br, cf, B1);
    }

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
        if constexpr (COMB) {
            if constexpr (p == 0)
                ge_level<T, K, COMP, 2, WALL, p, NW == 1 && !WALL>(s, e, B0, bl, br, xl, xl2, xr,
                                                                   xr2, yl, yl2, yr, yr2, cf, an,
                                                                   wlv, ft);
            else
                ge_level<T, K, COMP, 2, WALL, p, NW == 1 && !WALL>(s, e, B1, bl, br, xl, xl2, xr,
                                                                   xr2, yl, yl2, yr, yr2, cf, an,
                                                                   wlv, ft);
        } else {
            ge_level<T, K, COMP, SRC ? 1 : 0, WALL, p, NW == 1 && !WALL>(
                s, e, b, bl, br, xl, xl2, xr, xr2, yl, yl2, yr, yr2, cf, an, wlv, ft);
        }
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

    T fin = T(0);
    if constexpr (WALL) {
        store_lane_guarded<T, K>(out_s + g0, g0, core_lo, core_hi, s, fin);
        if constexpr (COMP) store_lane_guarded<T, K>(out_e + g0, g0, core_lo, core_hi, e, fin);
    } else {
        store_lane_chunks<T, K>(out_s + g0, g0, core_lo, core_hi, s, fin);
        if constexpr (COMP) store_lane_chunks<T, K>(out_e + g0, g0, core_lo, core_hi, e, fin);
    }
    raise_if_nonfinite(a.status, fin);
}

template <typename T, int K, int NW, bool COMP, bool SRC, bool WALL>
__device__ __forceinline__ void run_tile(const TileArgs &a, int tid, int64_t t, int64_t ws)
{
    T s[K], e[K], b[K];
    load_tile<T, K, COMP, SRC, WALL>(a, tid, ws, s, e, b);
    sweep_tile<T, K, NW, COMP, SRC, WALL>(a, tid, t, ws, s, e, b);
}

}  // namespace dev
}  // namespace ge
