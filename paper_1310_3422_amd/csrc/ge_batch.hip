// Persistent batch sweep: thousands of independent rods (each with its own n,
// r and constant walls) advanced by the same number of levels in one launch.
//
// Each workgroup of 16 waves stays resident and pulls tasks from a queue
// (largest first).  A task is a bundle of rods that share a points-per-lane
// choice K; each rod owns a contiguous range of the workgroup's waves and is
// held entirely in registers for all levels, so a rod is read and written
// once per launch.  Per level the waves of a rod exchange their edge values
// through LDS (one workgroup barrier per level) and the per-point update is
// the shared ge_level (ge_level.h), so every rod evolves bit for bit as it
// does through ge_step_n.  The queue counter is reset by a kernel node, and
// the reset and the sweep are captured in a hipGraph that later calls
// replay.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "ge.h"
#include "ge_batch.h"
#include "ge_kernels.h"
#include "ge_level.h"
#include "ge_tile.h"

namespace ge {
namespace {

using namespace dev;

constexpr int kWaves = kBatchWaves;          // waves per workgroup
constexpr int kThreads = kWaves * kWave;

// Wait until a neighbouring wave has published the edges of the level this
// wave is on.  Every wave publishes before it waits, so a wait on level i
// ends once the neighbour has finished level i - 1 (a few microseconds).
// The bound on the polls (BatchArgs::wait_polls, by default 65536, about
// two milliseconds) only keeps a wave from spinning forever should that ever
// fail; a wait that gives up raises kStatusWaitGaveUp, which the next call
// on the plan reports, since the wave then goes on with edge values that
// may be stale.
__device__ __forceinline__ void wait_level(const int *flag, int tag, int polls, int *status)
{
    for (int n = 0;; ++n) {
        if (n >= polls) {
            if (status && (threadIdx.x & (kWave - 1)) == 0) raise_status(status, kStatusWaitGaveUp);
            break;
        }
        if (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) >= tag)
            break;
        __builtin_amdgcn_s_sleep(1);
    }
}

// NBR: the waves of a rod synchronise with their neighbours only (per-wave
// level flags in LDS) instead of the whole workgroup meeting at a barrier
// every level; hasR: the next wave holds the rest of this rod.
template <typename T, int K, bool COMP, bool WALL, bool NBR>
__device__ __forceinline__ void rod_levels(const BatchArgs &a, const BatchRod &rd, int wr,
                                           bool hasR, T (&s)[K], T (&e)[K],
                                           T (*xs)[kWaves][4], T (*xe)[kWaves][4], int *lvl)
{
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    // the wave index is uniform across the wave: let the compiler keep
    // everything derived from it in scalar registers
    const int w = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int64_t n = rd.n;
    const int64_t w0 = (int64_t)wr * kWave * K;       // rod index of this wave's first point
    const int64_t q = n - w0;                         // wave position of the right wall node
    const bool left_wall = (wr == 0);
    const bool ghost_in = (q >= 0) && (q < (int64_t)kWave * K);
    const bool ghost_edge = (q == (int64_t)kWave * K);
    const int kR = ghost_in ? (int)(q % K) : 0;
    const int lR = ghost_in ? (int)(q / K) : -1;
    const int64_t qS = q - 1;
    const bool has_S = (qS >= 0) && (qS < (int64_t)kWave * K);
    const int kS = has_S ? (int)(qS % K) : 0;
    const int lS = has_S ? (int)(qS / K) : -1;
    T gl_hi, gl_lo, gr_hi, gr_lo;
    split_wall<T, COMP>(rd.gl, gl_hi, gl_lo);
    split_wall<T, COMP>(rd.gr, gr_hi, gr_lo);
    const Coef<T> cf = lane_coef(Coef<T>{(T)rd.c1, (T)rd.c2, (T)rd.cs, T(0), T(0), T(0)});
    const T b0[K] = {};
    FluxTap ft{false, 0.0, 0.0, 1.0, 0.0};

    for_levels(a.step0, a.nsteps, [&](auto par, int lev) {
        constexpr int p = decltype(par)::value;
        if (WALL && ghost_in) {
            put_at<T, K>(s, kR, lane == lR, gr_hi);
            if constexpr (COMP) put_at<T, K>(e, kR, lane == lR, gr_lo);
        }
        const int pb = lev & 1;
        if (lane == 0) { xs[pb][w][0] = s[0]; xs[pb][w][1] = s[1]; }
        if (lane == kWave - 1) { xs[pb][w][2] = s[K - 2]; xs[pb][w][3] = s[K - 1]; }
        if constexpr (COMP) {
            if (lane == 0) { xe[pb][w][0] = e[0]; xe[pb][w][1] = e[1]; }
            if (lane == kWave - 1) { xe[pb][w][2] = e[K - 2]; xe[pb][w][3] = e[K - 1]; }
        }
        if constexpr (NBR) {
            // publish this level's edges (the release orders the writes
            // above before the flag), then wait for the neighbours' edges
            const int tag = lev + 1;   // lev counts this call's levels from 0
            if (lane == 0)
                __hip_atomic_store(&lvl[w], tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (wr > 0) wait_level(&lvl[w - 1], tag, a.wait_polls, a.status);
            if (hasR) wait_level(&lvl[w + 1], tag, a.wait_polls, a.status);
        } else {
            __syncthreads();
        }
        const int wl = w > 0 ? w - 1 : 0, wrr = w < kWaves - 1 ? w + 1 : kWaves - 1;
        T xl = xs[pb][wl][3], xr = xs[pb][wrr][0], xl2 = xs[pb][wl][2], xr2 = xs[pb][wrr][1];
        T yl = T(0), yr = T(0), yl2 = T(0), yr2 = T(0);
        if constexpr (COMP) {
            yl = xe[pb][wl][3]; yr = xe[pb][wrr][0]; yl2 = xe[pb][wl][2]; yr2 = xe[pb][wrr][1];
        }
        WallLevel<T> wlv{false, T(0)};
        bool singR = false;
        if constexpr (WALL) {
            if (left_wall) { xl = gl_hi; if constexpr (COMP) yl = gl_lo; }
            if (ghost_edge) { xr = gr_hi; if constexpr (COMP) yr = gr_lo; }
            wlv.isL = left_wall && (p == 1) && (lane == 0);
            singR = has_S && (((n - 1 + p) & 1) == 0);
        }
        Lone<T> lone{T(0), T(0)};
        if (WALL && singR)
            lone = right_lone<T, K, COMP, false>(s, e, b0, kS, xl, yl, gr_hi, gr_lo, T(0), cf,
                                                 T(0));
        ge_level<T, K, COMP, false, WALL, p>(s, e, b0, T(0), T(0), xl, xl2, xr, xr2, yl, yl2,
                                             yr, yr2, cf, T(0), wlv, ft);
        if (WALL && singR) {
            put_at<T, K>(s, kS, lane == lS, lone.s);
            if constexpr (COMP) put_at<T, K>(e, kS, lane == lS, lone.e);
        }
    });
}

// Barrier mode: every wave of the workgroup executes the same number of
// barriers, so waves without a rod in this task run the level loop on dummy
// data.  Neighbour mode: such waves skip the loop.
template <typename T, int K, bool COMP, bool NBR>
__device__ __forceinline__ void run_task(const BatchArgs &a, const BatchTask &tk)
{
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    // the wave index is uniform across the wave: let the compiler keep
    // everything derived from it in scalar registers
    const int w = __builtin_amdgcn_readfirstlane(tid / kWave);
    __shared__ T xs[2][kWaves][4];
    __shared__ T xe[2][kWaves][4];
    __shared__ int lvl[kWaves];
    const int rod = tk.wave_rod[w];
    const int wr = tk.wave_idx[w];
    const bool hasR = rod >= 0 && w + 1 < kWaves && tk.wave_rod[w + 1] == rod;
    if constexpr (NBR) {
        if (lane == 0) lvl[w] = 0;
        __syncthreads();   // every flag reset before any wave publishes
    }
    T s[K], e[K];
    BatchRod rd{};
    T *us = nullptr, *ue = nullptr;
    int64_t g0 = 0;
    if (rod >= 0) {
        rd = a.rods[rod];
        us = static_cast<T *>(a.u) + rd.off;
        ue = static_cast<T *>(a.u) + a.estride + rd.off;
        g0 = ((int64_t)wr * kWave + lane) * K;
        load_lane_guarded<T, K>(us + g0, g0, rd.n, s);
        if constexpr (COMP) load_lane_guarded<T, K>(ue + g0, g0, rd.n, e);
    } else {
        rd.n = (int64_t)kWave * K;
        rd.c1 = rd.c2 = rd.cs = 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j) s[j] = T(0);
    }
    if constexpr (!COMP) {
#pragma unroll
        for (int j = 0; j < K; ++j) e[j] = T(0);
    }
    const int64_t w0 = (int64_t)wr * kWave * K;
    const bool wall = (rod >= 0) && (wr == 0 || rd.n - w0 <= (int64_t)kWave * K);
    if (!NBR || rod >= 0) {
        if (wall)
            rod_levels<T, K, COMP, true, NBR>(a, rd, wr, hasR, s, e, xs, xe, lvl);
        else
            rod_levels<T, K, COMP, false, NBR>(a, rd, wr, hasR, s, e, xs, xe, lvl);
    }
    if (rod >= 0) {
        T fin = T(0);
        store_lane_upto<T, K>(us + g0, g0, rd.n, s, fin);
        if constexpr (COMP) store_lane_upto<T, K>(ue + g0, g0, rd.n, e, fin);
        raise_if_nonfinite(a.status, fin);
    }
    __syncthreads();   // LDS slots are reused by the next task
}

// ---- halo-lane tasks ------------------------------------------------------
// Wave j of a rod holds the window [62 k j, 62 k j + 64 k): its lanes 0 and
// 63 duplicate values of the neighbouring waves (their lanes 62 and 1).  A
// level-(m+1) value depends on level-m values at most two places away, and a
// value that is wrong at an open window edge spreads inward by at most one
// point per level after the first, so after the duplicated lanes are
// refreshed the wave can advance k-1 levels on its own (wave-edge values
// entering as zero) and lanes 1..62 stay exact.  The refresh goes through
// LDS with one workgroup barrier every k-1 levels instead of an exchange
// every level.
//
// Walls stay exact at the rod's ends.  The first wave starts at the left
// wall, which enters as the fill of its lane 0.  The last wave is placed so
// that the right wall node falls at (or within three points of) the end of
// its window, at a fixed element of lane 63: that costs a select or two per
// level, where a wall node at a data-dependent element costs a branch tree
// per access.  It then overlaps its neighbour by more than one lane, and the
// refresh copies values by position: the writer's lanes covering the
// positions store them to LDS, the reader takes k values at the offset.
// When the last window would reach into its neighbour's duplicated lane (a
// 1-in-62 case), or the rod has one wave, the wall node stays where the
// regular placement puts it.
constexpr int kMaxBatchK = 64;
constexpr int kSlot = 2 * kMaxBatchK;    // values per exchange slot (two lanes)

template <typename T, int K, bool COMP, bool WALL>
__device__ __forceinline__ void rod_block(const BatchRod &rd, int wr, int64_t ws, T (&s)[K],
                                          T (&e)[K], int64_t level0, int nlev)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t n = rd.n;
    const int64_t q = n - ws;                         // window position of the right wall node
    const bool left_wall = (wr == 0);
    const bool ghost_in = (q >= 0) && (q < (int64_t)kWave * K);
    const bool ghost_edge = (q == (int64_t)kWave * K);
    const int kR = ghost_in ? (int)(q % K) : 0;
    const int lR = ghost_in ? (int)(q / K) : -1;
    const int64_t qS = q - 1;
    const bool has_S = (qS >= 0) && (qS < (int64_t)kWave * K);
    const int kS = has_S ? (int)(qS % K) : 0;
    const int lS = has_S ? (int)(qS / K) : -1;
    T gl_hi, gl_lo, gr_hi, gr_lo;
    split_wall<T, COMP>(rd.gl, gl_hi, gl_lo);
    split_wall<T, COMP>(rd.gr, gr_hi, gr_lo);
    const Coef<T> cf = lane_coef(Coef<T>{(T)rd.c1, (T)rd.c2, (T)rd.cs, T(0), T(0), T(0)});
    const T b0[K] = {};
    FluxTap ft{false, 0.0, 0.0, 1.0, 0.0};

    for_levels(level0, nlev, [&](auto par, int) {
        constexpr int p = decltype(par)::value;
        if (WALL && ghost_in) {
            put_at<T, K>(s, kR, lane == lR, gr_hi);
            if constexpr (COMP) put_at<T, K>(e, kR, lane == lR, gr_lo);
        }
        // fills at a wall edge are the wall value; at an open edge they
        // only reach the duplicated lane
        T xl = T(0), xr = T(0), yl = T(0), yr = T(0);
        WallLevel<T> wlv{false, T(0)};
        bool singR = false;
        if constexpr (WALL) {
            if (left_wall) { xl = gl_hi; if constexpr (COMP) yl = gl_lo; }
            if (ghost_edge) { xr = gr_hi; if constexpr (COMP) yr = gr_lo; }
            wlv.isL = left_wall && (p == 1) && (lane == 0);
            singR = has_S && (((n - 1 + p) & 1) == 0);
        }
        Lone<T> lone{T(0), T(0)};
        if (WALL && singR)
            lone = right_lone<T, K, COMP, false>(s, e, b0, kS, xl, yl, gr_hi, gr_lo, T(0), cf,
                                                 T(0));
        ge_level<T, K, COMP, false, WALL, p, !WALL>(s, e, b0, T(0), T(0), xl, T(0), xr, T(0), yl,
                                                    T(0), yr, T(0), cf, T(0), wlv, ft);
        if (WALL && singR) {
            put_at<T, K>(s, kS, lane == lS, lone.s);
            if constexpr (COMP) put_at<T, K>(e, kS, lane == lS, lone.e);
        }
    });
}

// The last wave of a rod with its window ending RQ points (0..3) past the
// right wall node: the node is element K - RQ of lane 63 (RQ = 0: just
// beyond the window, the fill of lane 63), the lone point beside it element
// K - 1 - RQ.  Both indices are compile-time constants.  The window start
// is even, so the local pairing is the global one.
template <typename T, int K, bool COMP, int RQ>
__device__ __forceinline__ void rod_block_right(const BatchRod &rd, T (&s)[K], T (&e)[K],
                                                int64_t level0, int nlev)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t n = rd.n;
    T gr_hi, gr_lo;
    split_wall<T, COMP>(rd.gr, gr_hi, gr_lo);
    const Coef<T> cf = lane_coef(Coef<T>{(T)rd.c1, (T)rd.c2, (T)rd.cs, T(0), T(0), T(0)});
    const T b0[K] = {};
    FluxTap ft{false, 0.0, 0.0, 1.0, 0.0};
    const WallLevel<T> wlv{false, T(0)};
    constexpr int kS = K - 1 - RQ;
    const bool lone_odd = ((n - 1) & 1) == 0;   // the lone point exists at even global parity
    for_levels(level0, nlev, [&](auto par, int) {
        constexpr int p = decltype(par)::value;
        if constexpr (RQ > 0) {
            put_at<T, K>(s, K - RQ, lane == kWave - 1, gr_hi);
            if constexpr (COMP) put_at<T, K>(e, K - RQ, lane == kWave - 1, gr_lo);
        }
        const T xr = RQ == 0 ? gr_hi : T(0), yr = (RQ == 0 && COMP) ? gr_lo : T(0);
        const bool singR = lone_odd == (p == 0);
        Lone<T> lone{T(0), T(0)};
        if (singR)
            lone = right_lone<T, K, COMP, false>(s, e, b0, kS, T(0), T(0), gr_hi, gr_lo, T(0), cf,
                                                 T(0));
        ge_level<T, K, COMP, false, false, p, false>(s, e, b0, T(0), T(0), T(0), T(0), xr, T(0),
                                                     T(0), T(0), yr, T(0), cf, T(0), wlv, ft);
        if (singR) {
            put_at<T, K>(s, kS, lane == kWave - 1, lone.s);
            if constexpr (COMP) put_at<T, K>(e, kS, lane == kWave - 1, lone.e);
        }
    });
}

// The first wave of a rod that spans several: the left wall enters as the
// fill of lane 0 and the lone point beside it is element 0 of lane 0; the
// right edge is open.
template <typename T, int K, bool COMP>
__device__ __forceinline__ void rod_block_left(const BatchRod &rd, T (&s)[K], T (&e)[K],
                                               int64_t level0, int nlev)
{
    const int lane = threadIdx.x & (kWave - 1);
    T gl_hi, gl_lo;
    split_wall<T, COMP>(rd.gl, gl_hi, gl_lo);
    const Coef<T> cf = lane_coef(Coef<T>{(T)rd.c1, (T)rd.c2, (T)rd.cs, T(0), T(0), T(0)});
    const T b0[K] = {};
    FluxTap ft{false, 0.0, 0.0, 1.0, 0.0};
    for_levels(level0, nlev, [&](auto par, int) {
        constexpr int p = decltype(par)::value;
        const WallLevel<T> wlv{p == 1 && lane == 0, T(0)};
        ge_level<T, K, COMP, false, true, p, false>(s, e, b0, T(0), T(0), gl_hi, T(0), T(0), T(0),
                                                    COMP ? gl_lo : T(0), T(0), T(0), T(0), cf,
                                                    T(0), wlv, ft);
    });
}

// The levels of a halo-lane task for one wave, in blocks of K-1 levels with
// the duplicated lanes refreshed between blocks.  hx: [2 buffers][waves]
// [2 slots][kSlot] values of s (he: of e, for the pair).  Slot 0 of wave w
// carries the positions its right neighbour duplicates in lane 0, slot 1
// those its left neighbour duplicates in lane 63; a slot holds the two lanes
// that cover them, and the reader starts at the positions' offset within
// the first.  aL / aR: window start of this wave minus the left neighbour's,
// and of the right neighbour minus this wave's.  MODE: 0 = a wave without a
// rod (it only passes the barriers), 1 = both window edges open, 2 = a wave
// holding a wall at its regular place, 3 + RQ = the last wave ending RQ
// points past the right wall node, 7 = the first wave of several.  Every wave of the workgroup passes the
// same barriers (all rods of a task share K and the level count); the mode
// is chosen once per wave, outside the block loop, so each wave runs one
// instantiation of the level code.
template <typename T, int K, bool COMP, int MODE>
__device__ __forceinline__ void halo_blocks(const BatchArgs &a, const BatchRod &rd, int w, int wr,
                                            int64_t ws, int aL, int aR, bool hasL, bool hasR,
                                            T (&s)[K], T (&e)[K], T *hx, T *he)
{
    const int lane = threadIdx.x & (kWave - 1);
    auto slot = [&](int buf, int wave, int which) {
        return ((buf * kWaves + wave) * 2 + which) * kSlot;
    };
    // lanes that write slot 0 (positions [aR, aR + K) of this window) and
    // slot 1 (positions [63K - aL, 64K - aL))
    const int l0 = aR / K, r0 = aR % K;
    const int bL = 63 * K - aL, l1 = bL / K, r1 = bL % K;
    int64_t done = 0;
    for (int blk = 0;; ++blk) {
        const int nb = (int)((a.nsteps - done) < (K - 1) ? (a.nsteps - done) : (K - 1));
        if constexpr (MODE == 1)
            rod_block<T, K, COMP, false>(rd, wr, ws, s, e, a.step0 + done, nb);
        else if constexpr (MODE >= 3 && MODE <= 6)
            rod_block_right<T, K, COMP, MODE - 3>(rd, s, e, a.step0 + done, nb);
        else if constexpr (MODE == 7)
            rod_block_left<T, K, COMP>(rd, s, e, a.step0 + done, nb);
        done += nb;
        if (done >= a.nsteps)
            break;
        const int pb = blk & 1;
        if constexpr (MODE != 0) {
            if (hasR && (lane == l0 || (r0 != 0 && lane == l0 + 1))) {
                const int o = slot(pb, w, 0) + (lane - l0) * K;
#pragma unroll
                for (int j = 0; j < K; ++j) hx[o + j] = s[j];
                if constexpr (COMP) {
#pragma unroll
                    for (int j = 0; j < K; ++j) he[o + j] = e[j];
                }
            }
            if (hasL && (lane == l1 || (r1 != 0 && lane == l1 + 1))) {
                const int o = slot(pb, w, 1) + (lane - l1) * K;
#pragma unroll
                for (int j = 0; j < K; ++j) hx[o + j] = s[j];
                if constexpr (COMP) {
#pragma unroll
                    for (int j = 0; j < K; ++j) he[o + j] = e[j];
                }
            }
        }
        __syncthreads();
        if constexpr (MODE != 0) {
            if ((lane == 0 && hasL) || (lane == kWave - 1 && hasR)) {
                // left: the left neighbour's slot 0 at this window's offset in it;
                // right: the right neighbour's slot 1 at that window's offset
                const int o = lane == 0 ? slot(pb, w - 1, 0) + aL % K
                                        : slot(pb, w + 1, 1) + (63 * K - aR) % K;
#pragma unroll
                for (int j = 0; j < K; ++j) s[j] = hx[o + j];
                if constexpr (COMP) {
#pragma unroll
                    for (int j = 0; j < K; ++j) e[j] = he[o + j];
                }
            }
        }
    }
}

template <typename T, int K, bool COMP>
__device__ __forceinline__ void run_task_halo(const BatchArgs &a, const BatchTask &tk, T *hx,
                                              T *he)
{
    static_assert(K >= 4 && K <= kMaxBatchK, "points per lane");
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int rod = tk.wave_rod[w];
    const int wr = tk.wave_idx[w];
    const bool hasR = rod >= 0 && w + 1 < kWaves && tk.wave_rod[w + 1] == rod;
    const bool hasL = rod >= 0 && wr > 0;
    T s[K], e[K];
    BatchRod rd{};
    T *us = nullptr, *ue = nullptr;
    int64_t ws = 0, lo = 0;
    int aL = 62 * K, aR = 62 * K, mode = 0;
    if (rod >= 0) {
        rd = a.rods[rod];
        const HaloLayout L(rd.n, K);
        ws = L.start(wr);                           // a multiple of 4
        if (hasL) aL = (int)(ws - L.start(wr - 1));
        if (hasR) aR = (int)(L.start(wr + 1) - ws);
        // the last wave stores only beyond its neighbour's core
        lo = (wr == L.m - 1 && wr > 0) ? L.start(wr - 1) + 63 * K : 0;
        // the planner gives halo tasks only rods of two or more waves whose
        // last window ends at the wall
        if (!hasR)
            mode = 3 + (int)(ws + 64 * K - rd.n);   // RQ in 0..3
        else
            mode = wr == 0 ? 7 : 1;
        us = static_cast<T *>(a.u) + rd.off;
        ue = static_cast<T *>(a.u) + a.estride + rd.off;
    }
    const int64_t g0 = ws + (int64_t)lane * K;
    if (rod >= 0) {
        load_lane_guarded<T, K>(us + g0, g0, rd.n, s);
        if constexpr (COMP) load_lane_guarded<T, K>(ue + g0, g0, rd.n, e);
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) s[j] = T(0);
    }
    if constexpr (!COMP) {
#pragma unroll
        for (int j = 0; j < K; ++j) e[j] = T(0);
    }
    switch (__builtin_amdgcn_readfirstlane(mode)) {
    case 1: halo_blocks<T, K, COMP, 1>(a, rd, w, wr, ws, aL, aR, hasL, hasR, s, e, hx, he); break;
    case 3: halo_blocks<T, K, COMP, 3>(a, rd, w, wr, ws, aL, aR, hasL, hasR, s, e, hx, he); break;
    case 4: halo_blocks<T, K, COMP, 4>(a, rd, w, wr, ws, aL, aR, hasL, hasR, s, e, hx, he); break;
    case 5: halo_blocks<T, K, COMP, 5>(a, rd, w, wr, ws, aL, aR, hasL, hasR, s, e, hx, he); break;
    case 6: halo_blocks<T, K, COMP, 6>(a, rd, w, wr, ws, aL, aR, hasL, hasR, s, e, hx, he); break;
    case 7: halo_blocks<T, K, COMP, 7>(a, rd, w, wr, ws, aL, aR, hasL, hasR, s, e, hx, he); break;
    default: halo_blocks<T, K, COMP, 0>(a, rd, w, wr, ws, aL, aR, hasL, hasR, s, e, hx, he); break;
    }
    // lanes 1..62, lane 0 of the first wave and lane 63 of the last (the last
    // wave from its neighbour's core end on)
    T fin = T(0);
    if (rod >= 0 && (lane > 0 || wr == 0) && (lane < kWave - 1 || !hasR)) {
        store_lane_range<T, K>(us + g0, g0, lo, rd.n, s, fin);
        if constexpr (COMP) store_lane_range<T, K>(ue + g0, g0, lo, rd.n, e, fin);
    }
    if (rod >= 0) raise_if_nonfinite(a.status, fin);
    __syncthreads();   // LDS slots are reused by the next task
}

// ---- long-rod tasks ------------------------------------------------------
// A rod longer than the workgroup's registers hold is swept the way a single
// rod is (ge_tile.h): windows of 64 K points, one per wave, advance up to
// long_depth levels in registers with open edges and store their cores, the
// halo of long_halo >= levels + 1 points per side absorbing what enters from
// the open edges.  The 16 waves take the windows of a pass round-robin, and a
// workgroup barrier separates the passes; no other workgroup touches the
// rod, so no wait crosses workgroups.  The passes ping-pong between u and the
// rod's own second level buffer in u2 and their number is even, so the
// result lands in u.  Every point gets the same operations as in every other
// path, so the bits equal those of ge_step_n.
template <typename T, int K, bool COMP>
__device__ __forceinline__ void run_task_long(const BatchArgs &a, const BatchTask &tk)
{
    constexpr int64_t W = (int64_t)kWave * K;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const BatchRod rd = a.rods[tk.wave_rod[0]];
    TileArgs ta{};
    ta.n = rd.n;
    ta.halo = a.long_halo;
    ta.core = W - 2 * (int64_t)a.long_halo;
    ta.ntiles = (rd.n + ta.core - 1) / ta.core;
    ta.c1 = rd.c1;
    ta.c2 = rd.c2;
    ta.cs = rd.cs;
    ta.gl0 = rd.gl;
    ta.gr0 = rd.gr;
    ta.h = 1.0;
    ta.status = a.status;
    T *b0 = static_cast<T *>(a.u) + rd.off;
    T *b1 = static_cast<T *>(a.u2) + rd.woff;
    int64_t passes = (a.nsteps + a.long_depth - 1) / a.long_depth;
    passes += passes & 1;
    const int64_t base = a.nsteps / passes, extra = a.nsteps % passes;
    int64_t done = 0;
    for (int64_t ps = 0; ps < passes; ++ps) {
        const int lev = (int)(base + (ps < extra ? 1 : 0));
        ta.in = (ps & 1) ? b1 : b0;
        ta.out = (ps & 1) ? b0 : b1;
        ta.estride = (ps & 1) ? a.estride2 : a.estride;
        ta.estride_out = (ps & 1) ? a.estride : a.estride2;
        ta.level0 = a.step0 + done;
        ta.nlev = lev;
        for (int64_t t = w; t < ta.ntiles; t += kWaves) {
            const int64_t ws = t == 0 ? 0 : t * ta.core - ta.halo;
            if (ws == 0 || ws + W >= rd.n)
                run_tile<T, K, 1, COMP, false, true>(ta, lane, t, ws);
            else
                run_tile<T, K, 1, COMP, false, false>(ta, lane, t, ws);
        }
        // the next pass reads what every wave stored (same workgroup: the
        // barrier orders the global stores before the loads)
        __syncthreads();
        done += lev;
    }
}

// SYNC: 1 = barrier per level, 2 = neighbour flags, 3 = halo lanes (tasks
// the planner could not give halo lanes use neighbour flags).
template <typename T, bool COMP, int SYNC>
__global__ __launch_bounds__(kThreads) void batch_kernel(BatchArgs a)
{
    constexpr bool NBR = SYNC != 1;
    __shared__ int task_s;
    __shared__ T hx[SYNC == 3 ? 2 * kWaves * 2 * kSlot : 1];
    __shared__ T he[SYNC == 3 && COMP ? 2 * kWaves * 2 * kSlot : 1];
    for (;;) {
        if (threadIdx.x == 0)
            task_s = atomicAdd(a.counter, 1);
        __syncthreads();
        const int task = task_s;
        __syncthreads();
        if (task >= a.ntasks)
            break;
        const BatchTask &tk = a.tasks[task];
        if (tk.halo == 2) {
            run_task_long<T, batch_long_k(sizeof(T) == 8 ? kFP64 : (COMP ? kFP32C : kFP32)), COMP>(
                a, tk);
            continue;
        }
        if (SYNC == 3 && tk.halo) {
            switch (tk.k) {
            case 4: run_task_halo<T, 4, COMP>(a, tk, hx, he); break;
            case 8: run_task_halo<T, 8, COMP>(a, tk, hx, he); break;
            case 16: run_task_halo<T, 16, COMP>(a, tk, hx, he); break;
            case 32: run_task_halo<T, 32, COMP>(a, tk, hx, he); break;
            case 64:
                if constexpr (sizeof(T) == 4 && !COMP) run_task_halo<T, 64, COMP>(a, tk, hx, he);
                break;
            default: break;
            }
            continue;
        }
        switch (tk.k) {
        case 4: run_task<T, 4, COMP, NBR>(a, tk); break;
        case 8: run_task<T, 8, COMP, NBR>(a, tk); break;
        case 16: run_task<T, 16, COMP, NBR>(a, tk); break;
        case 32: run_task<T, 32, COMP, NBR>(a, tk); break;
        case 64:
            if constexpr (sizeof(T) == 4 && !COMP) run_task<T, 64, COMP, NBR>(a, tk);
            break;
        default: break;
        }
    }
}

__global__ void reset_counter_kernel(int *counter) { *counter = 0; }

// The allocation-free entry point's scratch (see batch_scratch).  Host code
// never passes this name to a kernel: it is a host-side stand-in, and the
// device address comes from hipGetSymbolAddress, per device.
__device__ __align__(256) unsigned char scratch[kBatchScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices];

}  // namespace

void *batch_scratch(hipError_t *err)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && (dev < 0 || dev >= kMaxDevices)) e = hipErrorInvalidDevice;
    if (e != hipSuccess) {
        *err = e;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        g_scratch_addr[dev] = p;
    }
    *err = hipSuccess;
    return g_scratch_addr[dev];
}

hipError_t launch_batch(int prec, const BatchArgs &a, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, a.counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define GE_BK(T, C)                                                                          \
    if (a.sync == 3)                                                                          \
        hipLaunchKernelGGL((batch_kernel<T, C, 3>), dim3(grid), dim3(kThreads), 0, stream, a);   \
    else if (a.sync == 2)                                                                     \
        hipLaunchKernelGGL((batch_kernel<T, C, 2>), dim3(grid), dim3(kThreads), 0, stream, a);   \
    else                                                                                      \
        hipLaunchKernelGGL((batch_kernel<T, C, 1>), dim3(grid), dim3(kThreads), 0, stream, a);
    switch (prec) {
    case kFP64:
        GE_BK(double, false)
        break;
    case kFP32:
        GE_BK(float, false)
        break;
    case kFP32C:
        GE_BK(float, true)
        break;
#undef GE_BK
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int batch_max_k(int prec) { return prec == kFP32 ? 64 : 32; }

}  // namespace ge
