// Tiled, temporally blocked GE sweep for gfx950.
//
// Scheme (Section 2, two-point groups): at level m with p = m mod 2 the
// points are coupled as (0,1),(2,3),... (0-based) when p = 0 and
// (1,2),(3,4),... when p = 1.  A coupled pair solved by the confluence
// formulas Eq. (3)/(4) is written here in the equivalent second-difference
// form: with D_i = u_{i-1} - 2u_i + u_{i+1},
//     u_i' = u_i + c1 D_i + c2 D_q,   c1 = (r+r^2)/(1+2r), c2 = r^2/(1+2r),
// where q is i's partner.  A point alone beside a wall (point 0 when p = 1,
// point n-1 when n-1+p is even) takes scheme A, Eq. (1), or scheme B,
// Eq. (2), in the same form: u_i' = u_i + cs (D_i + g(t_{m+1}) - g(t_m)),
// cs = r/(1+r), where D_i used the wall value at t_m.  A source f = a(t) b(x)
// adds a(t_m + tau/2) (e1 b_i + e2 b_q) to a pair member and
// a(t_m + tau/2) es b_i to a lone point.
//
// D_i is formed from first differences d_i = u_{i+1} - u_i as
// D_i = d_i - d_{i-1}; for smooth data the differences are exact, so the
// increment carries a relative (not absolute) rounding error.  FP64 then
// applies u' = fma(c2, D_q, fma(c1, D_i, u)); FP32 forms the increment
// first and rounds u once per level.  The compensated FP32 pair (s, e),
// value s + e, takes D from the s and e second differences summed at the
// end, and adds the increment with Kahan's compensated sum.
//
// Mapping: one workgroup of NW waves owns a window of W = NW*64*K points;
// lane l of wave w holds points (64w + l)K .. (64w + l)K + K-1 of the window
// in registers.  Neighbour values cross lanes by DPP wave shifts and waves by
// LDS (one barrier per level).  A value at level m+1 depends on level-m
// values at most two places away, and after the first level the invalid
// region entering from an open window edge grows by one point per level, so
// a halo of H >= nlev + 1 points each side leaves the core exact; halos are
// recomputed by the neighbouring tiles instead of being exchanged.
//
// Determinism: every point of every tile, halo or core, wall tile or not, is
// advanced by the same expression sequence with explicit fma() and no
// contraction (-ffp-contract=off), so results do not depend on the tiling,
// the levels per launch or the grid.
#include "ge_kernels.h"

namespace ge {
namespace {

constexpr int kWave = 64;

// ---- cross-lane moves ------------------------------------------------------
// DPP wave shifts by one lane; the lane with no source (lane 0 for a shift
// right, lane 63 for a shift left) receives `fill`.
__device__ __forceinline__ int shr1_i(int fill, int v)
{
    return __builtin_amdgcn_update_dpp(fill, v, 0x138, 0xF, 0xF, false);  // wave_shr:1
}
__device__ __forceinline__ int shl1_i(int fill, int v)
{
    return __builtin_amdgcn_update_dpp(fill, v, 0x130, 0xF, 0xF, false);  // wave_shl:1
}
// value held by lane l-1 (lane 0: fill)
__device__ __forceinline__ float from_left(float fill, float v)
{
    return __int_as_float(shr1_i(__float_as_int(fill), __float_as_int(v)));
}
// value held by lane l+1 (lane 63: fill)
__device__ __forceinline__ float from_right(float fill, float v)
{
    return __int_as_float(shl1_i(__float_as_int(fill), __float_as_int(v)));
}
__device__ __forceinline__ double from_left(double fill, double v)
{
    const long long b = __double_as_longlong(v), f = __double_as_longlong(fill);
    const int lo = shr1_i((int)(f & 0xffffffffll), (int)(b & 0xffffffffll));
    const int hi = shr1_i((int)(f >> 32), (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double from_right(double fill, double v)
{
    const long long b = __double_as_longlong(v), f = __double_as_longlong(fill);
    const int lo = shl1_i((int)(f & 0xffffffffll), (int)(b & 0xffffffffll));
    const int hi = shl1_i((int)(f >> 32), (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---- 16-byte vector access to a lane's K contiguous values ----------------
template <typename T> struct V16;
template <> struct V16<float> { using type = float4; static constexpr int E = 4; };
template <> struct V16<double> { using type = double2; static constexpr int E = 2; };

template <typename T, int K>
__device__ __forceinline__ void load_lane(const T *__restrict__ p, T (&v)[K])
{
    using V = typename V16<T>::type;
    constexpr int E = V16<T>::E;
    static_assert(K % E == 0, "K must fill whole 16-byte chunks");
    const V *q = reinterpret_cast<const V *>(p);
#pragma unroll
    for (int c = 0; c < K / E; ++c) {
        const V x = q[c];
        if constexpr (E == 4) {
            v[4 * c] = x.x; v[4 * c + 1] = x.y; v[4 * c + 2] = x.z; v[4 * c + 3] = x.w;
        } else {
            v[2 * c] = x.x; v[2 * c + 1] = x.y;
        }
    }
}

template <typename T, int K>
__device__ __forceinline__ void load_lane_guarded(const T *__restrict__ p, int64_t g0,
                                                  int64_t n, T (&v)[K])
{
    using V = typename V16<T>::type;
    constexpr int E = V16<T>::E;
    const V *q = reinterpret_cast<const V *>(p);
#pragma unroll
    for (int c = 0; c < K / E; ++c) {
        if (g0 + (c + 1) * E <= n) {
            const V x = q[c];
            if constexpr (E == 4) {
                v[4 * c] = x.x; v[4 * c + 1] = x.y; v[4 * c + 2] = x.z; v[4 * c + 3] = x.w;
            } else {
                v[2 * c] = x.x; v[2 * c + 1] = x.y;
            }
        } else {
#pragma unroll
            for (int i = 0; i < E; ++i)
                v[c * E + i] = (g0 + c * E + i < n) ? p[c * E + i] : T(0);
        }
    }
}

// Store the values whose global index lies in [lo, hi).  lo and hi are
// multiples of the chunk width on the fast path.
template <typename T, int K>
__device__ __forceinline__ void store_lane_chunks(T *__restrict__ p, int64_t g0, int64_t lo,
                                                  int64_t hi, const T (&v)[K])
{
    using V = typename V16<T>::type;
    constexpr int E = V16<T>::E;
    V *q = reinterpret_cast<V *>(p);
#pragma unroll
    for (int c = 0; c < K / E; ++c) {
        const int64_t g = g0 + c * E;
        if (g >= lo && g < hi) {
            V x;
            if constexpr (E == 4) {
                x.x = v[4 * c]; x.y = v[4 * c + 1]; x.z = v[4 * c + 2]; x.w = v[4 * c + 3];
            } else {
                x.x = v[2 * c]; x.y = v[2 * c + 1];
            }
            q[c] = x;
        }
    }
}

template <typename T, int K>
__device__ __forceinline__ void store_lane_guarded(T *__restrict__ p, int64_t g0, int64_t lo,
                                                   int64_t hi, const T (&v)[K])
{
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (g0 + j >= lo && g0 + j < hi)
            p[j] = v[j];
}

// v[k] = x in the lanes where `pred` holds; k is uniform across the wave.
template <typename T, int K>
__device__ __forceinline__ void put_at(T (&v)[K], int k, bool pred, T x)
{
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (j == k)
            v[j] = pred ? x : v[j];
}

// A first difference: one value, or the (s, e) parts of the pair kept apart.
template <typename T, bool COMP> struct Dif { T s; };
template <typename T> struct Dif<T, true> { T s, e; };

// Wall value split for the state type: (hi, lo) with hi + lo ~ g.
template <typename T, bool COMP>
__device__ __forceinline__ void split_wall(double g, T &hi, T &lo)
{
    hi = (T)g;
    lo = COMP ? (T)(g - (double)hi) : T(0);
}

template <typename T, int K, int NW, bool COMP, bool SRC, bool WALL>
__device__ __forceinline__ void run_tile(const TileArgs &a, int64_t t, int64_t ws)
{
    constexpr int W = NW * kWave * K;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const int64_t n = a.n;
    const int64_t core_lo = t * a.core;
    const int64_t core_hi = min(core_lo + a.core, n);
    const int64_t g0 = ws + (int64_t)tid * K;       // global index of my first point

    const T *in_s = static_cast<const T *>(a.in);
    T *out_s = static_cast<T *>(a.out);
    const T *in_e = in_s + a.estride;
    T *out_e = out_s + a.estride;
    const T *srcb = static_cast<const T *>(a.src_b);

    T s[K], e[K], b[K];
    if constexpr (WALL) {
        load_lane_guarded<T, K>(in_s + g0, g0, n, s);
        if constexpr (COMP) load_lane_guarded<T, K>(in_e + g0, g0, n, e);
        if constexpr (SRC) load_lane_guarded<T, K>(srcb + g0, g0, n, b);
    } else {
        load_lane<T, K>(in_s + g0, s);
        if constexpr (COMP) load_lane<T, K>(in_e + g0, e);
        if constexpr (SRC) load_lane<T, K>(srcb + g0, b);
    }
    if constexpr (!COMP) {
#pragma unroll
        for (int j = 0; j < K; ++j) e[j] = T(0);
    }

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

    const T c1 = (T)a.c1, c2 = (T)a.c2, cs = (T)a.cs;
    const T e1 = (T)a.e1, e2 = (T)a.e2, es = (T)a.es;

    for (int lev = 0; lev < a.nlev; ++lev) {
        const int p = (int)((a.level0 + lev) & 1);
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
        T dgl = T(0), dgr = T(0);
        bool isL = false, isS = false;
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
            dgl = (T)(gln - glo);
            dgr = (T)(grn - gro);
            isL = left_wall && (p == 1) && (tid == 0);
            isS = has_S && (((n - 1 + p) & 1) == 0) && (tid == lS);
        }
        // u_{-1} and u_K: neighbour lanes' edge points
        const T sl = from_left(xl, s[K - 1]), sr = from_right(xr, s[0]);
        T el = T(0), er = T(0);
        if constexpr (COMP) { el = from_left(yl, e[K - 1]); er = from_right(yr, e[0]); }
        const T an = SRC ? (T)a.src_a[lev] : T(0);

        // First difference u_{j+1} - u_j of two points given as (s, e).  For
        // the pair the s and e parts stay apart: for smooth data the s
        // differences (and their differences) are exact, and summing the s
        // and e second differences only at the end keeps D accurate to the
        // precision of the pair.
        auto dif = [&](T s1, T e1_, T s0, T e0) -> Dif<T, COMP> {
            if constexpr (COMP) return Dif<T, COMP>{s1 - s0, e1_ - e0};
            else return Dif<T, COMP>{s1 - s0};
        };
        // second difference D = db - da from consecutive first differences
        auto sd = [&](Dif<T, COMP> da, Dif<T, COMP> db) -> T {
            if constexpr (COMP) return (db.s - da.s) + (db.e - da.e);
            else return db.s - da.s;
        };
        // advance point j from D_self and D_partner (bp: partner's profile)
        auto upd = [&](int j, T Ds, T Dp, T bp) {
            if constexpr (COMP) {
                T inc = fmaT(c1, Ds, c2 * Dp);
                if constexpr (SRC) inc = fmaT(an, fmaT(e1, b[j], e2 * bp), inc);
                if constexpr (WALL) {
                    if (j == kS) {
                        T alt = cs * (Ds + dgr);
                        if constexpr (SRC) alt = fmaT(an, es * b[j], alt);
                        inc = isS ? alt : inc;
                    }
                    if (j == 0) {
                        T alt = cs * (Ds + dgl);
                        if constexpr (SRC) alt = fmaT(an, es * b[j], alt);
                        inc = isL ? alt : inc;
                    }
                }
                // Kahan: the pair absorbs the increment, e keeps what s lost
                const T y = inc + e[j];
                const T tt = s[j] + y;
                e[j] = y - (tt - s[j]);
                s[j] = tt;
            } else if constexpr (sizeof(T) == 8) {
                // FP64: two fused steps, u + c1 D_self, then + c2 D_partner
                T t = fmaT(c1, Ds, s[j]);
                if constexpr (SRC) t = fmaT(an, fmaT(e1, b[j], e2 * bp), t);
                T v = fmaT(c2, Dp, t);
                if constexpr (WALL) {
                    if (j == kS) {
                        T alt = fmaT(cs, Ds + dgr, s[j]);
                        if constexpr (SRC) alt = fmaT(an, es * b[j], alt);
                        v = isS ? alt : v;
                    }
                    if (j == 0) {
                        T alt = fmaT(cs, Ds + dgl, s[j]);
                        if constexpr (SRC) alt = fmaT(an, es * b[j], alt);
                        v = isL ? alt : v;
                    }
                }
                s[j] = v;
            } else {
                // FP32: form the increment first, so u is rounded once per level
                T inc = fmaT(c1, Ds, c2 * Dp);
                if constexpr (SRC) inc = fmaT(an, fmaT(e1, b[j], e2 * bp), inc);
                if constexpr (WALL) {
                    if (j == kS) {
                        T alt = cs * (Ds + dgr);
                        if constexpr (SRC) alt = fmaT(an, es * b[j], alt);
                        inc = isS ? alt : inc;
                    }
                    if (j == 0) {
                        T alt = cs * (Ds + dgl);
                        if constexpr (SRC) alt = fmaT(an, es * b[j], alt);
                        inc = isL ? alt : inc;
                    }
                }
                s[j] = s[j] + inc;
            }
            if constexpr (WALL) {
                // wall first differences at the new level, accumulated in FP64
                if (own_L && j == 0 && tid == 0) {
                    const double v = (double)s[j] + (COMP ? (double)e[j] : 0.0);
                    accL = accL + a.tau * (v - gln) / a.h;
                }
                if (own_R && j == kS && tid == lS) {
                    const double v = (double)s[j] + (COMP ? (double)e[j] : 0.0);
                    accR = accR + a.tau * (v - grn) / a.h;
                }
            }
        };

        if (p == 0) {
            // pairs (2q, 2q+1) inside the lane
            auto dprev = dif(s[0], e[0], sl, el);                    // d_{-1}
#pragma unroll
            for (int q = 0; q < K / 2; ++q) {
                const int j = 2 * q;
                const auto d0 = dif(s[j + 1], e[j + 1], s[j], e[j]); // d_j
                const auto d1 = (j + 2 < K) ? dif(s[j + 2], e[j + 2], s[j + 1], e[j + 1])
                                            : dif(sr, er, s[j + 1], e[j + 1]);
                const T Da = sd(dprev, d0), Db = sd(d0, d1);
                upd(j, Da, Db, b[j + 1]);
                upd(j + 1, Db, Da, b[j]);
                dprev = d1;
            }
        } else {
            // pairs (-1,0), (1,2), ..., (K-1,K): the lane's edge points pair
            // with the neighbouring lanes' edge points, so u_{-2} and u_{K+1}
            // are needed too
            const T sl2 = from_left(xl2, s[K - 2]), sr2 = from_right(xr2, s[1]);
            T el2 = T(0), er2 = T(0);
            if constexpr (COMP) { el2 = from_left(yl2, e[K - 2]); er2 = from_right(yr2, e[1]); }
            const auto dm2 = dif(sl, el, sl2, el2);                   // d_{-2}
            const auto dm1 = dif(s[0], e[0], sl, el);                 // d_{-1}
            const auto d0 = dif(s[1], e[1], s[0], e[0]);              // d_0
            const auto dK1 = dif(sr, er, s[K - 1], e[K - 1]);         // d_{K-1}
            const auto dK = dif(sr2, er2, sr, er);                    // d_K
            const auto dK2 = dif(s[K - 1], e[K - 1], s[K - 2], e[K - 2]);  // d_{K-2}
            upd(0, sd(dm1, d0), sd(dm2, dm1), bl);
            auto dprev = d0;
#pragma unroll
            for (int q = 1; q < K / 2; ++q) {
                const int j = 2 * q - 1;
                const auto da = dif(s[j + 1], e[j + 1], s[j], e[j]); // d_j
                const auto db = dif(s[j + 2], e[j + 2], s[j + 1], e[j + 1]);  // d_{j+1}
                const T Da = sd(dprev, da), Db = sd(da, db);
                upd(j, Da, Db, b[j + 1]);
                upd(j + 1, Db, Da, b[j]);
                dprev = db;
            }
            upd(K - 1, sd(dK2, dK1), sd(dK1, dK), br);
        }
    }

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

bool tile_config_supported(int prec, int k, int nw)
{
    if (nw != 1 && nw != 4)
        return false;
    switch (prec) {
    case kFP64: return k == 2 || k == 4 || k == 8 || k == 16;
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
