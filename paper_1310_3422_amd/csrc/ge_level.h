// One level of the GE sweep on a register tile, shared by the single-rod
// tile kernel (ge_sweep_kernels.h) and the persistent batch kernel (ge_batch.hip).
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
// Layout: each lane holds K consecutive points in registers; neighbour
// values cross lanes by DPP wave shifts, and the lanes at a wave's edges
// receive theirs as the DPP fill value.
//
// Determinism: every point, in every kernel and tile, halo or core, is
// advanced by the same expression sequence with explicit fma() and no
// contraction (-ffp-contract=off), so results do not depend on the tiling,
// the levels per launch, the grid, or whether a rod runs alone or in a batch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ge_kernels.h"

namespace ge {
namespace dev {

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

// The same shifts where the lane without a source may receive any value (a
// wave whose edges are open window edges: those points lie in the halo).
// bound_ctrl makes that lane read zero, so no fill operand has to be set up.
__device__ __forceinline__ int shr1z_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ int shl1z_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ float from_left_open(float v)
{
    return __int_as_float(shr1z_i(__float_as_int(v)));
}
__device__ __forceinline__ float from_right_open(float v)
{
    return __int_as_float(shl1z_i(__float_as_int(v)));
}
__device__ __forceinline__ double from_left_open(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = shr1z_i((int)(b & 0xffffffffll)), hi = shr1z_i((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double from_right_open(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = shl1z_i((int)(b & 0xffffffffll)), hi = shl1z_i((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// edge value from the left / right neighbour lane, with the fill used only
// when the wave's edge is not open
template <bool OPEN, typename T>
__device__ __forceinline__ T edge_left(T fill, T v)
{
    if constexpr (OPEN) return from_left_open(v);
    else return from_left(fill, v);
}
template <bool OPEN, typename T>
__device__ __forceinline__ T edge_right(T fill, T v)
{
    if constexpr (OPEN) return from_right_open(v);
    else return from_right(fill, v);
}

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Raise a status word (StatusWord, ge_kernels.h): host-mapped memory of the
// plan, written with a plain system-scope store, so no read-modify-write
// crosses the bus.
__device__ __forceinline__ void raise_status(int *status, int word)
{
    __hip_atomic_store(status + word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The stored values are tested as they are stored: acc + v * 0 over them
// stays 0 while they are finite and becomes NaN once one is NaN or infinite
// (one FMA per value, no compare).  Values a lane holds but does not store
// (halo points, points past a wall) are not tested: past a wall they are
// not part of the problem and may grow without bound.
template <typename T>
__device__ __forceinline__ void finite_acc(T &acc, T v)
{
    acc = fmaT(v, T(0), acc);
}

// Raise kStatusNonfinite if some lane's stored values were not all finite;
// at most one store per wave.  Called by every lane of the wave.
template <typename T>
__device__ __forceinline__ void raise_if_nonfinite(int *status, T acc)
{
    if (!status) return;
    const uint64_t m = __ballot(!__builtin_isfinite(acc));
    if (m != 0 && (threadIdx.x & (kWave - 1)) == (unsigned)__builtin_ctzll(m))
        raise_status(status, kStatusNonfinite);
}

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
                                                  int64_t hi, const T (&v)[K], T &fin)
{
    using V = typename V16<T>::type;
    constexpr int E = V16<T>::E;
    V *q = reinterpret_cast<V *>(p);
#pragma unroll
    for (int c = 0; c < K / E; ++c) {
        const int64_t g = g0 + c * E;
        if (g >= lo && g < hi) {
#pragma unroll
            for (int i = 0; i < E; ++i) finite_acc(fin, v[c * E + i]);
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
                                                   int64_t hi, const T (&v)[K], T &fin)
{
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (g0 + j >= lo && g0 + j < hi) {
            finite_acc(fin, v[j]);
            p[j] = v[j];
        }
}

// Store the values whose global index is below n: whole 16-byte chunks
// where they lie below n, single values in the chunk that straddles n.
template <typename T, int K>
__device__ __forceinline__ void store_lane_upto(T *__restrict__ p, int64_t g0, int64_t n,
                                                const T (&v)[K], T &fin)
{
    using V = typename V16<T>::type;
    constexpr int E = V16<T>::E;
    V *q = reinterpret_cast<V *>(p);
#pragma unroll
    for (int c = 0; c < K / E; ++c) {
        if (g0 + (c + 1) * E <= n) {
#pragma unroll
            for (int i = 0; i < E; ++i) finite_acc(fin, v[c * E + i]);
            V x;
            if constexpr (E == 4) {
                x.x = v[4 * c]; x.y = v[4 * c + 1]; x.z = v[4 * c + 2]; x.w = v[4 * c + 3];
            } else {
                x.x = v[2 * c]; x.y = v[2 * c + 1];
            }
            q[c] = x;
        } else {
#pragma unroll
            for (int i = 0; i < E; ++i)
                if (g0 + c * E + i < n) {
                    finite_acc(fin, v[c * E + i]);
                    p[c * E + i] = v[c * E + i];
                }
        }
    }
}

// Store the values whose global index lies in [lo, n): lo is a multiple of
// the chunk width, so a chunk is wholly below lo or not; the chunk that
// straddles n goes value by value.
template <typename T, int K>
__device__ __forceinline__ void store_lane_range(T *__restrict__ p, int64_t g0, int64_t lo,
                                                 int64_t n, const T (&v)[K], T &fin)
{
    using V = typename V16<T>::type;
    constexpr int E = V16<T>::E;
    V *q = reinterpret_cast<V *>(p);
#pragma unroll
    for (int c = 0; c < K / E; ++c) {
        if (g0 + c * E < lo)
            continue;
        if (g0 + (c + 1) * E <= n) {
#pragma unroll
            for (int i = 0; i < E; ++i) finite_acc(fin, v[c * E + i]);
            V x;
            if constexpr (E == 4) {
                x.x = v[4 * c]; x.y = v[4 * c + 1]; x.z = v[4 * c + 2]; x.w = v[4 * c + 3];
            } else {
                x.x = v[2 * c]; x.y = v[2 * c + 1];
            }
            q[c] = x;
        } else {
#pragma unroll
            for (int i = 0; i < E; ++i)
                if (g0 + c * E + i < n) {
                    finite_acc(fin, v[c * E + i]);
                    p[c * E + i] = v[c * E + i];
                }
        }
    }
}

// Access to element k of a lane's register tile for a wave-uniform k, as a
// switch: one scalar branch tree and a single move per call.  (An equality
// chain over the tile would be folded into one dynamically indexed access,
// which for tiles above 32 registers goes through scratch memory.)
#define GE_CASES8(b) GE_C(b + 0) GE_C(b + 1) GE_C(b + 2) GE_C(b + 3) \
    GE_C(b + 4) GE_C(b + 5) GE_C(b + 6) GE_C(b + 7)
#define GE_CASES64 GE_CASES8(0) GE_CASES8(8) GE_CASES8(16) GE_CASES8(24) \
    GE_CASES8(32) GE_CASES8(40) GE_CASES8(48) GE_CASES8(56)

// v[k] = x in the lanes where `pred` holds (k outside [0, K): no change).
template <typename T, int K>
__device__ __forceinline__ void put_at(T (&v)[K], int k, bool pred, T x)
{
    static_assert(K <= 64, "tiles are at most 64 values per lane");
    switch (k) {
#define GE_C(i) \
    case i: \
        if constexpr ((i) < K) v[i] = pred ? x : v[i]; \
        break;
        GE_CASES64
#undef GE_C
    default: break;
    }
}

// v[k] (k outside [0, K): `otherwise`).
template <typename T, int K>
__device__ __forceinline__ T get_at(const T (&v)[K], int k, T otherwise)
{
    T r = otherwise;
    switch (k) {
#define GE_C(i) \
    case i: \
        if constexpr ((i) < K) r = v[i]; \
        break;
        GE_CASES64
#undef GE_C
    default: break;
    }
    return r;
}


// A first difference: one value, or the (s, e) parts of the pair kept apart.
template <typename T, bool COMP> struct Dif { T s; };
template <typename T> struct Dif<T, true> { T s, e; };

// First difference u_{j+1} - u_j of two points given as (s, e).  For the
// pair the s and e parts stay apart: for smooth data the s differences (and
// their differences) are exact, and summing the s and e second differences
// only at the end keeps D accurate to the precision of the pair.
template <typename T, bool COMP>
__device__ __forceinline__ Dif<T, COMP> dif(T s1, T e1, T s0, T e0)
{
    if constexpr (COMP) return Dif<T, COMP>{s1 - s0, e1 - e0};
    else return Dif<T, COMP>{s1 - s0};
}

// second difference D = db - da from consecutive first differences
template <typename T, bool COMP>
__device__ __forceinline__ T sd(Dif<T, COMP> da, Dif<T, COMP> db)
{
    if constexpr (COMP) return (db.s - da.s) + (db.e - da.e);
    else return db.s - da.s;
}

// Wall value split for the state type: (hi, lo) with hi + lo ~ g.
template <typename T, bool COMP>
__device__ __forceinline__ void split_wall(double g, T &hi, T &lo)
{
    hi = (T)g;
    lo = COMP ? (T)(g - (double)hi) : T(0);
}


// Per-level constants of the scheme in the state's type.
template <typename T> struct Coef {
    T c1, c2, cs;   // (r+r^2)/(1+2r), r^2/(1+2r), r/(1+r)
    T e1, e2, es;   // tau(1+r)/(1+2r), tau r/(1+2r), tau/(1+r)
};

// The coefficients as the level loop reads them.  For FP32 they are moved
// to vector registers once: measured on MI355X, chains of FP32 VALU
// instructions with a scalar-register operand issued at half the rate of
// the same chains with vector-register operands only (no packed forms in
// either).  FP64 instructions issue at one rate either way.
template <typename T>
__device__ __forceinline__ Coef<T> lane_coef(Coef<T> c)
{
    if constexpr (sizeof(T) == 4)
        asm("" : "+v"(c.c1), "+v"(c.c2), "+v"(c.cs), "+v"(c.e1), "+v"(c.e2), "+v"(c.es));
    return c;
}

// What a level needs to know about the left wall, seen from one lane (the
// right wall, at a data-dependent element, is handled by right_lone /
// put_at around the level).
template <typename T> struct WallLevel {
    bool isL;       // this lane's point 0 is the lone point at the left wall now
    T dgl;          // g_L(t_{m+1}) - g_L(t_m)
};

// Optional FP64 wall-flux accumulation at the left wall (first difference
// tau (u_1 - g_L)/h at every new level); the right wall's is taken by the
// caller after the level.
struct FluxTap {
    bool left;             // this lane owns the left accumulation
    double accL;
    double tau, h, gln;
};

// The source weight of every point of the lane at parity P,
// B_i = e1 b_i + e2 b_q with q the partner of i (neighbouring lanes' points
// through bl = b_{-1}, br = b_K), formed by the same expression the
// per-level update uses; a launch's profile is fixed, so these are formed
// once per launch and each level adds a(t) B_i with one FMA.
template <typename T, int K, int P>
__device__ __forceinline__ void source_weights(const T (&b)[K], T bl, T br, const Coef<T> &c,
                                               T (&B)[K])
{
    if constexpr (P == 0) {
#pragma unroll
        for (int q = 0; q < K / 2; ++q) {
            B[2 * q] = fmaT(c.e1, b[2 * q], c.e2 * b[2 * q + 1]);
            B[2 * q + 1] = fmaT(c.e1, b[2 * q + 1], c.e2 * b[2 * q]);
        }
    } else {
        B[0] = fmaT(c.e1, b[0], c.e2 * bl);
#pragma unroll
        for (int q = 1; q < K / 2; ++q) {
            const int j = 2 * q - 1;
            B[j] = fmaT(c.e1, b[j], c.e2 * b[j + 1]);
            B[j + 1] = fmaT(c.e1, b[j + 1], c.e2 * b[j]);
        }
        B[K - 1] = fmaT(c.e1, b[K - 1], c.e2 * br);
    }
}

// Advance the K points of every lane by one level of parity P (known at
// compile time: a runtime parity would merge the two groupings' results for
// every point each level and cost the register file).
//   s, e : the lane's points (e is the compensation of the pair, else 0)
//   b    : SRC = 1: the lane's source profile, bl, br: profile of u_{-1}
//          and u_K; SRC = 2: the weights of this parity (source_weights)
//   xl, xl2, xr, xr2 : u_{-1}, u_{-2}, u_K, u_{K+1} for lanes 0 / 63 (DPP
//          fill from the neighbouring waves, a wall value, or anything at
//          an open window edge); yl.. the same for e
// WALL instantiations apply the lone-point formulas and the flux tap; every
// other point of every instantiation evaluates the same expressions.  OPEN:
// both edges of the wave are open window edges, so the fills are not used.
template <typename T, int K, bool COMP, int SRC, bool WALL, int P, bool OPEN = false>
__device__ __forceinline__ void ge_level(T (&s)[K], T (&e)[K], const T (&b)[K], T bl, T br,
                                         T xl, T xl2, T xr, T xr2, T yl, T yl2, T yr, T yr2,
                                         const Coef<T> &c, T an,
                                         const WallLevel<T> &wl, FluxTap &ft)
{
    static_assert(!(WALL && SRC == 2), "wall tiles take the source from the profile");
    const T c1 = c.c1, c2 = c.c2, cs = c.cs, e1 = c.e1, e2 = c.e2, es = c.es;
    // u_{-1} and u_K: neighbour lanes' edge points
    const T sl = edge_left<OPEN>(xl, s[K - 1]), sr = edge_right<OPEN>(xr, s[0]);
    T el = T(0), er = T(0);
    if constexpr (COMP) { el = edge_left<OPEN>(yl, e[K - 1]); er = edge_right<OPEN>(yr, e[0]); }

    auto dif = [](T s1, T e1_, T s0, T e0) { return ::ge::dev::dif<T, COMP>(s1, e1_, s0, e0); };
    auto sd = [](Dif<T, COMP> da, Dif<T, COMP> db) { return ::ge::dev::sd<T, COMP>(da, db); };
    // advance point j from D_self and D_partner (bp: partner's profile)
    auto upd = [&](int j, T Ds, T Dp, T bp) {
        if constexpr (COMP) {
            T inc = fmaT(c1, Ds, c2 * Dp);
            if constexpr (SRC == 1) inc = fmaT(an, fmaT(e1, b[j], e2 * bp), inc);
            if constexpr (SRC == 2) inc = fmaT(an, b[j], inc);
            if constexpr (WALL) {
                if (j == 0) {
                    T alt = cs * (Ds + wl.dgl);
                    if constexpr (SRC) alt = fmaT(an, es * b[j], alt);
                    inc = wl.isL ? alt : inc;
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
            if constexpr (SRC == 1) t = fmaT(an, fmaT(e1, b[j], e2 * bp), t);
            if constexpr (SRC == 2) t = fmaT(an, b[j], t);
            T v = fmaT(c2, Dp, t);
            if constexpr (WALL) {
                if (j == 0) {
                    T alt = fmaT(cs, Ds + wl.dgl, s[j]);
                    if constexpr (SRC) alt = fmaT(an, es * b[j], alt);
                    v = wl.isL ? alt : v;
                }
            }
            s[j] = v;
        } else {
            // FP32: form the increment first, so u is rounded once per level
            T inc = fmaT(c1, Ds, c2 * Dp);
            if constexpr (SRC == 1) inc = fmaT(an, fmaT(e1, b[j], e2 * bp), inc);
            if constexpr (SRC == 2) inc = fmaT(an, b[j], inc);
            if constexpr (WALL) {
                if (j == 0) {
                    T alt = cs * (Ds + wl.dgl);
                    if constexpr (SRC) alt = fmaT(an, es * b[j], alt);
                    inc = wl.isL ? alt : inc;
                }
            }
            s[j] = s[j] + inc;
        }
        if constexpr (WALL) {
            // wall first differences at the new level, accumulated in FP64
            if (ft.left && j == 0) {
                const double v = (double)s[j] + (COMP ? (double)e[j] : 0.0);
                ft.accL = ft.accL + ft.tau * (v - ft.gln) / ft.h;
            }
        }
    };

    if constexpr (P == 0) {
        // pairs (2q, 2q+1) inside the lane
        auto dprev = dif(s[0], e[0], sl, el);                       // d_{-1}
#pragma unroll
        for (int q = 0; q < K / 2; ++q) {
            const int j = 2 * q;
            const auto d0 = dif(s[j + 1], e[j + 1], s[j], e[j]);    // d_j
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
        const T sl2 = edge_left<OPEN>(xl2, s[K - 2]), sr2 = edge_right<OPEN>(xr2, s[1]);
        T el2 = T(0), er2 = T(0);
        if constexpr (COMP) {
            el2 = edge_left<OPEN>(yl2, e[K - 2]);
            er2 = edge_right<OPEN>(yr2, e[1]);
        }
        const auto dm2 = dif(sl, el, sl2, el2);                     // d_{-2}
        const auto dm1 = dif(s[0], e[0], sl, el);                   // d_{-1}
        const auto d0 = dif(s[1], e[1], s[0], e[0]);                // d_0
        const auto dK1 = dif(sr, er, s[K - 1], e[K - 1]);           // d_{K-1}
        const auto dK = dif(sr2, er2, sr, er);                      // d_K
        const auto dK2 = dif(s[K - 1], e[K - 1], s[K - 2], e[K - 2]);  // d_{K-2}
        upd(0, sd(dm1, d0), sd(dm2, dm1), bl);
        auto dprev = d0;
#pragma unroll
        for (int q = 1; q < K / 2; ++q) {
            const int j = 2 * q - 1;
            const auto da = dif(s[j + 1], e[j + 1], s[j], e[j]);   // d_j
            const auto db = dif(s[j + 2], e[j + 2], s[j + 1], e[j + 1]);  // d_{j+1}
            const T Da = sd(dprev, da), Db = sd(da, db);
            upd(j, Da, Db, b[j + 1]);
            upd(j + 1, Db, Da, b[j]);
            dprev = db;
        }
        upd(K - 1, sd(dK2, dK1), sd(dK1, dK), br);
    }
}

// The lone point n-1 beside the right wall (scheme B, Eq. (2), in the
// second-difference form): its new value from the level's old values.  It
// sits at element kS of lane lS; u_{n-2} is element kS-1, or for kS = 0 the
// last element of the lane to the left (xl/yl: that lane's fill value for
// lane 0).  g_hi/g_lo: the wall value at t_m as state values; dgr:
// g_R(t_{m+1}) - g_R(t_m).  The arithmetic is the per-point update's.
template <typename T> struct Lone { T s, e; };

template <typename T, int K, bool COMP, bool SRC>
__device__ __forceinline__ Lone<T> right_lone(const T (&s)[K], const T (&e)[K], const T (&b)[K],
                                              int kS, T xl, T yl, T g_hi, T g_lo, T dgr,
                                              const Coef<T> &c, T an)
{
    const T sl = from_left(xl, s[K - 1]);
    const T el = COMP ? from_left(yl, e[K - 1]) : T(0);
    const T u1 = get_at<T, K>(s, kS, T(0));
    const T e1 = COMP ? get_at<T, K>(e, kS, T(0)) : T(0);
    const T u0 = get_at<T, K>(s, kS - 1, sl);
    const T e0 = COMP ? get_at<T, K>(e, kS - 1, el) : T(0);
    const T Ds = sd<T, COMP>(dif<T, COMP>(u1, e1, u0, e0), dif<T, COMP>(g_hi, g_lo, u1, e1));
    Lone<T> out{u1, e1};
    if constexpr (COMP) {
        T inc = c.cs * (Ds + dgr);
        if constexpr (SRC) inc = fmaT(an, c.es * get_at<T, K>(b, kS, T(0)), inc);
        const T y = inc + e1;
        const T tt = u1 + y;
        out.e = y - (tt - u1);
        out.s = tt;
    } else if constexpr (sizeof(T) == 8) {
        T alt = fmaT(c.cs, Ds + dgr, u1);
        if constexpr (SRC) alt = fmaT(an, c.es * get_at<T, K>(b, kS, T(0)), alt);
        out.s = alt;
    } else {
        T inc = c.cs * (Ds + dgr);
        if constexpr (SRC) inc = fmaT(an, c.es * get_at<T, K>(b, kS, T(0)), inc);
        out.s = u1 + inc;
    }
    return out;
}

// Run levels level0 .. level0+nlev-1 as f(parity, lev) with the parity a
// compile-time constant: an odd first level alone, then even/odd pairs, then
// a last even level if one is left.
template <int V> struct Par { static constexpr int value = V; };

template <typename F>
__device__ __forceinline__ void for_levels(int64_t level0, int nlev, F &&f)
{
    int lev = 0;
    if ((level0 & 1) && nlev > 0) {
        f(Par<1>{}, 0);
        lev = 1;
    }
    for (; lev + 1 < nlev; lev += 2) {
        f(Par<0>{}, lev);
        f(Par<1>{}, lev + 1);
    }
    if (lev < nlev)
        f(Par<0>{}, lev);
}

}  // namespace dev
}  // namespace ge
