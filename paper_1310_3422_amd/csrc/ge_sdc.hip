// The scheme with sub-domains of k nodes (Section 2: the complementary
// scheme with odd and even sub-domains of width k; Eq. (3)/(4) where
// sub-domains meet, Saul'yev's scheme A, Eq. (1), and scheme B, Eq. (2),
// swept through the sub-domains).
//
// Nodes x_0..x_M (h = 1/M, M = n + 1 = 2ek); node j is array element j-1.
// A sub-domain couple (SDC) is an odd sub-domain followed by an even one,
// 2k = K nodes: SDC i holds nodes iK .. iK+K-1.  Lane l of a window holds
// array elements [lK, lK + K) of its SDC i, i.e. nodes iK+1 .. iK+K: SDC i
// without its first node, plus the first node of SDC i+1 (element K-1).
// With that layout every confluence pair lies inside one lane, and each
// level needs one value from a neighbouring lane before its sweeps and at
// most one after.  For the last SDC, element K-1 is the right wall node x_M
// (one past the array); it holds the wall value of the current level.
//
// Levels of even global index take the first kind (pairs where two SDCs
// meet: nodes (iK-1, iK) = elements K-2, K-1 of lane i-1; scheme A through
// the odd sub-domain from its first node, B through the even one from its
// last), odd levels the second kind (pairs at each SDC's centre, nodes
// (iK+k-1, iK+k) = elements k-2, k-1; B through the odd sub-domain down to
// its first node, which the lane to the left holds; A through the even one).
// The pairs take Eq. (3)/(4) with denominator 1 + 2r in second-difference
// form; a sweep step is fma(c, v_prev, fma(ca, w, c w_other)), c = r/(1+r),
// ca = (1-r)/(1+r), taken two nodes at a time (see sweep_run).
//
// Temporal blocking: a launch advances `nlev` levels of a window of NW x 64
// SDCs (NW waves of one workgroup) and writes back its core; the window
// moves through LDS on the way in and out, so that HBM sees consecutive
// 16-byte chunks across the lanes.  A wrong value at an open window edge
// spreads at most k + 1 nodes per level (through a sweep), so the halo is
// ceil((D (k+1) + 2) / K) whole SDCs on each side (measured tight to within
// one SDC on the CPU against the oracle), whatever the window's width: wider
// windows recompute a smaller share of halo.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ge_kernels.h"
#include "ge_level.h"

namespace ge {
namespace {

using namespace dev;

template <typename T> struct SdcCoef {
    T c, ca;      // r/(1+r), (1-r)/(1+r): the sweep step
    T c1, c2;     // (r+r^2)/(1+2r), r^2/(1+2r): the pair
    T cc;         // c * c: two sweep steps at once
};

// in vector registers for FP32 (see lane_coef)
template <typename T>
__device__ __forceinline__ SdcCoef<T> sdc_lane_coef(SdcCoef<T> k)
{
    k.cc = k.c * k.c;
    if constexpr (sizeof(T) == 4)
        asm("" : "+v"(k.c), "+v"(k.ca), "+v"(k.c1), "+v"(k.c2), "+v"(k.cc));
    return k;
}

// Eq. (3)/(4) for the pair (u0, u1), outer neighbours um, u2 (old level)
template <typename T>
__device__ __forceinline__ void sdc_pair(T um, T u0, T u1, T u2, const SdcCoef<T> &k, T &n0,
                                         T &n1)
{
    const T dm = u0 - um, d0 = u1 - u0, d1 = u2 - u1;
    const T Da = d0 - dm, Db = d1 - d0;
    n0 = fmaT(k.c2, Db, fmaT(k.c1, Da, u0));
    n1 = fmaT(k.c2, Da, fmaT(k.c1, Db, u1));
}

// One Saul'yev step: (r v + (1-r) w + r wo) / (1+r), with v the new value
// of the sweep predecessor and wo the old value of the other neighbour
template <typename T>
__device__ __forceinline__ T sweep(T v, T w, T wo, const SdcCoef<T> &k)
{
    return fmaT(k.c, v, fmaT(k.ca, w, k.c * wo));
}

// A sweep through elements FROM..TO (in either direction) of the lane's
// registers, starting from the new value v of the node before FROM.  The
// recurrence v_e = c v_prev + t_e, t_e = ca w_e + c wo_e, is a chain of
// dependent FMAs; two steps are taken at once, v_{e+1} = c^2 v + (c t_e +
// t_{e+1}), with v_e off the chain, which halves its length.  other(e) is
// the old value of e's neighbour on the far side (read before anything is
// written over it).  Returns the value of the last node.
template <typename T, int K, int FROM, int TO, typename Other>
__device__ __forceinline__ T sweep_run(T (&s)[K], T v, const SdcCoef<T> &k, Other other)
{
    constexpr int step = FROM <= TO ? 1 : -1;
    constexpr int len = (TO - FROM) * step + 1;
#pragma unroll
    for (int j = 0; j + 1 < len; j += 2) {
        const int e0 = FROM + j * step, e1 = e0 + step;
        const T t0 = fmaT(k.ca, s[e0], k.c * other(e0));
        const T t1 = fmaT(k.ca, s[e1], k.c * other(e1));
        const T u = fmaT(k.c, t0, t1);
        const T v0 = fmaT(k.c, v, t0);
        v = fmaT(k.cc, v, u);
        s[e0] = v0;
        s[e1] = v;
    }
    if constexpr (len % 2 == 1) {
        constexpr int e = TO;
        v = fmaT(k.c, v, fmaT(k.ca, s[e], k.c * other(e)));
        s[e] = v;
    }
    return v;
}

// Values that cross a wave's edges.  A level needs, besides its own lanes,
// one value from each side: at even levels the right neighbour's element 0
// before the level and the left neighbour's new element K-1 (its pair's
// right value) half-way through; at odd levels the left neighbour's element
// K-1 before the level and the right neighbour's new element 0 at its end.
// Each of the two mid-level values is also the other side's start value of
// the next level, so a window of NW waves exchanges its waves' edge lanes
// through LDS once per level (one barrier), plus once when a window is
// loaded.  Lanes 0 and 63 of the window's outer waves take zeros, which
// reach only the halo; a single-wave window (NW = 1) exchanges nothing.
template <typename T, int NW>
struct SdcEdge {
    T (*slot)[NW][2];    // [3][NW][2] in LDS: per level parity, and at load
    int w;               // this wave in the workgroup
    T xr0 = T(0);        // right wave's element 0 of lane 0, current level
    T xl63 = T(0);       // left wave's element K-1 of lane 63, current level

    // a window's registers are loaded: both start values
    template <int K>
    __device__ __forceinline__ void start(int lane, const T (&s)[K])
    {
        if constexpr (NW > 1) {
            if (lane == 0) slot[2][w][0] = s[0];
            if (lane == kWave - 1) slot[2][w][1] = s[K - 1];
            __syncthreads();
            xr0 = w < NW - 1 ? slot[2][w + 1][0] : T(0);
            xl63 = w > 0 ? slot[2][w - 1][1] : T(0);
        }
    }
    // even level, mid-way: lane 63's new pair value to the right wave
    __device__ __forceinline__ T mid_left(int lane, int buf, T pb)
    {
        if constexpr (NW > 1) {
            if (lane == kWave - 1) slot[buf][w][1] = pb;
            __syncthreads();
            xl63 = w > 0 ? slot[buf][w - 1][1] : T(0);
            return xl63;
        } else {
            return T(0);
        }
    }
    // odd level, at its end: lane 0's new element 0 to the left wave
    __device__ __forceinline__ T end_right(int lane, int buf, T s0)
    {
        if constexpr (NW > 1) {
            if (lane == 0) slot[buf][w][0] = s0;
            __syncthreads();
            xr0 = w < NW - 1 ? slot[buf][w + 1][0] : T(0);
            return xr0;
        } else {
            return T(0);
        }
    }
};

// One level of the lane's SDC.  first / last: the lane holds the rod's first
// / last SDC (walls); gl_old, gl_new: left wall at this and the next level;
// gr_new: right wall at the next level.  Values entering the wave from
// outside come from `edge` (zeros at the window's open edges: they only
// reach the halo); buf: the level's exchange slot (its parity in the launch).
template <typename T, int K, int KIND, int NW>
__device__ __forceinline__ void sdc_level(T (&s)[K], const SdcCoef<T> &cf, bool first, bool last,
                                          T gl_old, T gl_new, T gr_new, SdcEdge<T, NW> &edge,
                                          int lane, int buf)
{
    constexpr int k = K / 2;
    static_assert(k >= 2, "sub-domains of two or more nodes");
    if constexpr (KIND == 1) {
        // pair at the boundary with the next SDC: elements K-2, K-1
        const T oR = from_right(edge.xr0, s[0]);
        T pA, pB;
        sdc_pair(s[K - 3], s[K - 2], s[K - 1], oR, cf, pA, pB);
        if (last) {
            // node M-1 by scheme B against the wall, node M the wall
            pA = sweep(gr_new, s[K - 2], s[K - 3], cf);
            pB = gr_new;
        }
        // scheme A through the odd sub-domain, from its first node (the
        // left lane's pair value, or the left wall)
        T v = from_left(edge.mid_left(lane, buf, pB), pB);
        if (first) v = gl_new;
        const T o_odd_last = s[k - 2];
        sweep_run<T, K, 0, k - 2>(s, v, cf, [&](int e) { return s[e + 1]; });
        // scheme B through the even sub-domain, from its last node
        sweep_run<T, K, K - 3, k - 1>(s, pA, cf,
                                      [&](int e) { return e - 1 == k - 2 ? o_odd_last : s[e - 1]; });
        s[K - 2] = pA;
        s[K - 1] = pB;
    } else {
        // node iK (this SDC's first node) lives in the left lane
        const T fl = from_left(edge.xl63, s[K - 1]);
        const T oL = first ? gl_old : fl;
        // pair at the centre: elements k-2, k-1
        T qA, qB;
        sdc_pair(k == 2 ? oL : s[k == 2 ? 0 : k - 3], s[k - 2], s[k - 1], s[k], cf, qA, qB);
        const T o_last = s[K - 1], o_prev = s[K - 2];
        // scheme B down the odd sub-domain
        if constexpr (k >= 3)
            sweep_run<T, K, k - 3, 0>(s, qA, cf, [&](int e) { return e >= 1 ? s[e - 1] : oL; });
        // scheme A up the even sub-domain
        sweep_run<T, K, k, K - 2>(s, qB, cf, [&](int e) { return s[e + 1]; });
        s[k - 2] = qA;
        s[k - 1] = qB;
        // element K-1 is the first node of the next SDC, the end of its
        // scheme-B sweep: it needs that lane's new element 0
        const T r0 = from_right(edge.end_right(lane, buf, s[0]), s[0]);
        const T nk = sweep(r0, o_last, o_prev, cf);
        s[K - 1] = last ? gr_new : nk;
    }
}

// A window's 64 K values go between HBM and the lanes through LDS: the
// global side moves consecutive 16-byte chunks across the lanes (coalesced;
// a lane's own K values are 16 K bytes apart from its neighbours'), the LDS
// side hands each lane its row.  Rows are padded by 16 bytes, so the 16
// lanes of a row read hit distinct banks.
template <typename T, int K>
struct Stage {
    static constexpr int E = 16 / sizeof(T);          // values per chunk
    static constexpr int P = K + E;                   // padded row
    static constexpr int CH = kWave * K / E;          // chunks per window
};

// values base .. base + 64K of `in` (those below n; zero beyond) into the
// lanes' rows
template <typename T, int K>
__device__ __forceinline__ void stage_load(const T *__restrict__ in, int64_t base, int64_t n,
                                           T *lds, T (&s)[K])
{
    using S = Stage<T, K>;
    using V = typename V16<T>::type;
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int j = 0; j < S::CH / kWave; ++j) {
        const int c = j * kWave + lane;               // chunk of the window
        const int e0 = c * S::E;                      // its first value
        const int64_t g = base + e0;
        V x;
        if (g + S::E <= n) {
            x = *reinterpret_cast<const V *>(in + g);
        } else {
            T t[S::E];
#pragma unroll
            for (int q = 0; q < S::E; ++q) t[q] = (g + q < n) ? in[g + q] : T(0);
            if constexpr (S::E == 4) x = V{t[0], t[1], t[2], t[3]};
            else x = V{t[0], t[1]};
        }
        *reinterpret_cast<V *>(&lds[(e0 / K) * S::P + e0 % K]) = x;
    }
    __syncthreads();
    const V *row = reinterpret_cast<const V *>(&lds[lane * S::P]);
#pragma unroll
    for (int q = 0; q < K / S::E; ++q) {
        const V x = row[q];
        if constexpr (S::E == 4) {
            s[4 * q] = x.x; s[4 * q + 1] = x.y; s[4 * q + 2] = x.z; s[4 * q + 3] = x.w;
        } else {
            s[2 * q] = x.x; s[2 * q + 1] = x.y;
        }
    }
    __syncthreads();   // the rows are free again
}

// the lanes' rows back to `out`, values of window positions [lo, hi) that
// lie below n (lo, hi multiples of K)
template <typename T, int K>
__device__ __forceinline__ void stage_store(T *__restrict__ out, int64_t base, int64_t n, int lo,
                                            int hi, T *lds, const T (&s)[K], T &fin)
{
    using S = Stage<T, K>;
    using V = typename V16<T>::type;
    const int lane = threadIdx.x % kWave;
    V *row = reinterpret_cast<V *>(&lds[lane * S::P]);
#pragma unroll
    for (int q = 0; q < K / S::E; ++q) {
        V x;
        if constexpr (S::E == 4) x = V{s[4 * q], s[4 * q + 1], s[4 * q + 2], s[4 * q + 3]};
        else x = V{s[2 * q], s[2 * q + 1]};
        row[q] = x;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < S::CH / kWave; ++j) {
        const int c = j * kWave + lane;
        const int e0 = c * S::E;
        if (e0 < lo || e0 >= hi)
            continue;
        const int64_t g = base + e0;
        const V x = *reinterpret_cast<const V *>(&lds[(e0 / K) * S::P + e0 % K]);
        T u[S::E];
        if constexpr (S::E == 4) {
            u[0] = x.x; u[1] = x.y; u[2] = x.z; u[3] = x.w;
        } else {
            u[0] = x.x; u[1] = x.y;
        }
        if (g + S::E <= n) {
#pragma unroll
            for (int q = 0; q < S::E; ++q) finite_acc(fin, u[q]);
            *reinterpret_cast<V *>(out + g) = x;
        } else {
#pragma unroll
            for (int q = 0; q < S::E; ++q)
                if (g + q < n) {
                    finite_acc(fin, u[q]);
                    out[g + q] = u[q];
                }
        }
    }
}

// window positions [c0, c1) of the core, as values of the part of wave w
// (SDCs wb .. wb+63), clipped to the part
__device__ __forceinline__ int part_pos(int64_t c, int64_t wb, int K)
{
    const int64_t e = (c - wb) * K;
    return e < 0 ? 0 : e > (int64_t)kWave * K ? kWave * K : (int)e;
}

template <typename T, int K, int NW>
__global__ __launch_bounds__(NW * kWave) void sdc_tile_kernel(TileArgs a)
{
    // consecutive tiles on one XCD, as in the two-point sweep
    const int64_t per = gridDim.x / 8;
    const int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (t >= a.ntiles)
        return;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t c0 = t * a.core;                              // first core SDC
    const int64_t w0 = c0 - a.halo < 0 ? 0 : c0 - a.halo;       // first SDC of the window
    const int64_t wb = w0 + (int64_t)w * kWave;                 // first SDC of this wave
    const int64_t i = wb + lane;                                // this lane's SDC
    const T *in = static_cast<const T *>(a.in);
    T *out = static_cast<T *>(a.out);
    __shared__ __attribute__((aligned(16))) T lds[NW][kWave * Stage<T, K>::P];
    __shared__ T slot[3][NW][2];
    T s[K];
    stage_load<T, K>(in, wb * K, a.n, lds[w], s);
    const bool first = (i == 0), last = (i == a.nsdc - 1);
    auto gl = [&](int lev) { return a.gl_t ? a.gl_t[lev] : a.gl0; };
    auto gr = [&](int lev) { return a.gr_t ? a.gr_t[lev] : a.gr0; };
    if (last) s[K - 1] = (T)gr(0);
    const SdcCoef<T> cf = sdc_lane_coef(SdcCoef<T>{(T)a.cs, (T)a.ca, (T)a.c1, (T)a.c2});
    SdcEdge<T, NW> edge{slot, w};
    edge.start(lane, s);
    for_levels(a.level0, a.nlev, [&](auto par, int lev) {
        constexpr int p = decltype(par)::value;
        sdc_level<T, K, p == 0 ? 1 : 2, NW>(s, cf, first, last, (T)gl(lev), (T)gl(lev + 1),
                                             (T)gr(lev + 1), edge, lane, lev & 1);
    });
    const int64_t c1 = c0 + a.core < a.nsdc ? c0 + a.core : a.nsdc;
    T fin = T(0);
    stage_store<T, K>(out, wb * K, a.n, part_pos(c0, wb, K), part_pos(c1, wb, K), lds[w], s, fin);
    raise_if_nonfinite(a.status, fin);
}

// Persistent form.  Workgroups of NW waves stay resident and take the tiles
// round by round (each wave the same 64-SDC part of every window); while a tile advances through its levels, the next tile's
// window is copied from HBM straight into the wave's LDS buffer
// (global_load_lds: no registers held), so the HBM traffic of a launch
// hides behind its arithmetic instead of alternating with it.  When the
// levels are done the registers and the buffer swap contents chunk by chunk:
// the registers take the next window, the buffer the results, which then go
// out in coalesced chunks before the following copy is issued.
//
// The buffer holds the window's 64 rows of K values as 16-byte chunks; the
// chunks of row l sit in the row's slots permuted by XOR with l mod Q (Q
// chunks per row), so that lanes reading their own rows spread over the
// banks, while each copy instruction still fills 64 consecutive slots from
// one contiguous kilobyte of HBM.
template <typename T, int K>
struct Swz {
    static constexpr int E = 16 / sizeof(T);          // values per chunk
    static constexpr int Q = K / E;                   // chunks per row
    static_assert(Q >= 1 && (Q & (Q - 1)) == 0, "rows of a power-of-two number of chunks");
    // slot of chunk q of row l
    static __device__ __forceinline__ int slot(int l, int q) { return l * Q + (q ^ (l % Q)); }
    // window chunk held by slot s
    static __device__ __forceinline__ int chunk(int s)
    {
        const int l = s / Q;
        return l * Q + ((s % Q) ^ (l % Q));
    }
};

using lds_void = __attribute__((address_space(3))) void;

// One 16-byte chunk per lane from global memory straight into LDS.  (A plain
// function: the builtin exists only for the device, and the host pass would
// otherwise reject every use of a template that calls it but the first.)
__device__ __forceinline__ void copy16_to_lds(const void *src, void *dst)
{
    __builtin_amdgcn_global_load_lds(src, (lds_void *)dst, 16, 0, 0);
}

// Issue the copy of window values base .. base + 64K of `in` into the
// buffer.  A chunk that reaches past the rod is replaced by chunk 0 (any
// valid address; tail_fix overwrites those values).
template <typename T, int K>
__device__ __forceinline__ void dma_window(const T *__restrict__ in, int64_t base, int64_t n,
                                           T *lds)
{
    using S = Swz<T, K>;
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int j = 0; j < S::Q; ++j) {
        const int64_t g = base + (int64_t)S::chunk(j * kWave + lane) * S::E;
        const T *src = g + S::E <= n ? in + g : in;
        copy16_to_lds(src, lds + j * kWave * S::E);
    }
}

// the copies into LDS count as vector-memory operations; the compiler does
// not order LDS reads after them, so the wave waits explicitly
__device__ __forceinline__ void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
// LDS reads finished before a copy may overwrite what they read
__device__ __forceinline__ void wait_lds() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

template <typename T, int K>
__device__ __forceinline__ void unpack(const typename V16<T>::type &x, T (&s)[K], int q)
{
    if constexpr (V16<T>::E == 4) {
        s[4 * q] = x.x; s[4 * q + 1] = x.y; s[4 * q + 2] = x.z; s[4 * q + 3] = x.w;
    } else {
        s[2 * q] = x.x; s[2 * q + 1] = x.y;
    }
}

template <typename T, int K>
__device__ __forceinline__ typename V16<T>::type pack(const T (&s)[K], int q)
{
    using V = typename V16<T>::type;
    if constexpr (V16<T>::E == 4) return V{s[4 * q], s[4 * q + 1], s[4 * q + 2], s[4 * q + 3]};
    else return V{s[2 * q], s[2 * q + 1]};
}

// the lane's row out of the buffer
template <typename T, int K>
__device__ __forceinline__ void rows_read(const T *lds, T (&s)[K])
{
    using S = Swz<T, K>;
    using V = typename V16<T>::type;
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int q = 0; q < S::Q; ++q)
        unpack<T, K>(*reinterpret_cast<const V *>(&lds[S::slot(lane, q) * S::E]), s, q);
}

// the lane's row into the buffer
template <typename T, int K>
__device__ __forceinline__ void rows_write(T *lds, const T (&s)[K])
{
    using S = Swz<T, K>;
    using V = typename V16<T>::type;
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int q = 0; q < S::Q; ++q)
        *reinterpret_cast<V *>(&lds[S::slot(lane, q) * S::E]) = pack<T, K>(s, q);
}

// registers and buffer exchange contents, one chunk at a time (each slot is
// read before the lane writes it)
template <typename T, int K>
__device__ __forceinline__ void rows_swap(T *lds, T (&s)[K])
{
    using S = Swz<T, K>;
    using V = typename V16<T>::type;
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int q = 0; q < S::Q; ++q) {
        V *p = reinterpret_cast<V *>(&lds[S::slot(lane, q) * S::E]);
        const V x = *p;
        *p = pack<T, K>(s, q);
        unpack<T, K>(x, s, q);
    }
}

// values of window positions [lo, hi) below n, from the buffer to `out`
template <typename T, int K>
__device__ __forceinline__ void chunks_store(T *__restrict__ out, int64_t base, int64_t n, int lo,
                                             int hi, const T *lds, T &fin)
{
    using S = Swz<T, K>;
    using V = typename V16<T>::type;
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int j = 0; j < S::Q; ++j) {
        const int sl = j * kWave + lane;
        const int e0 = S::chunk(sl) * S::E;
        if (e0 < lo || e0 >= hi)
            continue;
        const int64_t g = base + e0;
        const V x = *reinterpret_cast<const V *>(&lds[sl * S::E]);
        T u[K];
        unpack<T, K>(x, u, 0);
        if (g + S::E <= n) {
#pragma unroll
            for (int q = 0; q < S::E; ++q) finite_acc(fin, u[q]);
            *reinterpret_cast<V *>(out + g) = x;
        } else {
#pragma unroll
            for (int q = 0; q < S::E; ++q)
                if (g + q < n) {
                    finite_acc(fin, u[q]);
                    out[g + q] = u[q];
                }
        }
    }
}

// A window that reaches past the rod, after its copy has landed: each lane
// rewrites its own row in the buffer from plain loads, zero past the rod
// (the copy read chunk 0 there).  Wave-uniform branch; the loads are waited
// for inside it, so no load is pending in registers when the branch ends.
template <typename T, int K>
__device__ __forceinline__ void tail_fix(const T *__restrict__ in, int64_t base, int64_t n,
                                         T *lds)
{
    if (base + (int64_t)kWave * K <= n)
        return;
    const int64_t b = base + (int64_t)(threadIdx.x % kWave) * K;
    T v[K];
#pragma unroll
    for (int e = 0; e < K; ++e)
        v[e] = b + e < n ? in[b + e] : T(0);
    rows_write<T, K>(lds, v);
}

template <typename T, int K, int NW>
__global__ __launch_bounds__(NW * kWave) void sdc_persistent_kernel(TileArgs a, int nwg)
{
    __shared__ __attribute__((aligned(16))) T lds_all[NW][kWave * K];
    __shared__ double walls[2][kSdcMaxLevels + 1];
    __shared__ T slot[3][NW][2];
    const int per = nwg / 8;
    int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;   // XCD-aware
    if (t >= a.ntiles)
        return;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    T *lds = lds_all[w];
    const T *in = static_cast<const T *>(a.in);
    T *out = static_cast<T *>(a.out);
    // first SDC of this wave's part of tile tt's window
    auto wstart = [&](int64_t tt) {
        const int64_t c0 = tt * a.core;
        return (c0 - a.halo < 0 ? (int64_t)0 : c0 - a.halo) + (int64_t)w * kWave;
    };
    // The wall values of the launch's levels, read once: inside the loop
    // every wait on vector memory would also wait for the pending copy.
    for (int j = threadIdx.x; j <= a.nlev; j += NW * kWave) {
        walls[0][j] = a.gl_t ? a.gl_t[j] : a.gl0;
        walls[1][j] = a.gr_t ? a.gr_t[j] : a.gr0;
    }
    if constexpr (NW > 1)
        __syncthreads();
    auto gl = [&](int lev) { return walls[0][lev]; };
    auto gr = [&](int lev) { return walls[1][lev]; };
    T s[K];
    dma_window<T, K>(in, wstart(t) * K, a.n, lds);
    wait_vmem();
    tail_fix<T, K>(in, wstart(t) * K, a.n, lds);
    rows_read<T, K>(lds, s);
    const SdcCoef<T> cf = sdc_lane_coef(SdcCoef<T>{(T)a.cs, (T)a.ca, (T)a.c1, (T)a.c2});
    SdcEdge<T, NW> edge{slot, w};
    for (;;) {
        const int64_t wb = wstart(t);
        const int64_t tn = t + nwg;
        const bool more = tn < a.ntiles;
        wait_lds();
        if (more)
            dma_window<T, K>(in, wstart(tn) * K, a.n, lds);
        const int64_t i = wb + lane;
        const bool first = (i == 0), last = (i == a.nsdc - 1);
        if (last) s[K - 1] = (T)gr(0);
        edge.start(lane, s);
        for_levels(a.level0, a.nlev, [&](auto par, int lev) {
            constexpr int p = decltype(par)::value;
            sdc_level<T, K, p == 0 ? 1 : 2, NW>(s, cf, first, last, (T)gl(lev), (T)gl(lev + 1),
                                                 (T)gr(lev + 1), edge, lane, lev & 1);
        });
        const int64_t c0 = t * a.core;
        const int64_t c1 = c0 + a.core < a.nsdc ? c0 + a.core : a.nsdc;
        if (more) {
            wait_vmem();
            tail_fix<T, K>(in, wstart(tn) * K, a.n, lds);
            rows_swap<T, K>(lds, s);
        } else {
            rows_write<T, K>(lds, s);
        }
        T fin = T(0);
        chunks_store<T, K>(out, wb * K, a.n, part_pos(c0, wb, K), part_pos(c1, wb, K), lds, fin);
        raise_if_nonfinite(a.status, fin);
        if (!more)
            break;
        t = tn;
    }
}

template <typename T, int K, int NW>
hipError_t launch_persistent_sdc(const TileArgs &a, hipStream_t stream)
{
    static int per_cu = 0, ncu = 0;
    if (per_cu == 0) {
        int dev = 0, nb = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sdc_persistent_kernel<T, K, NW>,
                                                         NW * kWave, 0) != hipSuccess ||
            nb < 1 || ncu < 1)
            return hipErrorInvalidValue;
        per_cu = nb;
    }
    // as many workgroups as stay resident, trimmed so that every one gets
    // the same number of tiles (to one), in multiples of 8
    const int64_t cap = (int64_t)per_cu * ncu;
    const int64_t rounds = (a.ntiles + cap - 1) / cap;
    int64_t nwg = (a.ntiles + rounds - 1) / rounds;
    nwg = (nwg + 7) / 8 * 8;
    hipLaunchKernelGGL((sdc_persistent_kernel<T, K, NW>), dim3((unsigned)nwg), dim3(NW * kWave), 0,
                       stream, a, (int)nwg);
    return hipGetLastError();
}

template <typename T, int K, int NW>
hipError_t launch_one_sdc(const TileArgs &a, hipStream_t stream)
{
    const int64_t grid = (a.ntiles + 7) / 8 * 8;
    hipLaunchKernelGGL((sdc_tile_kernel<T, K, NW>), dim3((unsigned)grid), dim3(NW * kWave), 0,
                       stream, a);
    return hipGetLastError();
}

template <typename T, int K>
hipError_t launch_sdc_nw(int nw, bool persistent, const TileArgs &a, hipStream_t stream)
{
    switch (nw) {
    case 1: return persistent ? launch_persistent_sdc<T, K, 1>(a, stream) : launch_one_sdc<T, K, 1>(a, stream);
    case 2: return persistent ? launch_persistent_sdc<T, K, 2>(a, stream) : launch_one_sdc<T, K, 2>(a, stream);
    case 4: return persistent ? launch_persistent_sdc<T, K, 4>(a, stream) : launch_one_sdc<T, K, 4>(a, stream);
    case 8: return persistent ? launch_persistent_sdc<T, K, 8>(a, stream) : launch_one_sdc<T, K, 8>(a, stream);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_sdc_t(int k, int nw, bool persistent, const TileArgs &a, hipStream_t stream)
{
    switch (k) {
    case 2: return launch_sdc_nw<T, 4>(nw, persistent, a, stream);
    case 4: return launch_sdc_nw<T, 8>(nw, persistent, a, stream);
    case 8: return launch_sdc_nw<T, 16>(nw, persistent, a, stream);
    case 16: return launch_sdc_nw<T, 32>(nw, persistent, a, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool sdc_supported(int prec, int k)
{
    return (prec == kFP64 || prec == kFP32) && (k == 2 || k == 4 || k == 8 || k == 16);
}

bool sdc_waves_supported(int nw) { return nw == 1 || nw == 2 || nw == 4 || nw == 8; }

hipError_t launch_sdc(int prec, int k, int nw, const TileArgs &a, hipStream_t stream)
{
    if (prec == kFP64) return launch_sdc_t<double>(k, nw, false, a, stream);
    if (prec == kFP32) return launch_sdc_t<float>(k, nw, false, a, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_sdc_persistent(int prec, int k, int nw, const TileArgs &a, hipStream_t stream)
{
    if (a.ntiles < 3 || a.in == a.out || a.nlev > kSdcMaxLevels)
        return hipErrorInvalidValue;
    if (prec == kFP64) return launch_sdc_t<double>(k, nw, true, a, stream);
    if (prec == kFP32) return launch_sdc_t<float>(k, nw, true, a, stream);
    return hipErrorInvalidValue;
}

}  // namespace ge
