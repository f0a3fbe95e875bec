// The surrogate's 64-level jump with all six layers fused: one workgroup
// takes a tile of kFP points of one rod from u to u_next, keeping every
// activation in LDS, so HBM sees only u (read) and u_next (written) -- the
// layer-by-layer path writes and re-reads 128 bytes per point per layer.
//
// Each layer is computed on kFR = kFP + 128 rows (64 beyond each side of the
// tile).  A layer of tap spacing d reads its input 2d rows either side, so
// after each layer the rows whose inputs were not all computed grow by 2d at
// each edge of the computed range; after the six layers (spacings 1, 2, 4,
// 8, 16, 1) that is 64 rows, and the valid rows are exactly the tile.  Rows
// outside the rod are set to zero after every layer, which is the zero
// padding of the layer-by-layer path.  The
// arithmetic (the features, the MFMA accumulation order, the epilogues and
// the jump) is the same expression sequence as the layer-by-layer kernels,
// so both paths give the same bits.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ge_nn.h"
#include "ge_nn_dev.h"

namespace ge {
namespace nn {
namespace {

using namespace dev;

constexpr int kFP = 512;                   // output points per workgroup
constexpr int kFHalo = 64;                 // computed rows beyond each side (= 2 x sum of spacings)
constexpr int kFR = kFP + 2 * kFHalo;      // rows computed per layer (40 M-tiles)
constexpr int kFWaves = 8;                 // 5 M-tiles of 16 rows per wave, two waves per SIMD
constexpr int kFMT = kFR / 16 / kFWaves;
constexpr int kFPad = 2 * kMaxDil;         // LDS rows beyond the computed rows on each side
constexpr int kFRows = kFR + 2 * kFPad;
constexpr int kFXS = 72;                   // LDS row pitch (bf16): 64 channels + 16 bytes
constexpr int kFThreads = 64 * kFWaves;
static_assert(kFR % (16 * kFWaves) == 0, "rows per wave");

// LDS row i holds position w0 - kFHalo - kFPad + i; computed row q is LDS
// row q + kFPad.

// One layer's packed weights ([5][cout][cin] bf16), staged through
// registers: fetch() issues every global load of the thread's share at
// once, store() writes them to LDS rows of kFXS later, so the loads of the
// next layer overlap the current layer's matrix work.
template <int CIN, int COUT>
struct WeightStage {
    static constexpr int CPR = CIN / 8;                  // 16-byte chunks per row
    static constexpr int TOTAL = kTaps * COUT * CPR;
    static constexpr int N = (TOTAL + kFThreads - 1) / kFThreads;
    // one vector of 4N words (a plain array here ends up in scratch memory)
    typedef uint32_t Vec __attribute__((ext_vector_type(4 * N)));
    Vec v;
    __device__ __forceinline__ void fetch(const bf16 *wt, int tid)
    {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const int i = tid + j * kFThreads;
            if (TOTAL % kFThreads == 0 || i < TOTAL) {
                const uint4 x = *reinterpret_cast<const uint4 *>(&wt[(i / CPR) * CIN + (i % CPR) * 8]);
                v[4 * j] = x.x;
                v[4 * j + 1] = x.y;
                v[4 * j + 2] = x.z;
                v[4 * j + 3] = x.w;
            }
        }
        // keep the loads here, ahead of the work they are meant to overlap
        __builtin_amdgcn_sched_barrier(0);
    }
    __device__ __forceinline__ void store(bf16 *ws, int tid) const
    {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const int i = tid + j * kFThreads;
            if (TOTAL % kFThreads == 0 || i < TOTAL)
                *reinterpret_cast<uint4 *>(&ws[(i / CPR) * kFXS + (i % CPR) * 8]) =
                    make_uint4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
        }
    }
};

// acc[m][n] += conv of the activations with the layer's weights for the
// wave's M-tiles: same k-outer, channel-chunk-inner order as conv_kernel.
// The product is taken transposed (weights as the A operand, activations
// as B), so that each lane ends with four consecutive output channels of one
// position: acc[m][n][j] is channel 16 n + 4 (lane / 16) + j of position
// 16 (M-tile) + lane % 16, which the epilogue stores as one 8-byte word.
template <int CIN, int COUT>
__device__ __forceinline__ void layer_mfma(const bf16 *act, const bf16 *ws, int wv, int lane, int d,
                                           f32x4 (&acc)[kFMT][COUT / 16])
{
    constexpr int NT = COUT / 16, KC = CIN / 32;
    const int r16 = lane & 15, g4 = lane >> 4;
#pragma unroll
    for (int m = 0; m < kFMT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < kTaps; ++k) {
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            bf16x8 bfr[NT];
#pragma unroll
            for (int n = 0; n < NT; ++n)
                bfr[n] = *reinterpret_cast<const bf16x8 *>(
                    &ws[(k * COUT + 16 * n + r16) * kFXS + 32 * c + 8 * g4]);
#pragma unroll
            for (int m = 0; m < kFMT; ++m) {
                // computed row q reads LDS rows q + kFPad + (k - 2) d
                const int q = 16 * (kFMT * wv + m) + r16;
                const bf16x8 af = *reinterpret_cast<const bf16x8 *>(
                    &act[(q + kFPad + (k - 2) * d) * kFXS + 32 * c + 8 * g4]);
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[n], af, acc[m][n],
                                                                       0, 0, 0);
            }
        }
    }
}

// The epilogue of a GELU layer for the wave's M-tiles, in two halves.
// gelu_compute: bias, GELU and the residual (layers 2..5; it reads only the
// wave's own rows), into registers as four bfloat16 channels per lane and
// M-tile.  It only reads the activations, so it runs before the layer's
// barrier, while other waves (two share a SIMD) are still at their matrix
// work: the GELU's VALU work overlaps their MFMAs.  gelu_store, after the
// barrier (every wave done reading the layer's input): the values in place,
// and rows outside the rod back to zero.
template <bool RES>
__device__ __forceinline__ void gelu_compute(const bf16 *act, const f32x4 (&acc)[kFMT][4],
                                             const float *bias, int wv, int lane,
                                             bf16x4 (&out)[kFMT][4])
{
    const int r16 = lane & 15, g4 = lane >> 4;
    float bl[4][4];
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int j = 0; j < 4; ++j) bl[n][j] = bias[16 * n + 4 * g4 + j];
#pragma unroll
    for (int m = 0; m < kFMT; ++m) {
        const int q = 16 * (kFMT * wv + m) + r16;          // computed row (position)
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            bf16x4 hv;
            if (RES)
                hv = *reinterpret_cast<const bf16x4 *>(&act[(q + kFPad) * kFXS + 16 * n + 4 * g4]);
            f32x4 h;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                h[j] = gelu(acc[m][n][j] + bl[n][j]);
                if (RES) h[j] += bf2f(hv[j]);
            }
            // two values per conversion instruction (round to nearest even)
            out[m][n] = __builtin_convertvector(h, bf16x4);
        }
        // one M-tile at a time: no hoisting of later tiles' reads, which
        // would crowd out the registers of the weights in flight
        __builtin_amdgcn_sched_barrier(0);
    }
}

__device__ __forceinline__ void gelu_store(bf16 *act, const bf16x4 (&out)[kFMT][4], int wv,
                                           int lane, int w0, int W)
{
    const int r16 = lane & 15, g4 = lane >> 4;
    const bf16x4 zero{f2bf(0.f), f2bf(0.f), f2bf(0.f), f2bf(0.f)};
#pragma unroll
    for (int m = 0; m < kFMT; ++m) {
        const int q = 16 * (kFMT * wv + m) + r16;
        const int w = w0 - kFHalo + q;
        // rows outside the rod are zero (the layer-by-layer path's padding);
        // tile_in is wave-uniform, so only the M-tiles at a rod's ends test
        const int wt = w0 - kFHalo + 16 * (kFMT * wv + m);
        const bool tile_in = wt >= 0 && wt + 15 < W;
        const bool in = tile_in || (w >= 0 && w < W);
#pragma unroll
        for (int n = 0; n < 4; ++n)
            *reinterpret_cast<bf16x4 *>(&act[(q + kFPad) * kFXS + 16 * n + 4 * g4]) =
                in ? out[m][n] : zero;
    }
}

__global__ __launch_bounds__(kFThreads) void jump_fused_kernel(FusedArgs a)
{
    __shared__ __attribute__((aligned(16))) bf16 act[kFRows * kFXS];
    __shared__ __attribute__((aligned(16))) bf16 ws[kTaps * 64 * kFXS];
    __shared__ float bias[6][64];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int b = blockIdx.y;
    const int W = a.width;
    const int w0 = blockIdx.x * kFP;
    const int64_t base = (int64_t)b * W;
    const float *ub = a.u + base;
    const float sc = a.scale[b];
    const float rb = a.r[b];
    const float rn = (rb - 1.25f) / 0.75f;

    {
        WeightStage<32, 64> w1;
        w1.fetch(static_cast<const bf16 *>(a.w[0]), tid);
        // features of every LDS row (zero outside the rod), channels 2..63
        // zero, written as 16-byte chunks
        for (int i = tid; i < kFRows; i += kFThreads) {
            const int w = w0 - kFHalo - kFPad + i;
            float f0 = 0.f, f1 = 0.f;
            if (w >= 0 && w < W) {
                const float um = w > 0 ? ub[w - 1] : 0.f, up = w < W - 1 ? ub[w + 1] : 0.f;
                const float d = (um - ub[w]) + (up - ub[w]);
                f0 = d / sc;
                f1 = rn;
            }
            uint4 *row = reinterpret_cast<uint4 *>(&act[i * kFXS]);
            const uint32_t lo = (uint32_t)__builtin_bit_cast(uint16_t, f2bf(f0)) |
                                ((uint32_t)__builtin_bit_cast(uint16_t, f2bf(f1)) << 16);
            row[0] = make_uint4(lo, 0, 0, 0);
#pragma unroll
            for (int c = 1; c < 8; ++c) row[c] = make_uint4(0, 0, 0, 0);
        }
        for (int i = tid; i < 6 * 64; i += kFThreads) {
            const int l = i / 64, c = i % 64;
            bias[l][c] = (l < 5 || c < 16) ? a.bias[l][c] : 0.f;
        }
        w1.store(ws, tid);
    }
    __syncthreads();

    // layers 1..5 (GELU; residual from layer 2 on).  After its matrix work a
    // wave fetches the next layer's weights into registers and computes its
    // epilogue values, both before the barrier, so they overlap the other
    // waves' matrix work; after the barrier it writes the values and the
    // weights to LDS.
    {
        f32x4 acc[kFMT][4];
        bf16x4 outv[kFMT][4];
        {
            layer_mfma<32, 64>(act, ws, wv, lane, a.dil[0], acc);
            WeightStage<64, 64> nx;
            nx.fetch(static_cast<const bf16 *>(a.w[1]), tid);
            gelu_compute<false>(act, acc, bias[0], wv, lane, outv);
            __syncthreads();   // every wave has finished reading act and ws
            gelu_store(act, outv, wv, lane, w0, W);
            nx.store(ws, tid);
            __syncthreads();
        }
#pragma unroll 1
        for (int l = 1; l < 5; ++l) {
            layer_mfma<64, 64>(act, ws, wv, lane, a.dil[l], acc);
            if (l < 4) {
                WeightStage<64, 64> nx;
                nx.fetch(static_cast<const bf16 *>(a.w[l + 1]), tid);
                gelu_compute<true>(act, acc, bias[l], wv, lane, outv);
                __syncthreads();
                gelu_store(act, outv, wv, lane, w0, W);
                nx.store(ws, tid);
            } else {
                WeightStage<64, 16> nx;
                nx.fetch(static_cast<const bf16 *>(a.w[5]), tid);
                gelu_compute<true>(act, acc, bias[l], wv, lane, outv);
                __syncthreads();
                gelu_store(act, outv, wv, lane, w0, W);
                nx.store(ws, tid);
            }
            __syncthreads();   // activations and weights are in place
        }
    }
    // layer 6 (64 -> 1, padded to 16 outputs) and the jump; the lanes that
    // write (channel 0) load their points of u first, to overlap the matrix
    // work
    const int r16 = lane & 15, g4 = lane >> 4;
    float uo[kFMT];
#pragma unroll
    for (int m = 0; m < kFMT; ++m) {
        const int p = 16 * (kFMT * wv + m) + r16 - kFHalo;   // point within the tile
        const int w = w0 + p;
        uo[m] = (g4 == 0 && p >= 0 && p < kFP && w < W) ? ub[w] : 0.f;
    }
    __builtin_amdgcn_sched_barrier(0);
    f32x4 acc6[kFMT][1];
    layer_mfma<64, 16>(act, ws, wv, lane, a.dil[5], acc6);
    if (g4 == 0) {
        // channel 0 of position 16 (M-tile) + r16
        const float b0 = bias[5][0];
        const float amp = 64.0f * rb * sc;
#pragma unroll
        for (int m = 0; m < kFMT; ++m) {
            const int q = 16 * (kFMT * wv + m) + r16;
            const int p = q - kFHalo;                       // point within the tile
            const int w = w0 + p;
            if (p >= 0 && p < kFP && w < W) {
                const float out = acc6[m][0][0] + b0;
                a.u_next[base + w] = uo[m] + amp * out;
            }
        }
    }
}

// Per-rod scale: RMS of the rod's second differences (zero walls), in the
// same summation order as features_kernel.
__global__ __launch_bounds__(256) void rod_scale_kernel(const float *u, int W, float *scale)
{
    const int b = blockIdx.x, tid = threadIdx.x;
    const float *ub = u + (int64_t)b * W;
    __shared__ float red[256];
    float ss = 0.f;
    for (int i = tid; i < W; i += 256) {
        const float um = i > 0 ? ub[i - 1] : 0.f, up = i < W - 1 ? ub[i + 1] : 0.f;
        const float d = (um - ub[i]) + (up - ub[i]);
        ss += d * d;
    }
    red[tid] = ss;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) scale[b] = sqrtf(red[0] / W) + 1e-30f;
}

}  // namespace

hipError_t launch_jump_fused(const FusedArgs &a, int batch, hipStream_t s)
{
    int reach = 0;
    for (int l = 0; l < 6; ++l) {
        if (a.dil[l] < 1 || a.dil[l] > kMaxDil) return hipErrorInvalidValue;
        reach += 2 * a.dil[l];
    }
    if (reach > kFHalo) return hipErrorInvalidValue;   // the tile would not stay valid
    hipLaunchKernelGGL(rod_scale_kernel, dim3(batch), dim3(256), 0, s, a.u, a.width, a.scale);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((a.width + kFP - 1) / kFP, batch);
    hipLaunchKernelGGL(jump_fused_kernel, grid, dim3(kFThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace ge
