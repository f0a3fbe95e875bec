// Kernels of the learned 64-level propagator (the surrogate): a 1D
// convolutional network over the points of a rod, channels last
// (x[b][w][c], bfloat16 storage, FP32 accumulation on the matrix cores).
//
//   layer 1 : pre1 = conv(x, W1) + b1,          h1 = gelu(pre1)         (2 -> 64)
//   layer l : pre_l = conv(h_{l-1}, W_l) + b_l, h_l = h_{l-1} + gelu(pre_l)  (l=2..5)
//   layer 6 : out = conv(h5, W6) + b6                                     (64 -> 1)
//   conv(x, W)[b, w, o] = sum_{k<5} sum_i W[k, o, i] x[b, w + k - 2, i], zero padding.
//
// Channel counts are padded to the matrix-core tiles: the 2 input features
// to 32 channels, the single output to 16.  Every convolution -- forward,
// input gradient (a convolution with the taps reversed and the weight
// transposed) -- runs in conv_kernel as an implicit GEMM on
// v_mfma_f32_16x16x32_bf16: A = activations (positions x input channels),
// B = weights (input x output channels), K = 5 taps x input channels.  The
// weight gradient runs in wgrad_kernel (K = positions) with a fixed-order
// reduction over workgroups, so training is deterministic.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ge_nn.h"
#include "ge_nn_dev.h"

namespace ge {
namespace nn {
namespace {

using namespace dev;

constexpr int kMT = 128;          // positions per workgroup tile
constexpr int kThreads = 256;     // 4 waves, 32 positions each

// ---------------------------------------------------------------------------
// Convolution as an implicit GEMM.
//   x   : [B][W][CIN] bf16 input, read at offsets (k - 2) d from each output
//   wt  : [5][COUT][CIN] bf16 weights (B operand layout: output channel rows)
//   bias: [COUT] fp32 (may be null)
// Epilogues (EPI):
//   kEpiGelu    : pre = acc + bias -> pre_out (bf16), act_out = gelu(pre)
//   kEpiGeluRes : as kEpiGelu with act_out = x + gelu(pre) (CIN == COUT)
//   kEpiOut     : out_f32[b][w] = acc + bias (channel 0)
//   kEpiBwd     : gh = acc (+ res_in) -> gh_out (bf16, optional);
//                 gp_out = bf16(gh) * gelu'(pre_in) (bf16)
//   kEpiF32     : out_f32[b][w][o] = acc + bias, every channel, unrounded
//                 (the per-layer probe that checks the products)
// LDS rows are padded by 16 bytes so that 16 lanes reading 16 bytes from 16
// consecutive rows hit distinct banks.
template <int CIN, int COUT, int EPI>
__global__ __launch_bounds__(kThreads) void conv_kernel(ConvArgs a)
{
    constexpr int XS = CIN + 8;                 // padded row (bf16 elements)
    constexpr int NT = COUT / 16;               // output channel tiles
    constexpr int KC = CIN / 32;                // 32-channel K chunks per tap
    __shared__ __attribute__((aligned(16))) bf16 xs[(kMT + 4 * kMaxDil) * XS];
    __shared__ __attribute__((aligned(16))) bf16 ws[kTaps * COUT * XS];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int b = blockIdx.y;
    const int w0 = blockIdx.x * kMT;
    const int W = a.width;
    const int d = a.dil;
    const bf16 *x = static_cast<const bf16 *>(a.x) + (int64_t)b * W * CIN;

    // input rows w0-2d .. w0+kMT+2d-1 (zero outside the rod), 16 bytes per copy
    constexpr int CPR = CIN / 8;                // 16-byte chunks per row
    for (int i = tid; i < (kMT + 4 * d) * CPR; i += kThreads) {
        const int row = i / CPR, ch = (i % CPR) * 8;
        const int w = w0 - 2 * d + row;
        bf16 *dst = &xs[row * XS + ch];
        if (w >= 0 && w < W)
            copy16(dst, &x[(int64_t)w * CIN + ch]);
        else
            *reinterpret_cast<uint4 *>(dst) = make_uint4(0, 0, 0, 0);
    }
    const bf16 *wt = static_cast<const bf16 *>(a.w);
    for (int i = tid; i < kTaps * COUT * CPR; i += kThreads) {
        const int row = i / CPR, ch = (i % CPR) * 8;
        copy16(&ws[row * XS + ch], &wt[row * CIN + ch]);
    }
    __syncthreads();

    f32x4 acc[2][NT];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int r16 = lane & 15, g4 = lane >> 4;
#pragma unroll
    for (int k = 0; k < kTaps; ++k) {
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            bf16x8 af[2], bfr[NT];
#pragma unroll
            for (int m = 0; m < 2; ++m)
                af[m] = *reinterpret_cast<const bf16x8 *>(
                    &xs[(32 * wv + 16 * m + r16 + k * d) * XS + 32 * c + 8 * g4]);
#pragma unroll
            for (int n = 0; n < NT; ++n)
                bfr[n] = *reinterpret_cast<const bf16x8 *>(
                    &ws[(k * COUT + 16 * n + r16) * XS + 32 * c + 8 * g4]);
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[n], af[m], acc[m][n],
                                                                       0, 0, 0);
        }
    }

    // epilogue: the product is taken transposed (weights as the A operand),
    // so lane holds channels 16 n + 4 (lane / 16) + j of position
    // 32 wv + 16 m + lane % 16, four consecutive channels: one 8-byte access
    const int64_t rowbase = (int64_t)b * W;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int pl = 32 * wv + 16 * m + r16;              // position within the tile
        const int w = w0 + pl;
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int ch0 = 16 * n + 4 * g4;
            const int64_t o = (rowbase + w) * COUT + ch0;
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[j] = acc[m][n][j];
                if (a.bias) v[j] += a.bias[ch0 + j];
            }
            if constexpr (EPI == kEpiGelu || EPI == kEpiGeluRes) {
                bf16x4 pre, act, xres;
                if constexpr (EPI == kEpiGeluRes)
                    xres = *reinterpret_cast<const bf16x4 *>(&xs[(pl + 2 * d) * XS + ch0]);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    pre[j] = f2bf(v[j]);
                    float h = gelu(v[j]);
                    if constexpr (EPI == kEpiGeluRes) h += bf2f(xres[j]);
                    act[j] = f2bf(h);
                }
                if (a.pre_out) *reinterpret_cast<bf16x4 *>(&static_cast<bf16 *>(a.pre_out)[o]) = pre;
                *reinterpret_cast<bf16x4 *>(&static_cast<bf16 *>(a.act_out)[o]) = act;
            } else if constexpr (EPI == kEpiOut) {
                if (ch0 == 0) a.out_f32[rowbase + w] = v[0];
            } else if constexpr (EPI == kEpiF32) {
                *reinterpret_cast<float4 *>(&a.out_f32[o]) = float4{v[0], v[1], v[2], v[3]};
            } else {   // kEpiBwd
                bf16x4 gh, gp;
                const bf16x4 pre = *reinterpret_cast<const bf16x4 *>(
                    &static_cast<const bf16 *>(a.pre_in)[o]);
                bf16x4 res;
                if (a.res_in)
                    res = *reinterpret_cast<const bf16x4 *>(&static_cast<const bf16 *>(a.res_in)[o]);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float g = v[j];
                    if (a.res_in) g += bf2f(res[j]);
                    gh[j] = f2bf(g);
                    gp[j] = f2bf(bf2f(gh[j]) * gelu_grad(bf2f(pre[j])));
                }
                if (a.gh_out) *reinterpret_cast<bf16x4 *>(&static_cast<bf16 *>(a.gh_out)[o]) = gh;
                *reinterpret_cast<bf16x4 *>(&static_cast<bf16 *>(a.gp_out)[o]) = gp;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient dW[k][o][i] = sum_{b,w} g[b][w][o] x[b][w + (k - 2) d][i] and
// bias gradient db[o] = sum g[b][w][o].  One wave per tap (5 waves); each
// workgroup reduces a fixed range of 128-position segments into registers
// and writes its partial sums; wgrad_reduce adds the partials in order.
// The GEMM runs with M = output channels, N = input channels, K = positions,
// from LDS tiles stored transposed (positions contiguous): gT[o][p] and, per
// tap, xT[i][p] = x[p + (k - 2) d][i].
constexpr int kWP = 128;               // positions per segment
constexpr int kWS = kWP + 8;           // padded LDS row (bf16)

template <int CIN, int COUT>
__global__ __launch_bounds__(64 * kTaps) void wgrad_kernel(WgradArgs a)
{
    constexpr int MT = COUT / 16, NT = CIN / 16;
    __shared__ __attribute__((aligned(16))) bf16 gT[COUT * kWS];
    __shared__ __attribute__((aligned(16))) bf16 xT[kTaps * CIN * kWS];
    const int tid = threadIdx.x, lane = tid & 63;
    const int tap = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r16 = lane & 15, g4 = lane >> 4;
    const int W = a.width;
    const int segs_per_rod = W / kWP;
    const int64_t nseg = (int64_t)a.batch * segs_per_rod;
    const int64_t s_lo = nseg * blockIdx.x / gridDim.x;
    const int64_t s_hi = nseg * (blockIdx.x + 1) / gridDim.x;

    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dbias = 0.f;   // thread tid < COUT accumulates db[tid]

    const bf16 *gsrc = static_cast<const bf16 *>(a.g);
    const bf16 *xsrc = static_cast<const bf16 *>(a.x);
    for (int64_t sg = s_lo; sg < s_hi; ++sg) {
        const int64_t b = sg / segs_per_rod;
        const int p0 = (int)(sg % segs_per_rod) * kWP;
        __syncthreads();   // previous segment's tiles are no longer read
        // g tile, transposed: gT[o][p] = g[b][p0 + p][o]
        for (int i = tid; i < kWP * COUT; i += 64 * kTaps) {
            const int p = i / COUT, o = i % COUT;
            gT[o * kWS + p] = gsrc[((int64_t)b * W + p0 + p) * COUT + o];
        }
        // x tiles per tap, transposed and shifted: xT[k][i][p] = x[b][p0 + p + (k - 2) d][i]
        for (int i = tid; i < kTaps * kWP * CIN; i += 64 * kTaps) {
            const int k = i / (kWP * CIN), rem = i % (kWP * CIN);
            const int p = rem / CIN, ci = rem % CIN;
            const int w = p0 + p + (k - 2) * a.dil;
            xT[(k * CIN + ci) * kWS + p] =
                (w >= 0 && w < W) ? xsrc[((int64_t)b * W + w) * CIN + ci] : (bf16)0.0f;
        }
        __syncthreads();
        if (tid < COUT) {
            float sacc = 0.f;
            for (int p = 0; p < kWP; ++p) sacc += bf2f(gT[tid * kWS + p]);
            dbias += sacc;
        }
#pragma unroll
        for (int ks = 0; ks < kWP / 32; ++ks) {
            bf16x8 af[MT], bfr[NT];
#pragma unroll
            for (int m = 0; m < MT; ++m)
                af[m] = *reinterpret_cast<const bf16x8 *>(
                    &gT[(16 * m + r16) * kWS + 32 * ks + 8 * g4]);
#pragma unroll
            for (int n = 0; n < NT; ++n)
                bfr[n] = *reinterpret_cast<const bf16x8 *>(
                    &xT[(tap * CIN + 16 * n + r16) * kWS + 32 * ks + 8 * g4]);
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[m], bfr[n], acc[m][n],
                                                                       0, 0, 0);
        }
    }
    // partial sums: part[block][k][o][i] and part_db[block][o]
    float *part = a.part + (int64_t)blockIdx.x * (kTaps * COUT * CIN + COUT);
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int o = 16 * m + 4 * g4 + j, ci = 16 * n + r16;
                part[(tap * COUT + o) * CIN + ci] = acc[m][n][j];
            }
    if (tid < COUT) part[kTaps * COUT * CIN + tid] = dbias;
}

// Sum the workgroups' partials in workgroup order into the flat, unpadded
// gradient of one layer: dw[(k*co + o)*ci + i] then db[o].
__global__ void wgrad_reduce_kernel(const float *part, int nblocks, int cinp, int coutp, int ci,
                                    int co, float *grad)
{
    const int64_t nw = (int64_t)kTaps * co * ci;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nw + co) return;
    int64_t src;
    if (e < nw) {
        const int k = (int)(e / ((int64_t)co * ci));
        const int o = (int)((e / ci) % co), i = (int)(e % ci);
        src = ((int64_t)k * coutp + o) * cinp + i;
    } else {
        src = (int64_t)kTaps * coutp * cinp + (e - nw);
    }
    const int64_t stride = (int64_t)kTaps * coutp * cinp + coutp;
    float s = 0.f;
    for (int bk = 0; bk < nblocks; ++bk) s += part[(int64_t)bk * stride + src];
    grad[e] = s;
}

// ---------------------------------------------------------------------------
// Features of one rod (one workgroup per rod): the second difference
// D_i = u_{i-1} - 2u_i + u_{i+1} (zero walls) scaled by its RMS s, and the
// mesh ratio mapped to [-1, 1] over [0.5, 2]; other channels zero.
__global__ __launch_bounds__(256) void features_kernel(const float *u, const float *r, int W,
                                                       bf16 *x, float *scale)
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
    const float sc = sqrtf(red[0] / W) + 1e-30f;
    if (tid == 0) scale[b] = sc;
    const float rn = (r[b] - 1.25f) / 0.75f;
    bf16 *xb = x + (int64_t)b * W * 32;
    for (int i = tid; i < W; i += 256) {
        const float um = i > 0 ? ub[i - 1] : 0.f, up = i < W - 1 ? ub[i + 1] : 0.f;
        const float d = (um - ub[i]) + (up - ub[i]);
        bf16 *row = xb + (int64_t)i * 32;
        row[0] = f2bf(d / sc);
        row[1] = f2bf(rn);
        for (int c = 2; c < 32; ++c) row[c] = f2bf(0.f);
    }
}

// Loss on the normalised increment t = (u64 - u) / (64 r s), and its
// gradient 2 (out - t) / M into channel 0 of a 32-channel bf16 tensor.
// Per-block partial sums of the squared error go to part (reduced in order).
__global__ __launch_bounds__(256) void loss_kernel(const float *out, const float *u,
                                                   const float *u64, const float *r,
                                                   const float *scale, int W, int64_t M,
                                                   bf16 *g, float *part)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    __shared__ float red[256];
    float e2 = 0.f;
    if (i < M) {
        const int64_t b = i / W;
        const float t = (u64[i] - u[i]) / (64.0f * r[b] * scale[b]);
        const float d = out[i] - t;
        e2 = d * d;
        bf16 *gr = g + i * 32;
        gr[0] = f2bf(2.0f * d / (float)M);
        for (int c = 1; c < 32; ++c) gr[c] = f2bf(0.f);
    }
    red[threadIdx.x] = e2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_in_order_kernel(const float *part, int n, float scale, float *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float s = 0.f;
        for (int i = 0; i < n; ++i) s += part[i];
        out[0] = s * scale;
    }
}

// u_next = u + 64 r s out (the jump), optionally to a separate buffer
__global__ void jump_kernel(const float *u, const float *out, const float *r,
                            const float *scale, int W, int64_t M, float *u_next)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int64_t b = i / W;
    u_next[i] = u[i] + 64.0f * r[b] * scale[b] * out[i];
}

// Widening and narrowing copies between the network's FP32 state and the
// FP64 state of the GE sweep.
__global__ void widen_kernel(const float *u, double *d, int64_t M)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) d[i] = (double)u[i];
}
__global__ void narrow_kernel(const double *d, float *u, int64_t M)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) u[i] = (float)d[i];
}

// Re-check of one jump, one workgroup per rod: rel-L2 distance of the
// network's result a (FP32) from the GE result b (FP64), in FP64.  A rod is
// flagged when the distance exceeds tol or is not a number; the per-rod
// counters of accepted and rejected windows are advanced.
__global__ __launch_bounds__(256) void recheck_kernel(const float *a, const double *b, int W,
                                                      double tol, int *flag, double *err,
                                                      int *acc, int *fb)
{
    const int rod = blockIdx.x, tid = threadIdx.x;
    const float *ar = a + (int64_t)rod * W;
    const double *br = b + (int64_t)rod * W;
    __shared__ double rd[256], rn[256];
    double d2 = 0.0, n2 = 0.0;
    for (int i = tid; i < W; i += 256) {
        const double d = (double)ar[i] - br[i];
        d2 += d * d;
        n2 += br[i] * br[i];
    }
    rd[tid] = d2;
    rn[tid] = n2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            rd[tid] += rd[tid + s];
            rn[tid] += rn[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double rel = rn[0] > 0.0 ? sqrt(rd[0] / rn[0]) : (rd[0] > 0.0 ? INFINITY : 0.0);
        const int f = !(rel <= tol);
        flag[rod] = f;
        if (err) err[rod] = rel;
        if (acc) acc[rod] += 1 - f;
        if (fb) fb[rod] += f;
    }
}

// Number of flagged rods, summed in order by one thread.
__global__ void count_kernel(const int *flag, int n, int *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int c = 0;
        for (int i = 0; i < n; ++i) c += flag[i];
        out[0] = c;
    }
}

// u = flagged ? saved : network result, rod by rod.
__global__ void select_kernel(float *u, const float *unn, const float *save, const int *flag,
                              int W, int64_t M)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    u[i] = flag[i / W] ? save[i] : unn[i];
}

// Flagged rods take the GE result.
__global__ void take_ge_kernel(float *u, const double *ge, const int *flag, int W, int64_t M)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    if (flag[i / W]) u[i] = (float)ge[i];
}

// Adam on the FP32 master parameters.
__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Master weights of one layer (FP32 [5][co][ci]) -> padded bf16 copies:
// forward B layout wf[k][o][i] (o < cop, i < cip) and input-gradient layout
// wd[k][i][o] = W[4 - k][o][i] (i < cip as output, o < cop_in as input).
__global__ void pack_kernel(const float *wm, const float *bm, int ci, int co, int cip, int cop,
                            int cod, bf16 *wf, float *bf, bf16 *wd)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nf = (int64_t)kTaps * cop * cip;
    if (idx < nf) {
        const int k = (int)(idx / (cop * cip)), rem = (int)(idx % (cop * cip));
        const int o = rem / cip, i = rem % cip;
        wf[idx] = f2bf((o < co && i < ci) ? wm[(k * co + o) * ci + i] : 0.f);
    }
    if (wd) {
        const int64_t nd = (int64_t)kTaps * cip * cod;
        if (idx < nd) {
            const int k = (int)(idx / (cip * cod)), rem = (int)(idx % (cip * cod));
            const int i = rem / cod, o = rem % cod;
            wd[idx] = f2bf((o < co && i < ci) ? wm[((kTaps - 1 - k) * co + o) * ci + i] : 0.f);
        }
    }
    if (idx < cop) bf[idx] = idx < co ? bm[idx] : 0.f;
}

}  // namespace

hipError_t launch_conv(int cin, int cout, int epi, const ConvArgs &a, int batch, hipStream_t s)
{
    if (a.dil < 1 || a.dil > kMaxDil) return hipErrorInvalidValue;
    const dim3 grid(a.width / kMT, batch);
#define GE_CONV(CI, CO, E) \
    if (cin == CI && cout == CO && epi == E) { \
        hipLaunchKernelGGL((conv_kernel<CI, CO, E>), grid, dim3(kThreads), 0, s, a); \
        return hipGetLastError(); \
    }
    GE_CONV(32, 64, kEpiGelu)
    GE_CONV(64, 64, kEpiGeluRes)
    GE_CONV(64, 16, kEpiOut)
    GE_CONV(32, 64, kEpiBwd)
    GE_CONV(64, 64, kEpiBwd)
    GE_CONV(32, 64, kEpiF32)
    GE_CONV(64, 64, kEpiF32)
    GE_CONV(64, 16, kEpiF32)
#undef GE_CONV
    return hipErrorInvalidValue;
}

hipError_t launch_wgrad(int cin, int cout, const WgradArgs &a, int blocks, hipStream_t s)
{
    if (a.dil < 1 || a.dil > kMaxDil) return hipErrorInvalidValue;
#define GE_WG(CI, CO) \
    if (cin == CI && cout == CO) { \
        hipLaunchKernelGGL((wgrad_kernel<CI, CO>), dim3(blocks), dim3(64 * kTaps), 0, s, a); \
        return hipGetLastError(); \
    }
    GE_WG(32, 64)
    GE_WG(64, 64)
    GE_WG(64, 32)
#undef GE_WG
    return hipErrorInvalidValue;
}

hipError_t launch_wgrad_reduce(const float *part, int nblocks, int cinp, int coutp, int ci,
                               int co, float *grad, hipStream_t s)
{
    const int64_t n = (int64_t)kTaps * co * ci + co;
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       part, nblocks, cinp, coutp, ci, co, grad);
    return hipGetLastError();
}

hipError_t launch_features(const float *u, const float *r, int W, int batch, void *x,
                           float *scale, hipStream_t s)
{
    hipLaunchKernelGGL(features_kernel, dim3(batch), dim3(256), 0, s, u, r, W,
                       static_cast<bf16 *>(x), scale);
    return hipGetLastError();
}

hipError_t launch_loss(const float *out, const float *u, const float *u64, const float *r,
                       const float *scale, int W, int batch, void *g, float *part,
                       float *loss, hipStream_t s)
{
    const int64_t M = (int64_t)W * batch;
    const int nb = (int)((M + 255) / 256);
    hipLaunchKernelGGL(loss_kernel, dim3(nb), dim3(256), 0, s, out, u, u64, r, scale, W, M,
                       static_cast<bf16 *>(g), part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !loss) return e;
    hipLaunchKernelGGL(sum_in_order_kernel, dim3(1), dim3(64), 0, s, part, nb, 1.0f / (float)M,
                       loss);
    return hipGetLastError();
}

int loss_blocks(int W, int batch) { return (int)(((int64_t)W * batch + 255) / 256); }

hipError_t launch_jump(const float *u, const float *out, const float *r, const float *scale,
                       int W, int batch, float *u_next, hipStream_t s)
{
    const int64_t M = (int64_t)W * batch;
    hipLaunchKernelGGL(jump_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, u, out,
                       r, scale, W, M, u_next);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                       float b1, float b2, float eps, int step, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m,
                       v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_pack(const float *wm, const float *bm, int ci, int co, int cip, int cop,
                       int cod, void *wf, float *bf, void *wd, hipStream_t s)
{
    const int64_t n = (int64_t)kTaps * (cop > cod ? cop : cod) * cip + cop;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, wm, bm,
                       ci, co, cip, cop, cod, static_cast<bf16 *>(wf), bf,
                       static_cast<bf16 *>(wd));
    return hipGetLastError();
}

namespace {
inline dim3 grid_for(int64_t M) { return dim3((unsigned)((M + 255) / 256)); }
}  // namespace

hipError_t launch_widen(const float *u, double *d, int64_t M, hipStream_t s)
{
    hipLaunchKernelGGL(widen_kernel, grid_for(M), dim3(256), 0, s, u, d, M);
    return hipGetLastError();
}

hipError_t launch_narrow(const double *d, float *u, int64_t M, hipStream_t s)
{
    hipLaunchKernelGGL(narrow_kernel, grid_for(M), dim3(256), 0, s, d, u, M);
    return hipGetLastError();
}

hipError_t launch_recheck(const float *a, const double *b, int W, int batch, double tol, int *flag,
                          double *err, int *acc, int *fb, int *count, hipStream_t s)
{
    hipLaunchKernelGGL(recheck_kernel, dim3(batch), dim3(256), 0, s, a, b, W, tol, flag, err, acc,
                       fb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(count_kernel, dim3(1), dim3(64), 0, s, flag, batch, count);
    return hipGetLastError();
}

hipError_t launch_select(float *u, const float *unn, const float *save, const int *flag, int W,
                         int batch, hipStream_t s)
{
    const int64_t M = (int64_t)W * batch;
    hipLaunchKernelGGL(select_kernel, grid_for(M), dim3(256), 0, s, u, unn, save, flag, W, M);
    return hipGetLastError();
}

hipError_t launch_take_ge(float *u, const double *ge, const int *flag, int W, int batch,
                          hipStream_t s)
{
    const int64_t M = (int64_t)W * batch;
    hipLaunchKernelGGL(take_ge_kernel, grid_for(M), dim3(256), 0, s, u, ge, flag, W, M);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace ge
