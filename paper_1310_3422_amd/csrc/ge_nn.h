// Internal interface of the surrogate network kernels (ge_nn.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ge {
namespace nn {

enum Epi : int { kEpiGelu = 0, kEpiGeluRes = 1, kEpiOut = 2, kEpiBwd = 3, kEpiF32 = 4 };

struct ConvArgs {
    const void *x;        // bf16 [batch][width][cin]
    const void *w;        // bf16 [5][cout][cin]
    const float *bias;    // [cout] or null
    int width;            // points per rod, a multiple of 128
    int dil;              // tap spacing d: taps at offsets (k - 2) d, 1 <= d <= kMaxDil
    void *pre_out;        // bf16 [..][cout]  (kEpiGelu*; null: not stored)
    void *act_out;        // bf16 [..][cout]  (kEpiGelu*)
    float *out_f32;       // f32 [batch][width] (kEpiOut), [batch][width][cout] (kEpiF32)
    const void *res_in;   // bf16 [..][cout]  (kEpiBwd, or null)
    const void *pre_in;   // bf16 [..][cout]  (kEpiBwd)
    void *gh_out;         // bf16 [..][cout]  (kEpiBwd, or null)
    void *gp_out;         // bf16 [..][cout]  (kEpiBwd)
};

struct WgradArgs {
    const void *x;        // bf16 [batch][width][cin]
    const void *g;        // bf16 [batch][width][cout]
    float *part;          // per-workgroup partials
    int width;
    int batch;
    int dil;              // tap spacing of the layer
};

constexpr int kMaxWgradBlocks = 256;
constexpr int kMaxDil = 16;         // largest tap spacing of a layer

hipError_t launch_conv(int cin, int cout, int epi, const ConvArgs &a, int batch, hipStream_t s);
hipError_t launch_wgrad(int cin, int cout, const WgradArgs &a, int blocks, hipStream_t s);
hipError_t launch_wgrad_reduce(const float *part, int nblocks, int cinp, int coutp, int ci,
                               int co, float *grad, hipStream_t s);
hipError_t launch_features(const float *u, const float *r, int W, int batch, void *x,
                           float *scale, hipStream_t s);
hipError_t launch_loss(const float *out, const float *u, const float *u64, const float *r,
                       const float *scale, int W, int batch, void *g, float *part, float *loss,
                       hipStream_t s);
int loss_blocks(int W, int batch);
hipError_t launch_jump(const float *u, const float *out, const float *r, const float *scale,
                       int W, int batch, float *u_next, hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                       float b1, float b2, float eps, int step, hipStream_t s);
hipError_t launch_pack(const float *wm, const float *bm, int ci, int co, int cip, int cop,
                       int cod, void *wf, float *bf, void *wd, hipStream_t s);

// Six-layer jump in one kernel per tile (ge_nn_fused.hip): reads u, writes
// the per-rod scale and u_next = u + 64 r s out.
struct FusedArgs {
    const float *u;          // [batch][width]
    const float *r;          // [batch]
    float *scale;            // [batch], written
    int width;
    const void *w[6];        // packed forward weights of the six layers
    const float *bias[6];    // padded biases
    int dil[6];              // tap spacings of the six layers
    float *u_next;           // [batch][width]
};
hipError_t launch_jump_fused(const FusedArgs &a, int batch, hipStream_t s);

hipError_t launch_widen(const float *u, double *d, int64_t M, hipStream_t s);
hipError_t launch_narrow(const double *d, float *u, int64_t M, hipStream_t s);
hipError_t launch_recheck(const float *a, const double *b, int W, int batch, double tol, int *flag,
                          double *err, int *acc, int *fb, int *count, hipStream_t s);
hipError_t launch_select(float *u, const float *unn, const float *save, const int *flag, int W,
                         int batch, hipStream_t s);
hipError_t launch_take_ge(float *u, const double *ge, const int *flag, int W, int batch,
                          hipStream_t s);

}  // namespace nn
}  // namespace ge
