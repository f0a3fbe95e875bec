// C ABI of the learned 64-level propagator: a network object that owns its
// parameters, Adam state and activation buffers (allocated once, at
// creation), and the sequences of kernels for a forward pass, a jump and a
// training step.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "ge.h"
#include "ge_internal.h"
#include "ge_nn.h"

namespace {

using namespace ge::nn;

struct Layer {
    int ci, co;      // real channels
    int cip, cop;    // padded forward channels (input, output)
    int cod;         // padded channels of the gradient entering the layer (its output)
    int64_t off;     // offset of W[5][co][ci] then b[co] in the flat parameter array
    int dil;         // tap spacing: the taps read offsets (k - 2) dil
};

// flat layout: for each layer in order, W[5][co][ci] then b[co]
constexpr int64_t kOff1 = 5 * 64 * 2 + 64;
constexpr int64_t kOffH = 5 * 64 * 64 + 64;
// Tap spacings 1, 2, 4, 8, 16, 1: a receptive field of +-64 points, about
// the reach of 64 levels of the sweep.
const Layer kLayers[6] = {
    {2, 64, 32, 64, 64, 0, 1},
    {64, 64, 64, 64, 64, kOff1, 2},
    {64, 64, 64, 64, 64, kOff1 + kOffH, 4},
    {64, 64, 64, 64, 64, kOff1 + 2 * kOffH, 8},
    {64, 64, 64, 64, 64, kOff1 + 3 * kOffH, 16},
    {64, 1, 64, 16, 32, kOff1 + 4 * kOffH, 1},
};

int64_t layer_params(const Layer &l) { return 5LL * l.co * l.ci + l.co; }

int64_t total_params()
{
    int64_t n = 0;
    for (const Layer &l : kLayers) n += layer_params(l);
    return n;
}

ge_status fail(ge_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
ge_status fail(ge_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    ge::vset_error(st, fmt, ap);
    va_end(ap);
    return st;
}

// splitmix64 stream and Box-Muller normals for the seeded initialisation
struct Rng {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal()
    {
        const double u1 = uniform(), u2 = uniform();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    }
};

}  // namespace

struct ge_nn_s {
    int width, max_batch;
    int64_t nparam;
    float *p, *g, *m, *v;           // FP32 master parameters, gradient, Adam moments
    void *wf[6], *wd[6];            // packed bf16 weights (forward, input-gradient)
    float *bf[6];                   // padded biases
    void *x;                        // bf16 [B][W][32] features
    void *pre[5], *h[5];            // bf16 [B][W][64]
    float *out, *scale, *loss_part, *wpart;
    void *gl;                       // bf16 [B][W][32] loss gradient
    void *gh, *gp[2];               // bf16 [B][W][64]
    float *save, *unn;              // re-checked stepping: window start, network result
    double *gev;                    // re-checked stepping: GE state (FP64)
    int *flag, *count;              // per-rod rejection flags and their number
    int *h_count;                   // pinned host copy of the number
    int step;
    std::vector<void *> allocs;
};

namespace {

void free_nn(ge_nn_s *n)
{
    if (!n) return;
    for (void *p : n->allocs) (void)hipFree(p);
    if (n->h_count) (void)hipHostFree(n->h_count);
    delete n;
}

template <typename T>
bool dalloc(ge_nn_s *n, T **p, size_t bytes)
{
    void *q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) return false;
    n->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return true;
}

hipError_t pack_all(ge_nn_s *n, hipStream_t s)
{
    for (int l = 0; l < 6; ++l) {
        const Layer &L = kLayers[l];
        const float *wm = n->p + L.off;
        const float *bm = wm + 5LL * L.co * L.ci;
        hipError_t e = launch_pack(wm, bm, L.ci, L.co, L.cip, L.cop, L.cod, n->wf[l], n->bf[l],
                                   l > 0 ? n->wd[l] : nullptr, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

ge_status check_io(ge_nn_s *n, int batch, const char *what)
{
    if (!n) return fail(GE_ERR_INVALID, "%s: network is NULL", what);
    if (batch < 1 || batch > n->max_batch)
        return fail(GE_ERR_INVALID, "%s: batch %d outside [1, %d]", what, batch, n->max_batch);
    return GE_OK;
}

// train: keep the pre-activations for the backward pass
hipError_t forward(ge_nn_s *n, const float *u, const float *r, int batch, hipStream_t s,
                   bool train)
{
    const int W = n->width;
    hipError_t e = launch_features(u, r, W, batch, n->x, n->scale, s);
    if (e != hipSuccess) return e;
    for (int l = 0; l < 6; ++l) {
        const Layer &L = kLayers[l];
        ConvArgs a{};
        a.x = l == 0 ? n->x : n->h[l - 1];
        a.w = n->wf[l];
        a.bias = n->bf[l];
        a.width = W;
        a.dil = L.dil;
        if (l < 5) {
            a.pre_out = train ? n->pre[l] : nullptr;
            a.act_out = n->h[l];
        } else {
            a.out_f32 = n->out;
        }
        const int epi = l == 0 ? kEpiGelu : (l < 5 ? kEpiGeluRes : kEpiOut);
        e = launch_conv(L.cip, L.cop, epi, a, batch, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// u_next = u + 64 r s out by the six-layer fused kernel (u_next must not
// overlap u)
hipError_t fused_jump(ge_nn_s *n, const float *u, const float *r, int batch, float *u_next,
                      hipStream_t s)
{
    FusedArgs a{};
    a.u = u;
    a.r = r;
    a.scale = n->scale;
    a.width = n->width;
    for (int l = 0; l < 6; ++l) {
        a.w[l] = n->wf[l];
        a.bias[l] = n->bf[l];
        a.dil[l] = kLayers[l].dil;
    }
    a.u_next = u_next;
    return launch_jump_fused(a, batch, s);
}

int wgrad_blocks(ge_nn_s *n, int batch)
{
    const int64_t nseg = (int64_t)batch * (n->width / 128);
    return (int)std::min<int64_t>(kMaxWgradBlocks, nseg);
}

// loss gradient already in n->gl; fills n->g (flat parameter gradient)
hipError_t backward(ge_nn_s *n, int batch, hipStream_t s)
{
    const int W = n->width;
    const int nb = wgrad_blocks(n, batch);
    // layer 6: weight gradient from h5 and the loss gradient; input gradient
    {
        const Layer &L = kLayers[5];
        WgradArgs wa{n->h[4], n->gl, n->wpart, W, batch, L.dil};
        hipError_t e = launch_wgrad(64, 32, wa, nb, s);
        if (e == hipSuccess) e = launch_wgrad_reduce(n->wpart, nb, 64, 32, L.ci, L.co, n->g + L.off, s);
        if (e != hipSuccess) return e;
        ConvArgs a{};
        a.x = n->gl;
        a.w = n->wd[5];
        a.width = W;
        a.dil = L.dil;
        a.res_in = nullptr;
        a.pre_in = n->pre[4];
        a.gh_out = n->gh;
        a.gp_out = n->gp[0];
        e = launch_conv(32, 64, kEpiBwd, a, batch, s);
        if (e != hipSuccess) return e;
    }
    int cur = 0;
    for (int l = 4; l >= 1; --l) {
        const Layer &L = kLayers[l];
        WgradArgs wa{n->h[l - 1], n->gp[cur], n->wpart, W, batch, L.dil};
        hipError_t e = launch_wgrad(64, 64, wa, nb, s);
        if (e == hipSuccess) e = launch_wgrad_reduce(n->wpart, nb, 64, 64, L.ci, L.co, n->g + L.off, s);
        if (e != hipSuccess) return e;
        ConvArgs a{};
        a.x = n->gp[cur];
        a.w = n->wd[l];
        a.width = W;
        a.dil = L.dil;
        a.res_in = n->gh;             // residual path of layer l (read and rewritten in place)
        a.pre_in = n->pre[l - 1];
        a.gh_out = n->gh;
        a.gp_out = n->gp[1 - cur];
        e = launch_conv(64, 64, kEpiBwd, a, batch, s);
        if (e != hipSuccess) return e;
        cur = 1 - cur;
    }
    const Layer &L = kLayers[0];
    WgradArgs wa{n->x, n->gp[cur], n->wpart, W, batch, L.dil};
    hipError_t e = launch_wgrad(32, 64, wa, nb, s);
    if (e == hipSuccess) e = launch_wgrad_reduce(n->wpart, nb, 32, 64, L.ci, L.co, n->g + L.off, s);
    return e;
}

}  // namespace

extern "C" {

int64_t ge_nn_param_count(void) { return total_params(); }

ge_status ge_nn_create(ge_nn_t *out, int32_t width, int32_t max_batch, uint64_t seed)
{
    if (!out) return fail(GE_ERR_INVALID, "ge_nn_create: out is NULL");
    *out = nullptr;
    if (width < 128 || width % 128 != 0 || width > (1 << 20))
        return fail(GE_ERR_INVALID, "ge_nn_create: width %d must be a positive multiple of 128",
                    width);
    if (max_batch < 1 || (int64_t)max_batch * width > (1LL << 26))
        return fail(GE_ERR_INVALID, "ge_nn_create: max_batch %d out of range", max_batch);
    ge_nn_s *n = new (std::nothrow) ge_nn_s();
    if (!n) return fail(GE_ERR_NOMEM, "ge_nn_create: out of host memory");
    n->width = width;
    n->max_batch = max_batch;
    n->nparam = total_params();
    const size_t M = (size_t)max_batch * width;
    bool ok = dalloc(n, &n->p, n->nparam * 4) && dalloc(n, &n->g, n->nparam * 4) &&
              dalloc(n, &n->m, n->nparam * 4) && dalloc(n, &n->v, n->nparam * 4) &&
              dalloc(n, &n->x, M * 32 * 2) && dalloc(n, &n->out, M * 4) &&
              dalloc(n, &n->scale, (size_t)max_batch * 4) &&
              dalloc(n, &n->loss_part, ((M + 255) / 256 + 1) * 4) &&
              dalloc(n, &n->wpart, (size_t)kMaxWgradBlocks * (5 * 64 * 64 + 64) * 4) &&
              dalloc(n, &n->gl, M * 32 * 2) && dalloc(n, &n->gh, M * 64 * 2) &&
              dalloc(n, &n->gp[0], M * 64 * 2) && dalloc(n, &n->gp[1], M * 64 * 2);
    for (int l = 0; ok && l < 5; ++l)
        ok = dalloc(n, &n->pre[l], M * 64 * 2) && dalloc(n, &n->h[l], M * 64 * 2);
    ok = ok && dalloc(n, &n->save, M * 4) && dalloc(n, &n->unn, M * 4) &&
         dalloc(n, &n->gev, M * 8) && dalloc(n, &n->flag, (size_t)max_batch * 4) &&
         dalloc(n, &n->count, 256);
    ok = ok && hipHostMalloc((void **)&n->h_count, sizeof(int), hipHostMallocDefault) == hipSuccess;
    for (int l = 0; ok && l < 6; ++l) {
        const Layer &L = kLayers[l];
        ok = dalloc(n, &n->wf[l], 5LL * L.cop * L.cip * 2) && dalloc(n, &n->bf[l], L.cop * 4);
        if (ok && l > 0) ok = dalloc(n, &n->wd[l], 5LL * L.cip * L.cod * 2);
    }
    if (!ok) {
        free_nn(n);
        return fail(GE_ERR_NOMEM, "ge_nn_create: device buffers for batch %d x width %d",
                    max_batch, width);
    }
    // seeded He initialisation (the last layer starts small), zero biases
    std::vector<float> h(n->nparam, 0.f);
    Rng rng{seed};
    for (int l = 0; l < 6; ++l) {
        const Layer &L = kLayers[l];
        double sd = std::sqrt(2.0 / (5.0 * L.ci));
        if (l == 5) sd *= 0.1;
        for (int64_t i = 0; i < 5LL * L.co * L.ci; ++i) h[L.off + i] = (float)(rng.normal() * sd);
    }
    hipError_t e = hipMemcpy(n->p, h.data(), n->nparam * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(n->m, 0, n->nparam * 4);
    if (e == hipSuccess) e = hipMemset(n->v, 0, n->nparam * 4);
    if (e == hipSuccess) e = pack_all(n, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_nn(n);
        return fail(GE_ERR_HIP, "ge_nn_create: %s", hipGetErrorString(e));
    }
    *out = n;
    return GE_OK;
}

void ge_nn_destroy(ge_nn_t n) { free_nn(n); }

ge_status ge_nn_set_params(ge_nn_t n, const float *host, int64_t count)
{
    if (!n || !host) return fail(GE_ERR_INVALID, "ge_nn_set_params: NULL argument");
    if (count != n->nparam)
        return fail(GE_ERR_INVALID, "ge_nn_set_params: %lld values, need %lld", (long long)count,
                    (long long)n->nparam);
    hipError_t e = hipMemcpy(n->p, host, count * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(n->m, 0, count * 4);
    if (e == hipSuccess) e = hipMemset(n->v, 0, count * 4);
    if (e == hipSuccess) e = pack_all(n, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    n->step = 0;
    return e == hipSuccess ? GE_OK : fail(GE_ERR_HIP, "ge_nn_set_params: %s", hipGetErrorString(e));
}

ge_status ge_nn_get_params(ge_nn_t n, float *host, int64_t count)
{
    if (!n || !host) return fail(GE_ERR_INVALID, "ge_nn_get_params: NULL argument");
    if (count != n->nparam)
        return fail(GE_ERR_INVALID, "ge_nn_get_params: %lld values, need %lld", (long long)count,
                    (long long)n->nparam);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(host, n->p, count * 4, hipMemcpyDeviceToHost);
    return e == hipSuccess ? GE_OK : fail(GE_ERR_HIP, "ge_nn_get_params: %s", hipGetErrorString(e));
}

ge_status ge_nn_forward(ge_nn_t n, const float *u, const float *r, int32_t batch, float *out,
                        float *scale, void *stream)
{
    ge_status st = check_io(n, batch, "ge_nn_forward");
    if (st != GE_OK) return st;
    if (!u || !r) return fail(GE_ERR_INVALID, "ge_nn_forward: u and r must be given");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = forward(n, u, r, batch, s, false);
    const size_t M = (size_t)batch * n->width;
    if (e == hipSuccess && out) e = hipMemcpyAsync(out, n->out, M * 4, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && scale)
        e = hipMemcpyAsync(scale, n->scale, (size_t)batch * 4, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? GE_OK : fail(GE_ERR_HIP, "ge_nn_forward: %s", hipGetErrorString(e));
}

ge_status ge_nn_jump(ge_nn_t n, const float *u, const float *r, int32_t batch, float *u_next,
                     void *stream)
{
    ge_status st = check_io(n, batch, "ge_nn_jump");
    if (st != GE_OK) return st;
    if (!u || !r || !u_next) return fail(GE_ERR_INVALID, "ge_nn_jump: NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t M = (size_t)batch * n->width;
    // the fused kernel reads neighbouring tiles' points: never in place
    float *dst = u_next == u ? n->unn : u_next;
    hipError_t e = fused_jump(n, u, r, batch, dst, s);
    if (e == hipSuccess && dst != u_next)
        e = hipMemcpyAsync(u_next, dst, M * 4, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? GE_OK : fail(GE_ERR_HIP, "ge_nn_jump: %s", hipGetErrorString(e));
}

ge_status ge_nn_grads(ge_nn_t n, const float *u, const float *u64, const float *r, int32_t batch,
                      float *loss, void *stream)
{
    ge_status st = check_io(n, batch, "ge_nn_grads");
    if (st != GE_OK) return st;
    if (!u || !u64 || !r) return fail(GE_ERR_INVALID, "ge_nn_grads: NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = forward(n, u, r, batch, s, true);
    if (e == hipSuccess)
        e = launch_loss(n->out, u, u64, r, n->scale, n->width, batch, n->gl, n->loss_part, loss, s);
    if (e == hipSuccess) e = backward(n, batch, s);
    return e == hipSuccess ? GE_OK : fail(GE_ERR_HIP, "ge_nn_grads: %s", hipGetErrorString(e));
}

ge_status ge_nn_gradient(ge_nn_t n, float *grad, void *stream)
{
    if (!n || !grad) return fail(GE_ERR_INVALID, "ge_nn_gradient: NULL argument");
    hipError_t e = hipMemcpyAsync(grad, n->g, n->nparam * 4, hipMemcpyDeviceToDevice,
                                  static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GE_OK : fail(GE_ERR_HIP, "ge_nn_gradient: %s", hipGetErrorString(e));
}

ge_status ge_nn_train_step(ge_nn_t n, const float *u, const float *u64, const float *r,
                           int32_t batch, float lr, float *loss, void *stream)
{
    if (!(lr > 0.f) || !std::isfinite(lr))
        return fail(GE_ERR_INVALID, "ge_nn_train_step: learning rate must be positive");
    ge_status st = ge_nn_grads(n, u, u64, r, batch, loss, stream);
    if (st != GE_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    n->step += 1;
    hipError_t e = launch_adam(n->p, n->g, n->m, n->v, n->nparam, lr, 0.9f, 0.999f, 1e-8f,
                               n->step, s);
    if (e == hipSuccess) e = pack_all(n, s);
    return e == hipSuccess ? GE_OK : fail(GE_ERR_HIP, "ge_nn_train_step: %s", hipGetErrorString(e));
}

ge_status ge_nn_layer_shape(int32_t layer, int32_t *ci, int32_t *co, int32_t *cip,
                            int32_t *cop, int32_t *cod, int32_t *dil)
{
    if (layer < 1 || layer > 6)
        return fail(GE_ERR_INVALID, "ge_nn_layer_shape: layer %d outside 1..6", layer);
    const Layer &L = kLayers[layer - 1];
    if (ci) *ci = L.ci;
    if (co) *co = L.co;
    if (cip) *cip = L.cip;
    if (cop) *cop = L.cop;
    if (cod) *cod = L.cod;
    if (dil) *dil = L.dil;
    return GE_OK;
}

ge_status ge_nn_layer_probe(ge_nn_t n, int32_t layer, int32_t op, const void *x, const void *g,
                            int32_t batch, float *out, void *stream)
{
    ge_status st = check_io(n, batch, "ge_nn_layer_probe");
    if (st != GE_OK) return st;
    if (layer < 1 || layer > 6)
        return fail(GE_ERR_INVALID, "ge_nn_layer_probe: layer %d outside 1..6", layer);
    if (!out) return fail(GE_ERR_INVALID, "ge_nn_layer_probe: out is NULL");
    const int l = layer - 1;
    const Layer &L = kLayers[l];
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (op == 0 || op == 1) {
        if (op == 0 ? !x : !g) return fail(GE_ERR_INVALID, "ge_nn_layer_probe: input is NULL");
        if (op == 1 && l == 0)
            return fail(GE_ERR_INVALID, "ge_nn_layer_probe: layer 1 has no input gradient");
        ConvArgs a{};
        a.x = op == 0 ? x : g;
        a.w = op == 0 ? n->wf[l] : n->wd[l];
        a.bias = op == 0 ? n->bf[l] : nullptr;
        a.width = n->width;
        a.dil = L.dil;
        a.out_f32 = out;
        e = op == 0 ? launch_conv(L.cip, L.cop, kEpiF32, a, batch, s)
                    : launch_conv(L.cod, L.cip, kEpiF32, a, batch, s);
    } else if (op == 2) {
        if (!x || !g) return fail(GE_ERR_INVALID, "ge_nn_layer_probe: x and g must be given");
        const int nb = wgrad_blocks(n, batch);
        WgradArgs wa{x, g, n->wpart, n->width, batch, L.dil};
        e = launch_wgrad(L.cip, L.cod, wa, nb, s);
        if (e == hipSuccess) e = launch_wgrad_reduce(n->wpart, nb, L.cip, L.cod, L.ci, L.co, out, s);
    } else {
        return fail(GE_ERR_INVALID, "ge_nn_layer_probe: op %d is not 0, 1 or 2", op);
    }
    return e == hipSuccess ? GE_OK : fail(GE_ERR_HIP, "ge_nn_layer_probe: %s", hipGetErrorString(e));
}

ge_status ge_f32_to_f64(const float *x, double *y, int64_t n, void *stream)
{
    if (n < 0 || (n > 0 && (!x || !y))) return fail(GE_ERR_INVALID, "ge_f32_to_f64: bad arguments");
    if (n == 0) return GE_OK;
    hipError_t e = launch_widen(x, y, n, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GE_OK : fail(GE_ERR_HIP, "ge_f32_to_f64: %s", hipGetErrorString(e));
}

ge_status ge_f64_to_f32(const double *x, float *y, int64_t n, void *stream)
{
    if (n < 0 || (n > 0 && (!x || !y))) return fail(GE_ERR_INVALID, "ge_f64_to_f32: bad arguments");
    if (n == 0) return GE_OK;
    hipError_t e = launch_narrow(x, y, n, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GE_OK : fail(GE_ERR_HIP, "ge_f64_to_f32: %s", hipGetErrorString(e));
}

ge_status ge_nn_advance(ge_nn_t n, ge_batch_t ge, void *ge_ws, float *u, const float *r,
                        int32_t batch, int64_t step0, int32_t njumps, int32_t check, double tol,
                        int32_t *accepted, int32_t *fallbacks, double *last_err,
                        int64_t *n_fallback, void *stream)
{
    ge_status st = check_io(n, batch, "ge_nn_advance");
    if (st != GE_OK) return st;
    if (!u || !r || !ge || !ge_ws) return fail(GE_ERR_INVALID, "ge_nn_advance: NULL argument");
    if (njumps < 0 || check < 1 || step0 < 0 || !(tol >= 0.0))
        return fail(GE_ERR_INVALID, "ge_nn_advance: need njumps >= 0, check >= 1, step0 >= 0, tol >= 0");
    int64_t nrods = 0;
    const int64_t *rod_n = nullptr;
    int prec = -1;
    ge::batch_shape(ge, &nrods, &rod_n, &prec);
    if (nrods != batch || prec != GE_FP64)
        return fail(GE_ERR_INVALID, "ge_nn_advance: the GE plan must be FP64 with %d rods", batch);
    for (int64_t i = 0; i < nrods; ++i)
        if (rod_n[i] != n->width)
            return fail(GE_ERR_INVALID, "ge_nn_advance: GE rod %lld has %lld points, need %d",
                        (long long)i, (long long)rod_n[i], n->width);
    if (n_fallback) *n_fallback = 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int W = n->width;
    const int64_t M = (int64_t)W * batch;
    hipError_t e = hipSuccess;
    for (int32_t j0 = 0; j0 < njumps && e == hipSuccess; j0 += check) {
        const int nj = std::min(check, njumps - j0);
        const int64_t lev0 = step0 + 64LL * j0;
        e = hipMemcpyAsync(n->save, u, M * 4, hipMemcpyDeviceToDevice, s);
        // jumps ping-pong between u and unn (the fused kernel is never in place)
        float *cur = u, *spare = n->unn;
        for (int j = 0; j + 1 < nj && e == hipSuccess; ++j) {
            e = fused_jump(n, cur, r, batch, spare, s);
            std::swap(cur, spare);
        }
        // the window's last jump, by the network (into spare) and by 64 GE
        // levels from the same input
        if (e == hipSuccess) e = fused_jump(n, cur, r, batch, spare, s);
        if (e == hipSuccess) e = launch_widen(cur, n->gev, M, s);
        if (e != hipSuccess) break;
        st = ge_solve_batch(ge, n->gev, ge_ws, lev0 + 64LL * (nj - 1), 64, s);
        if (st != GE_OK) return st;
        e = launch_recheck(spare, n->gev, W, batch, tol, n->flag, last_err, accepted, fallbacks,
                           n->count, s);
        if (e == hipSuccess) e = launch_select(u, spare, n->save, n->flag, W, batch, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(n->h_count, n->count, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess || *n->h_count == 0) continue;
        // rejected rods restart the window from its first state and take it by GE
        if (n_fallback) *n_fallback += *n->h_count;
        e = launch_widen(u, n->gev, M, s);
        if (e != hipSuccess) break;
        st = ge_solve_batch(ge, n->gev, ge_ws, lev0, 64LL * nj, s);
        if (st != GE_OK) return st;
        e = launch_take_ge(u, n->gev, n->flag, W, batch, s);
    }
    return e == hipSuccess ? GE_OK : fail(GE_ERR_HIP, "ge_nn_advance: %s", hipGetErrorString(e));
}

}  // extern "C"
