// C ABI of libge (declared in include/ge.h): argument validation, the choice
// of tiling and temporal depth, and the launch sequence of a run.
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "ge.h"
#include "ge_internal.h"
#include "ge_2d.h"
#include "ge_kernels.h"

namespace ge {

int64_t comp_offset(int64_t n) { return (n + 63) / 64 * 64; }

namespace {
thread_local std::string g_last_error;
}

ge_status vset_error(ge_status st, const char *fmt, va_list ap)
{
    char buf[512];
    vsnprintf(buf, sizeof buf, fmt, ap);
    g_last_error = buf;
    return st;
}

ge_status set_error(ge_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vset_error(st, fmt, ap);
    va_end(ap);
    return st;
}

const char *last_error_str() { return g_last_error.c_str(); }

bool status_alloc(StatusWords &w)
{
    w = StatusWords{};
    void *h = nullptr;
    if (hipHostMalloc(&h, kStatusWords * sizeof(int),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess || !h) {
        (void)hipGetLastError();
        return false;
    }
    void *d = nullptr;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess || !d) {
        (void)hipGetLastError();
        (void)hipHostFree(h);
        return false;
    }
    w.host = static_cast<int *>(h);
    w.dev = static_cast<int *>(d);
    for (int i = 0; i < kStatusWords; ++i) w.host[i] = 0;
    return true;
}

void status_free(StatusWords &w)
{
    if (!w.host) return;
    (void)hipDeviceSynchronize();
    (void)hipHostFree(w.host);
    w = StatusWords{};
}

bool status_take(StatusWords &w, int word)
{
    if (!w.host) return false;
    volatile int *h = w.host;
    if (h[word] == 0) return false;
    h[word] = 0;
    return true;
}

SchemeCoef scheme_coef(double r)
{
    SchemeCoef c;
    c.c1 = (r + r * r) / (1.0 + 2.0 * r);
    c.c2 = (r * r) / (1.0 + 2.0 * r);
    c.cs = r / (1.0 + r);
    return c;
}

}  // namespace ge

namespace {

ge_status fail(ge_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
ge_status fail(ge_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    ge::vset_error(st, fmt, ap);
    va_end(ap);
    return st;
}

ge_status hip_fail(hipError_t e, const char *what)
{
    return fail(GE_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int elem_bytes(int prec) { return prec == ge::kFP64 ? 8 : 4; }

// elements of one level buffer (the compensated pair stores two blocks)
int64_t state_elems(int prec, int64_t n)
{
    return prec == ge::kFP32C ? 2 * ge::comp_offset(n) : n;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Library defaults, measured on MI355X on rods of 2^24 points without a
// source and of 2^27 points with moving walls and a source.  At a few levels
// per launch the sweep streams HBM, and narrow per-lane rows (one or two
// 16-byte chunks) coalesce best; deep launches are issue-bound and want wide
// rows, few halo points and no workgroup barrier.  With a source the
// interior tiles hold two per-parity weight arrays besides the state, so
// the persistent schedule's prefetch registers cost more occupancy than the
// prefetch gains, and those rods stay on one workgroup per tile: FP64 at 28
// points per lane and 96 levels (238 registers, two waves per SIMD; 5.9e12
// updates/s against 5.5e12 at 16 points and three waves, the halo's share
// of the window falling from 13% to 7%; 32 points need more than the
// register file), FP32 at 32 (64 levels: 7.7e12 updates/s against 7.4e12
// at 16).
struct Choice {
    int tile, waves, depth;
};

Choice default_choice(int prec, int depth, bool src)
{
    if (prec == ge::kFP32C) {
        if (depth == 0) return {16, 4, 128};
        if (depth <= 4) return {4, 1, depth};
        return {depth <= 64 ? 8 : 16, 4, depth};
    }
    const bool f64 = prec == ge::kFP64;
    if (depth == 0) return src ? (f64 ? Choice{28, 1, 96} : Choice{32, 1, 64}) : Choice{32, 1, 96};
    if (depth <= 4) return {f64 ? 2 : 4, 1, depth};
    if (depth <= 8) return {(f64 || !src) ? (f64 ? 4 : 8) : 4, 1, depth};
    if (depth <= 16) return {f64 ? (src ? 4 : 8) : 16, 1, depth};
    if (src) return {f64 ? (depth <= 32 ? 16 : 28) : 32, 1, depth};
    if (depth <= 32) return {16, 1, depth};
    return {32, 1, depth};
}

// Whether the persistent schedule is the faster one for a single-wave tile:
// deep launches without a source, with rows of 32 points (FP64 also 16).
bool persistent_pays(int prec, int tile, int waves, int depth, bool src)
{
    return waves == 1 && !src && depth > 32 && prec != ge::kFP32C &&
           ge::persistent_supported(prec, tile) && (tile >= 32 || prec == ge::kFP64);
}

}  // namespace

struct ge_plan_s {
    int64_t n;
    double r;
    int prec;
    int tile;      // points per lane
    int waves;     // waves per workgroup
    int depth;     // levels per launch (multi-tile mode)
    int halo;      // window points each side of a tile's core
    int64_t window;
    int64_t core;
    int64_t ntiles;
    bool single;   // the whole rod fits one window: no halo, all levels per launch
    bool persistent;  // multi-tile launches by the persistent single-wave kernel
    int sdc;       // sub-domain width k >= 2 (the sub-domain scheme), or 0
    double g_left, g_right;
    const void *src_b;
    double c1, c2, cs, e1, e2, es, tau, h;
    ge::StatusWords status;   // word 0: a launch stored a NaN or infinite value
    bool launched;            // a kernel may hold the status pointer
    ge::SideStream side;      // wall kernel of split launches (side_state 1)
    int side_state;           // 1 created, else none
};

namespace {


// Fewest tiles at which a plan keeps a second stream for split launches
// (the split itself starts at 128 interior tiles per compute unit).
constexpr int64_t kSideStreamTiles = 128 * 64;

bool side_create(ge::SideStream &ss)
{
    bool ok = false;
    if (hipStreamCreateWithFlags(&ss.stream, hipStreamNonBlocking) == hipSuccess) {
        if (hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming) == hipSuccess) {
            if (hipEventCreateWithFlags(&ss.join, hipEventDisableTiming) == hipSuccess)
                ok = true;
            else
                (void)hipEventDestroy(ss.fork);
        }
        if (!ok) (void)hipStreamDestroy(ss.stream);
    }
    (void)hipGetLastError();
    return ok;
}

// The persistent form pays where one couple fills 32 FP64 registers per
// node pair (k = 16): two waves per SIMD, so the per-tile form leaves its
// loads exposed.  Measured there 2-9% faster; at k <= 8, or in FP32, the
// per-tile form is as fast or faster.
bool sdc_persistent_pays(int prec, int k) { return prec == ge::kFP64 && k == 16; }
constexpr int64_t kSdcPersistentMinTiles = 64;

// Halo, in sub-domain couples, for D levels: a wrong value at an open window
// edge moves at most k + 1 nodes per level, two more for the pair stencil.
int sdc_halo(int depth, int k) { return (depth * (k + 1) + 2 + 2 * k - 1) / (2 * k); }

// Levels per launch of the sub-domain scheme for a window of `waves` waves
// when the caller leaves the depth to the library.  The halo per side
// (about D/2 couples) does not depend on the window, so wider windows pay
// for deeper launches.  Measured on MI355X on rods of 2^24 - 1 points (960
// levels, k = 2..16, FP64 and FP32): single-wave windows peak at 20 levels
// (24 persistent), two waves at 24, four at 40, eight at 48 (64 for FP64
// with k = 16).
int sdc_default_depth(int prec, int k, int waves)
{
    const bool wide64 = prec == ge::kFP64 && k == 16;
    switch (waves) {
    case 1: return wide64 ? 24 : 20;
    case 2: return 24;
    case 4: return 40;
    default: return wide64 ? 64 : 48;
    }
}

// Waves per window when the caller leaves them to the library: the widest
// window measured fastest on 2^24 - 1 points (FP64 with k = 16: four waves
// at 40 levels, persistent, 4.7e12 updates/s against 3.7e12 single-wave;
// otherwise eight at 48 levels, per tile: FP64 k = 8 5.2e12 against 3.7e12,
// FP32 k = 16 9.1e12 against 6.0e12), as long as the rod gives that launch
// at least 8192 waves (4 per SIMD at two resident); shorter rods keep
// single-wave windows, whose many small tiles spread over the chip.
int sdc_default_waves(int prec, int k, int64_t nsdc, int depth_given)
{
    const int wide = (prec == ge::kFP64 && k == 16) ? 4 : 8;
    const int depth = depth_given ? depth_given : sdc_default_depth(prec, k, wide);
    const int64_t core = 64 * wide - 2 * (int64_t)sdc_halo(depth, k);
    if (core < 16)
        return 1;
    const int64_t tiles = (nsdc + core - 1) / core;
    return tiles * wide >= 8192 ? wide : 1;
}

ge_status plan_sdc(ge_plan_t *out, const ge_desc *d)
{
    const int prec = d->precision, k = d->k;
    if (!ge::sdc_supported(prec == ge::kFP32C ? ge::kFP64 : prec, k))
        return fail(GE_ERR_UNSUPPORTED, "ge_plan: sub-domains of %d nodes are not built (2, 4, 8, 16)",
                    k);
    if (prec == ge::kFP32C)
        return fail(GE_ERR_UNSUPPORTED, "ge_plan: the sub-domain scheme runs in FP64 or FP32");
    if (d->src_b)
        return fail(GE_ERR_UNSUPPORTED, "ge_plan: the sub-domain scheme takes no source");
    if ((d->n + 1) % (2 * (int64_t)k) != 0)
        return fail(GE_ERR_INVALID, "ge_plan: n + 1 = %lld is not a multiple of 2k = %d",
                    (long long)(d->n + 1), 2 * k);
    if (d->tile != 0 && d->tile != 2 * k)
        return fail(GE_ERR_INVALID, "ge_plan: the sub-domain scheme holds 2k = %d points per lane",
                    2 * k);
    if (d->waves != 0 && !ge::sdc_waves_supported(d->waves))
        return fail(GE_ERR_INVALID, "ge_plan: the sub-domain scheme runs windows of 1, 2, 4 or 8 waves");
    if (d->schedule < 0 || d->schedule > 2)
        return fail(GE_ERR_INVALID, "ge_plan: schedule = %d, need 0, 1 or 2", d->schedule);
    if (d->depth < 0)
        return fail(GE_ERR_INVALID, "ge_plan: depth = %d, need depth >= 1", d->depth);
    const bool auto_persistent = d->schedule == 0 && sdc_persistent_pays(prec, k);
    const int64_t nsdc = (d->n + 1) / (2 * k);
    const int waves = d->waves != 0 ? d->waves : sdc_default_waves(prec, k, nsdc, d->depth);
    int depth = d->depth;
    if (depth == 0) {
        depth = sdc_default_depth(prec, k, waves);
        // single-wave per-tile launches keep 20 levels (24 is the persistent one's)
        if (waves == 1 && !auto_persistent && d->schedule != 2) depth = 20;
    }
    if (d->schedule == 2 && depth > ge::kSdcMaxLevels)
        return fail(GE_ERR_INVALID,
                    "ge_plan: the persistent sub-domain form takes at most %d levels per launch",
                    ge::kSdcMaxLevels);
    const int halo = sdc_halo(depth, k);
    const int wsdc = 64 * waves;            // couples per window
    const bool single = nsdc <= wsdc;
    if (!single && wsdc - 2 * halo < 16)
        return fail(GE_ERR_INVALID,
                    "ge_plan: depth %d needs a halo of %d couples, too wide for %d-couple windows",
                    depth, halo, wsdc);
    ge_plan_s *p = new (std::nothrow) ge_plan_s();
    if (!p)
        return fail(GE_ERR_NOMEM, "ge_plan: out of host memory");
    p->n = d->n;
    p->r = d->r;
    p->prec = prec;
    p->sdc = k;
    p->tile = 2 * k;
    p->waves = waves;
    p->depth = depth;
    p->window = (int64_t)wsdc * 2 * k;
    p->g_left = d->g_left;
    p->g_right = d->g_right;
    p->src_b = nullptr;
    p->single = single;
    p->halo = single ? 0 : halo;          // in couples
    p->core = single ? nsdc : wsdc - 2 * halo;
    p->ntiles = (nsdc + p->core - 1) / p->core;
    p->persistent = !single && p->ntiles >= 3 &&
                    (d->schedule == 2 || (auto_persistent && p->ntiles >= kSdcPersistentMinTiles &&
                                          depth <= ge::kSdcMaxLevels));
    const double r = d->r;
    p->h = 1.0 / (double)(p->n + 1);
    p->tau = r * p->h * p->h;
    const ge::SchemeCoef sc = ge::scheme_coef(r);
    p->c1 = sc.c1;
    p->c2 = sc.c2;
    p->cs = sc.cs;
    p->e1 = (1.0 - r) / (1.0 + r);       // the sweep's own-value weight
    p->e2 = p->es = 0.0;
    (void)ge::status_alloc(p->status);
    *out = p;
    return GE_OK;
}

}  // namespace

extern "C" {

const char *ge_version(void) { return "0.1.0"; }

const char *ge_last_error(void) { return ge::last_error_str(); }

const char *ge_status_str(int status)
{
    switch (status) {
    case GE_OK: return "GE_OK";
    case GE_ERR_INVALID: return "GE_ERR_INVALID";
    case GE_ERR_NOMEM: return "GE_ERR_NOMEM";
    case GE_ERR_HIP: return "GE_ERR_HIP";
    case GE_ERR_UNSUPPORTED: return "GE_ERR_UNSUPPORTED";
    case GE_ERR_NONFINITE: return "GE_ERR_NONFINITE";
    case GE_ERR_SYNC: return "GE_ERR_SYNC";
    default: return "GE_ERR_UNKNOWN";
    }
}

int64_t ge_comp_offset(int64_t n) { return n < 0 ? -1 : ge::comp_offset(n); }

size_t ge_workspace_bytes(const ge_desc *d)
{
    if (!d || d->n < 1 || d->precision < GE_FP64 || d->precision > GE_FP32_COMP)
        return 0;
    return (size_t)state_elems(d->precision, d->n) * (size_t)elem_bytes(d->precision);
}

ge_status ge_plan(ge_plan_t *out, const ge_desc *d)
{
    if (!out)
        return fail(GE_ERR_INVALID, "ge_plan: out is NULL");
    *out = nullptr;
    if (!d)
        return fail(GE_ERR_INVALID, "ge_plan: desc is NULL");
    if (d->n < 1)
        return fail(GE_ERR_INVALID, "ge_plan: n = %lld, need n >= 1", (long long)d->n);
    if (d->precision < GE_FP64 || d->precision > GE_FP32_COMP)
        return fail(GE_ERR_INVALID, "ge_plan: unknown precision %d", d->precision);
    if (!std::isfinite(d->r) || !std::isfinite(d->g_left) || !std::isfinite(d->g_right))
        return fail(GE_ERR_NONFINITE, "ge_plan: r and the wall values must be finite");
    if (!(d->r > 0.0))
        return fail(GE_ERR_INVALID, "ge_plan: r = %g, need r > 0", d->r);
    if (d->src_b && !aligned16(d->src_b))
        return fail(GE_ERR_INVALID, "ge_plan: src_b must be 16-byte aligned");

    const int prec = d->precision;
    if (d->k < 0)
        return fail(GE_ERR_INVALID, "ge_plan: k = %d, need k >= 0", d->k);
    if (d->k >= 2)
        return plan_sdc(out, d);
    int tile = d->tile, waves = d->waves, depth = d->depth;
    const bool src = d->src_b != nullptr;
    if (depth < 0)
        return fail(GE_ERR_INVALID, "ge_plan: depth = %d, need depth >= 1", depth);
    const Choice ch = default_choice(prec, depth, src);
    if (tile == 0) {
        tile = ch.tile;
        if (waves == 0) waves = ch.waves;
    }
    if (waves == 0) waves = prec == ge::kFP32C ? 4 : 1;
    if (depth == 0) {
        // clipped so that the halo stays within a quarter of the window
        depth = ch.depth;
        const int al = (prec == ge::kFP64) ? 2 : 4;
        while (depth > 1 && 4 * round_up(depth + 1, al) > (int64_t)waves * 64 * tile) --depth;
    }
    if (depth < 1)
        return fail(GE_ERR_INVALID, "ge_plan: depth = %d, need depth >= 1", depth);
    if (!ge::tile_config_supported(prec, tile, waves))
        return fail(GE_ERR_INVALID, "ge_plan: tile %d with %d waves is not built for precision %d",
                    tile, waves, prec);
    if (d->schedule < 0 || d->schedule > 2)
        return fail(GE_ERR_INVALID, "ge_plan: schedule %d unknown", d->schedule);
    if (d->schedule == 2 && !(waves == 1 && ge::persistent_supported(prec, tile)))
        return fail(GE_ERR_INVALID,
                    "ge_plan: the persistent schedule needs one wave and a built tile (%d)", tile);

    ge_plan_s *p = new (std::nothrow) ge_plan_s();
    if (!p)
        return fail(GE_ERR_NOMEM, "ge_plan: out of host memory");
    p->n = d->n;
    p->r = d->r;
    p->prec = prec;
    p->tile = tile;
    p->waves = waves;
    p->window = (int64_t)waves * 64 * tile;
    p->g_left = d->g_left;
    p->g_right = d->g_right;
    p->src_b = d->src_b;
    const int align = (prec == ge::kFP64) ? 2 : 4;   // values per 16-byte chunk
    if (p->n <= p->window) {
        // One window holds the rod and both walls: nothing enters from an
        // open edge, so every level of a call runs in one in-place launch.
        p->single = true;
        p->depth = depth;
        p->halo = 0;
        p->core = p->window;
        p->ntiles = 1;
    } else {
        p->single = false;
        p->depth = depth;
        p->halo = (int)round_up(depth + 1, align);
        p->core = p->window - 2 * p->halo;
        if (p->core < p->window / 2) {
            delete p;
            return fail(GE_ERR_INVALID,
                        "ge_plan: depth %d needs a halo of %d, too wide for a %lld-point window",
                        depth, (int)round_up(depth + 1, align), (long long)(waves * 64 * tile));
        }
        p->ntiles = (p->n + p->core - 1) / p->core;
    }
    // the library's choice: persistent wherever it is built and the rod has
    // enough tiles for the prefetch to matter
    const bool auto_persistent = d->schedule == 0 && persistent_pays(prec, tile, waves, p->depth, src) &&
                                 p->ntiles >= 64;
    p->persistent = !p->single && p->ntiles >= 3 && (d->schedule == 2 || auto_persistent);
    const double r = p->r;
    p->h = 1.0 / (double)(p->n + 1);
    p->tau = r * p->h * p->h;
    const ge::SchemeCoef sc = ge::scheme_coef(r);
    p->c1 = sc.c1;
    p->c2 = sc.c2;
    p->cs = sc.cs;
    p->e1 = p->tau * (1.0 + r) / (1.0 + 2.0 * r);
    p->e2 = p->tau * r / (1.0 + 2.0 * r);
    p->es = p->tau / (1.0 + r);
    (void)ge::status_alloc(p->status);
    // Per-tile launches over many tiles may split off their wall tiles: a
    // second stream (default priority) lets the wall kernel run beside the
    // interior one; without it (not created) they run one after the other.
    // Made here, not at the first step, so that a step can be captured into
    // a graph.
    if (!p->persistent && !p->single && p->ntiles >= kSideStreamTiles)
        p->side_state = side_create(p->side) ? 1 : -1;
    *out = p;
    return GE_OK;
}

void ge_destroy(ge_plan_t plan)
{
    if (!plan) return;
    if (plan->launched) ge::status_free(plan->status);
    else if (plan->status.host) (void)hipHostFree(plan->status.host);
    if (plan->side_state == 1) {
        (void)hipStreamSynchronize(plan->side.stream);
        (void)hipEventDestroy(plan->side.fork);
        (void)hipEventDestroy(plan->side.join);
        (void)hipStreamDestroy(plan->side.stream);
    }
    delete plan;
}

ge_status ge_plan_check(ge_plan_t plan, void *stream)
{
    if (!plan)
        return fail(GE_ERR_INVALID, "ge_plan_check: plan is NULL");
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail(e, "ge_plan_check: stream synchronize");
    if (ge::status_take(plan->status, ge::kStatusNonfinite))
        return fail(GE_ERR_NONFINITE, "ge_plan_check: a launch stored a NaN or infinite value");
    return GE_OK;
}

ge_status ge_plan_config(ge_plan_t plan, int32_t *tile, int32_t *depth, int32_t *waves,
                         int32_t *halo)
{
    if (!plan)
        return fail(GE_ERR_INVALID, "ge_plan_config: plan is NULL");
    if (tile) *tile = plan->tile;
    if (depth) *depth = plan->depth;
    if (waves) *waves = plan->waves;
    if (halo) *halo = plan->sdc ? plan->halo * plan->tile : plan->halo;   // points
    return GE_OK;
}

int32_t ge_plan_schedule(ge_plan_t plan)
{
    if (!plan) return -1;
    return plan->persistent ? 2 : 1;
}

ge_status ge_step_n(ge_plan_t plan, void *u, void *workspace, int64_t step0, int64_t nsteps,
                    const double *g_left_t, const double *g_right_t, const double *src_a_t,
                    double *flux, void *stream)
{
    if (!plan)
        return fail(GE_ERR_INVALID, "ge_step_n: plan is NULL");
    if (!u)
        return fail(GE_ERR_INVALID, "ge_step_n: u is NULL");
    if (step0 < 0 || nsteps < 0)
        return fail(GE_ERR_INVALID, "ge_step_n: step0 and nsteps must be >= 0");
    if (!aligned16(u))
        return fail(GE_ERR_INVALID, "ge_step_n: u must be 16-byte aligned");
    if ((plan->src_b != nullptr) != (src_a_t != nullptr))
        return fail(GE_ERR_INVALID, "%s", plan->src_b ? "ge_step_n: the plan has a source, src_a_t is NULL"
                                                      : "ge_step_n: src_a_t given but the plan has no source");
    const size_t bytes = (size_t)state_elems(plan->prec, plan->n) * elem_bytes(plan->prec);
    if (!plan->single) {
        if (!workspace)
            return fail(GE_ERR_INVALID, "ge_step_n: workspace is NULL");
        if (!aligned16(workspace))
            return fail(GE_ERR_INVALID, "ge_step_n: workspace must be 16-byte aligned");
        const uintptr_t a0 = (uintptr_t)u, a1 = a0 + bytes;
        const uintptr_t b0 = (uintptr_t)workspace, b1 = b0 + bytes;
        if (a0 < b1 && b0 < a1)
            return fail(GE_ERR_INVALID, "ge_step_n: u and workspace overlap");
    }
    if (plan->sdc && flux)
        return fail(GE_ERR_UNSUPPORTED, "ge_step_n: the sub-domain scheme keeps no wall flux");
    if (ge::status_take(plan->status, ge::kStatusNonfinite))
        return fail(GE_ERR_NONFINITE,
                    "ge_step_n: an earlier launch of this plan stored a NaN or infinite value");
    if (nsteps == 0)
        return GE_OK;
    plan->launched = true;

    hipStream_t st = static_cast<hipStream_t>(stream);
    ge::TileArgs a{};
    a.src_b = plan->src_b;
    a.flux = flux;
    a.n = plan->n;
    a.core = plan->core;
    a.ntiles = plan->ntiles;
    a.halo = plan->halo;
    a.estride = plan->prec == ge::kFP32C ? ge::comp_offset(plan->n) : 0;
    a.estride_out = a.estride;
    a.c1 = plan->c1; a.c2 = plan->c2; a.cs = plan->cs;
    a.e1 = plan->e1; a.e2 = plan->e2; a.es = plan->es;
    a.gl0 = plan->g_left; a.gr0 = plan->g_right;
    a.tau = plan->tau; a.h = plan->h;
    a.status = plan->status.dev;
    const bool src = plan->src_b != nullptr;
    if (plan->sdc) {
        a.nsdc = (plan->n + 1) / plan->tile;
        a.ca = plan->e1;
    }
    // the plan's second stream for split launches, if it holds one
    const ge::SideStream *side = plan->side_state == 1 ? &plan->side : nullptr;
    // one launch of whichever kernel the plan runs
    auto launch = [&](const ge::TileArgs &la) {
        if (plan->sdc)
            return plan->persistent
                       ? ge::launch_sdc_persistent(plan->prec, plan->sdc, plan->waves, la, st)
                       : ge::launch_sdc(plan->prec, plan->sdc, plan->waves, la, st);
        if (plan->persistent && !plan->single)
            return ge::launch_tiles_persistent(plan->prec, plan->tile, src, la, st);
        return ge::launch_tiles(plan->prec, plan->tile, plan->waves, src, la, st, side);
    };

    if (plan->single) {
        // in place, bounded work per launch
        const int64_t chunk = 1 << 16;
        for (int64_t done = 0; done < nsteps; done += chunk) {
            const int64_t lev = (nsteps - done < chunk) ? nsteps - done : chunk;
            a.in = u;
            a.out = u;
            a.level0 = step0 + done;
            a.nlev = (int32_t)lev;
            a.gl_t = g_left_t ? g_left_t + done : nullptr;
            a.gr_t = g_right_t ? g_right_t + done : nullptr;
            a.src_a = src_a_t ? src_a_t + done : nullptr;
            hipError_t e = launch(a);
            if (e != hipSuccess)
                return hip_fail(e, "ge_step_n: launch");
        }
        return GE_OK;
    }

    // Ping-pong between u and the workspace.  An even number of launches
    // leaves the result in u; the levels are spread evenly over them.
    int64_t launches = (nsteps + plan->depth - 1) / plan->depth;
    if ((launches & 1) && nsteps > launches)
        ++launches;
    const int64_t base = nsteps / launches, extra = nsteps % launches;
    void *bufs[2] = {u, workspace};
    int64_t done = 0;
    for (int64_t k = 0; k < launches; ++k) {
        const int64_t lev = base + (k < extra ? 1 : 0);
        a.in = bufs[k & 1];
        a.out = bufs[(k + 1) & 1];
        a.level0 = step0 + done;
        a.nlev = (int32_t)lev;
        a.gl_t = g_left_t ? g_left_t + done : nullptr;
        a.gr_t = g_right_t ? g_right_t + done : nullptr;
        a.src_a = src_a_t ? src_a_t + done : nullptr;
        hipError_t e = launch(a);
        if (e != hipSuccess)
            return hip_fail(e, "ge_step_n: launch");
        done += lev;
    }
    if (launches & 1) {
        hipError_t e = hipMemcpyAsync(u, workspace, bytes, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess)
            return hip_fail(e, "ge_step_n: copy back");
    }
    return GE_OK;
}

ge_status ge_comp_to_fp64(const float *pair, double *x, int64_t n, void *stream)
{
    if (!pair || !x || n < 0)
        return fail(GE_ERR_INVALID, "ge_comp_to_fp64: bad arguments");
    hipError_t e = ge::launch_comp_to_fp64(pair, x, n, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GE_OK : hip_fail(e, "ge_comp_to_fp64");
}

ge_status ge_comp_from_fp64(const double *x, float *pair, int64_t n, void *stream)
{
    if (!pair || !x || n < 0)
        return fail(GE_ERR_INVALID, "ge_comp_from_fp64: bad arguments");
    hipError_t e = ge::launch_comp_from_fp64(x, pair, n, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GE_OK : hip_fail(e, "ge_comp_from_fp64");
}

// Levels per launch of the 2D extension when the caller leaves it to the
// library: measured on MI355X (4096^2 points, 200 levels), four levels per
// launch 8.7e11 updates/s in FP64 against 6.4e11 at two and 3.7e11 at one
// (FP32: 1.39e12, 1.06e12, 6.6e11).
constexpr int kDepth2d = 4;

size_t ge_2d_workspace_bytes(const ge_2d_desc *d)
{
    if (!d || d->nx < 1 || d->ny < 1 || d->nx > 0x7fffff00LL || d->ny > 0x7fffff00LL ||
        (d->precision != ge::kFP64 && d->precision != ge::kFP32))
        return 0;
    return (size_t)(d->nx * d->ny) * (size_t)elem_bytes(d->precision);
}

ge_status ge_2d_step_n(const ge_2d_desc *d, void *u, void *workspace, int64_t step0, int64_t nsteps,
                      void *stream)
{
    if (!d)
        return fail(GE_ERR_INVALID, "ge_2d_step_n: NULL description");
    if (d->precision == ge::kFP32C)
        return fail(GE_ERR_UNSUPPORTED, "ge_2d_step_n: the 2D extension runs in FP64 or FP32");
    if (d->precision != ge::kFP64 && d->precision != ge::kFP32)
        return fail(GE_ERR_INVALID, "ge_2d_step_n: precision = %d", d->precision);
    if (d->nx < 1 || d->ny < 1 || d->nx > 0x7fffff00LL || d->ny > 0x7fffff00LL ||
        d->nx * d->ny > (1LL << 40))
        return fail(GE_ERR_INVALID, "ge_2d_step_n: grid %lld x %lld out of range",
                    (long long)d->nx, (long long)d->ny);
    if (!(d->rx > 0.0) || !(d->ry > 0.0) || !std::isfinite(d->rx) || !std::isfinite(d->ry))
        return fail(GE_ERR_INVALID, "ge_2d_step_n: rx, ry must be positive and finite");
    if (!std::isfinite(d->g_west) || !std::isfinite(d->g_east) || !std::isfinite(d->g_south) ||
        !std::isfinite(d->g_north))
        return fail(GE_ERR_INVALID, "ge_2d_step_n: wall values must be finite");
    if (step0 < 0 || nsteps < 0)
        return fail(GE_ERR_INVALID, "ge_2d_step_n: step0 and nsteps must be >= 0");
    if (d->depth != 0 && d->depth != 1 && d->depth != 2 && d->depth != 4)
        return fail(GE_ERR_INVALID, "ge_2d_step_n: depth = %d, need 0, 1, 2 or 4", d->depth);
    if (nsteps == 0)
        return GE_OK;
    const size_t bytes = ge_2d_workspace_bytes(d);
    const uintptr_t a0 = (uintptr_t)u, b0 = (uintptr_t)workspace;
    if (!u || !workspace || (a0 < b0 + bytes && b0 < a0 + bytes))
        return fail(GE_ERR_INVALID, "ge_2d_step_n: u and workspace must be distinct, non-overlapping");
    ge::Grid2dArgs a;
    a.u = u;
    a.work = workspace;
    a.nx = d->nx;
    a.ny = d->ny;
    a.step0 = step0;
    a.nsteps = nsteps;
    a.rx = d->rx;
    a.ry = d->ry;
    a.gw = d->g_west;
    a.ge = d->g_east;
    a.gs = d->g_south;
    a.gn = d->g_north;
    a.depth = d->depth != 0 ? d->depth : kDepth2d;
    const hipError_t e = ge::launch_2d(d->precision, a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return ge::set_error(GE_ERR_HIP, "ge_2d_step_n: %s", hipGetErrorString(e));
    return GE_OK;
}

}  // extern "C"
