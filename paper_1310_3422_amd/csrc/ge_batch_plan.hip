// Host side of the batch sweep: the plan (per-rod points-per-lane choice,
// bundling of rods into workgroup tasks, largest-first order), the
// autotuner that measures the per-level cost of each choice on the device,
// and the hipGraph that captures one run.
#include <algorithm>
#include <cerrno>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <sys/stat.h>
#include <vector>

#include "ge.h"
#include "ge_batch.h"
#include "ge_internal.h"
#include "ge_kernels.h"

namespace {

using ge::BatchRod;
using ge::BatchTask;
using ge::kBatchWaves;

constexpr int kKs[] = {4, 8, 16, 32, 64};
constexpr int kNK = 5;

// Cost of one level of one task, in microseconds: `base` for a task whose
// rods span many waves, `wall` the extra when every wave holds a rod end.
struct KCost {
    double base = 0, wall = 0;
};

struct CostModel {
    KCost k[kNK];
    bool measured = false;
};

std::mutex g_tune_mu;
std::map<std::string, CostModel> g_tune;   // device key + precision -> model

int k_index(int k)
{
    for (int i = 0; i < kNK; ++i)
        if (kKs[i] == k) return i;
    return -1;
}

// Default model (per-level microseconds of a 16-wave task), from
// measurements of the batch kernel on MI355X; used until the device has
// been tuned.  VALU work grows with K; the constant covers the barrier and
// the LDS exchange, which halo-lane tasks pay once every K-1 levels.
CostModel default_model(int prec, int sync)
{
    CostModel m;
    const double per_k = prec == ge::kFP32 ? 0.0105 : (prec == ge::kFP64 ? 0.0135 : 0.0215);
    for (int i = 0; i < kNK; ++i) {
        m.k[i].base = (sync == 3 ? 0.25 / (kKs[i] - 1) : 0.25) + per_k * kKs[i];
        m.k[i].wall = 0.05 + 0.002 * kKs[i];
    }
    return m;
}

std::string device_key(int prec, int sync)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    const std::string tail = "/" + std::to_string(prec) + "/s" + std::to_string(sync);
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown" + tail;
    return std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) +
           "cu" + tail;
}

std::string cache_path()
{
    const char *p = getenv("GE_TUNE_CACHE");
    if (p && *p) return p;
    const char *home = getenv("HOME");
    std::string dir = std::string(home && *home ? home : "/tmp") + "/.cache";
    mkdir(dir.c_str(), 0755);
    dir += "/libge";
    mkdir(dir.c_str(), 0755);
    return dir + "/batch_tune.txt";
}

// Cache file: one line per (device key, K): "<key> <K> <base_us> <wall_us>".
void load_cache_locked()
{
    static bool loaded = false;
    if (loaded) return;
    loaded = true;
    FILE *f = fopen(cache_path().c_str(), "r");
    if (!f) return;
    char key[256];
    int k;
    double base, wall;
    while (fscanf(f, "%255s %d %lf %lf", key, &k, &base, &wall) == 4) {
        const int i = k_index(k);
        if (i < 0) continue;
        CostModel &m = g_tune[key];
        m.k[i].base = base;
        m.k[i].wall = wall;
        m.measured = true;
    }
    fclose(f);
}

void save_cache_locked()
{
    const std::string path = cache_path();
    const std::string tmp = path + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    for (const auto &kv : g_tune) {
        if (!kv.second.measured) continue;
        for (int i = 0; i < kNK; ++i)
            fprintf(f, "%s %d %.6f %.6f\n", kv.first.c_str(), kKs[i], kv.second.k[i].base,
                    kv.second.k[i].wall);
    }
    fclose(f);
    rename(tmp.c_str(), path.c_str());
}

int waves_for(int64_t n, int k) { return (int)((n + 64 * k - 1) / (64 * k)); }

// Waves of a rod at k points per lane, and whether it runs as a halo-lane
// task (halo mode, two or more overlapping waves that fit the workgroup, and
// a last window that can end at the wall).
int rod_waves(int64_t n, int k, bool halo_mode, int *halo)
{
    if (halo_mode) {
        const ge::HaloLayout L(n, k);
        if (L.fits && L.m <= kBatchWaves) {
            *halo = 1;
            return L.m;
        }
    }
    *halo = 0;
    return waves_for(n, k);
}

// Polls a neighbour wait makes before it gives up (about two milliseconds).
constexpr int kDefaultWaitPolls = 1 << 16;

struct Plan {
    std::vector<int> rod_k;
    std::vector<BatchTask> tasks;
    double est_us = 0;
    bool has_long = false;
};

// Levels per pass of a long-rod task, and its halo (levels + 1, rounded up
// to the 16-byte chunk of the state type).
constexpr int kLongDepth = 32;
int long_halo(int prec)
{
    const int align = prec == ge::kFP64 ? 2 : 4;
    return (kLongDepth + 1 + align - 1) / align * align;
}

// Points the registers of one workgroup hold (the on-chip limit); longer
// rods run as long-rod tasks.
int64_t on_chip_cap(int prec) { return (int64_t)kBatchWaves * 64 * ge::batch_max_k(prec); }

// Per-level cost of a long-rod task: its 16 waves take the rod's windows in
// rounds, each round about one level of a 16-wave task at the same points
// per lane, plus the pass's trip through memory.
double long_cost(int64_t n, int prec, const CostModel &cm)
{
    const int k = ge::batch_long_k(prec);
    const int64_t core = 64 * (int64_t)k - 2 * long_halo(prec);
    const int64_t wins = (n + core - 1) / core;
    const int64_t rounds = (wins + kBatchWaves - 1) / kBatchWaves;
    return (double)rounds * cm.k[k_index(k)].base * 1.15;
}

// Bundle rods into workgroup tasks.  Rods are placed largest first; each rod
// goes into an open task of some feasible K where it fits (those waves are
// already paid for), the tightest such fit; otherwise it opens the task whose
// per-level cost, weighted by the share of the workgroup it occupies, is
// lowest.  All choices give bit-identical results; only the time differs.
Plan make_plan(const std::vector<int64_t> &n, int prec, const CostModel &cm, int64_t nsteps,
               int grid, bool halo_mode)
{
    const int nr = (int)n.size();
    const int kmax = ge::batch_max_k(prec);
    std::vector<int> order(nr);
    for (int i = 0; i < nr; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n[a] > n[b]; });

    Plan P;
    P.rod_k.assign(nr, 0);
    struct Bin { int k; int halo; int used; int nwall; double cost; };
    std::vector<Bin> bins;
    std::vector<std::vector<int>> members;
    auto task_cost = [&](int k, int nwall) {
        const KCost &c = cm.k[k_index(k)];
        return c.base + c.wall * (double)nwall / kBatchWaves;
    };
    const int64_t cap = on_chip_cap(prec);
    for (int r : order) {
        if (n[r] > cap) {
            // a task of its own, swept in passes
            bins.push_back(Bin{ge::batch_long_k(prec), 2, kBatchWaves, 2, long_cost(n[r], prec, cm)});
            members.push_back({r});
            P.rod_k[r] = ge::batch_long_k(prec);
            P.has_long = true;
            continue;
        }
        int best_bin = -1, best_left = 1 << 30;
        int best_k = 0, best_h = 0;
        double best_new = 1e300;
        for (int ki = 0; ki < kNK; ++ki) {
            const int k = kKs[ki];
            if (k > kmax) continue;
            int h = 0;
            const int w = rod_waves(n[r], k, halo_mode, &h);
            if (w > kBatchWaves) continue;
            for (size_t b = 0; b < bins.size(); ++b) {
                if (bins[b].k != k || bins[b].halo != h) continue;
                const int left = kBatchWaves - bins[b].used - w;
                if (left >= 0 && left < best_left) {
                    best_left = left;
                    best_bin = (int)b;
                }
            }
            const double c = task_cost(k, std::min(w, 2)) * w / kBatchWaves;
            if (c < best_new) {
                best_new = c;
                best_k = k;
                best_h = h;
            }
        }
        if (best_bin < 0) {
            bins.push_back(Bin{best_k, best_h, 0, 0, 0.0});
            members.emplace_back();
            best_bin = (int)bins.size() - 1;
        }
        Bin &b = bins[best_bin];
        int hb = 0;
        const int w = rod_waves(n[r], b.k, halo_mode, &hb);
        b.used += w;
        b.nwall += std::min(w, 2);
        members[best_bin].push_back(r);
        P.rod_k[r] = b.k;
    }
    for (Bin &b : bins)
        if (b.halo != 2) b.cost = task_cost(b.k, b.nwall);
    // largest first
    std::vector<int> border(bins.size());
    for (size_t i = 0; i < bins.size(); ++i) border[i] = (int)i;
    std::stable_sort(border.begin(), border.end(),
                     [&](int a, int b) { return bins[a].cost > bins[b].cost; });
    std::vector<double> load(std::max(grid, 1), 0.0);
    for (int bi : border) {
        BatchTask t;
        memset(&t, 0, sizeof t);
        t.k = bins[bi].k;
        t.halo = bins[bi].halo;
        int w = 0;
        for (int r : members[bi]) {
            int hb = 0;
            const int nw = t.halo == 2 ? 1 : rod_waves(n[r], t.k, halo_mode, &hb);
            for (int j = 0; j < nw; ++j) {
                t.wave_rod[w] = r;
                t.wave_idx[w] = j;
                ++w;
            }
        }
        for (; w < kBatchWaves; ++w) {
            t.wave_rod[w] = -1;
            t.wave_idx[w] = 0;
        }
        P.tasks.push_back(t);
        // earliest-free workgroup takes the next task
        auto it = std::min_element(load.begin(), load.end());
        *it += bins[bi].cost * (double)nsteps;
    }
    P.est_us = load.empty() ? 0 : *std::max_element(load.begin(), load.end());
    return P;
}

int device_grid()
{
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int per_cu = 0;
    // one resident 16-wave workgroup per compute unit
    per_cu = 1;
    return std::max(1, cus * per_cu);
}

}  // namespace

struct ge_batch_s {
    int prec;
    int sync;               // 1: barrier per level, 2: neighbour flags, 3: halo lanes
    int64_t nrods;
    int64_t total;          // offsets[nrods]
    int64_t estride;        // e block offset (FP32C)
    std::vector<int64_t> n;
    std::vector<int> rod_k;
    int ntasks;
    int grid;
    double est_us;
    bool has_long;          // some rod runs as a long-rod task (workspace holds u2)
    int64_t long_elems;     // elements of one block of u2 (s; the pair has two)
    int64_t estride2;       // element offset of u2's e block (FP32C)
    int wait_polls;         // bound on a neighbour wait's polls
    ge::StatusWords status; // words raised by the kernels
    BatchRod *d_rods;
    BatchTask *d_tasks;
    hipStream_t cap;        // private stream used only for capture
    // instantiated graphs, one per (state, workspace, parity, level count),
    // the least recently used replaced when all slots are taken
    struct Graph {
        hipGraphExec_t exec;
        void *u, *ws;
        int parity;
        int64_t nsteps;
        uint64_t used;
    };
    static constexpr int kGraphs = 4;
    Graph graphs[kGraphs];
    int ngraphs;
    uint64_t clock;
};

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
    return ge::set_error(GE_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Report (and clear) what finished launches of the plan raised.
ge_status take_status(ge_batch_s *b, const char *who)
{
    if (ge::status_take(b->status, ge::kStatusWaitGaveUp))
        return fail(GE_ERR_SYNC, "%s: a wave's wait for its neighbour gave up; the results of "
                                 "that run are not valid", who);
    if (ge::status_take(b->status, ge::kStatusNonfinite))
        return fail(GE_ERR_NONFINITE, "%s: a run stored a NaN or infinite value", who);
    return GE_OK;
}

// Drop the instantiated graphs (their kernel arguments are out of date).
void drop_graphs(ge_batch_s *b)
{
    if (b->ngraphs > 0) (void)hipDeviceSynchronize();
    for (int i = 0; i < b->ngraphs; ++i) (void)hipGraphExecDestroy(b->graphs[i].exec);
    b->ngraphs = 0;
}

void free_batch(ge_batch_s *b)
{
    if (!b) return;
    drop_graphs(b);
    ge::status_free(b->status);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->d_rods) (void)hipFree(b->d_rods);
    if (b->d_tasks) (void)hipFree(b->d_tasks);
    delete b;
}

// Time one run of the batch kernel (synchronisation mode `sync`) on a
// synthetic batch whose tasks are all K-point-per-lane tasks; returns
// microseconds per level per task.
double time_tasks(int prec, int sync, int k, bool walls, int grid, void *u, size_t ubytes,
                  int *counter, BatchRod *d_rods, BatchTask *d_tasks, int nsteps, hipStream_t st)
{
    const int ntasks = 2 * grid;
    const int rods_per_task = walls ? kBatchWaves : 1;
    const bool halo = sync == 3;
    // rods of one wave each, or one rod over all 16 waves
    const int64_t rod_n = walls ? (int64_t)64 * k - 1
                                : (halo ? (int64_t)64 * k + (int64_t)(kBatchWaves - 1) * 62 * k - 1
                                        : (int64_t)64 * k * kBatchWaves - 1);
    std::vector<BatchRod> rods(ntasks * rods_per_task);
    std::vector<BatchTask> tasks(ntasks);
    const int esz = prec == ge::kFP64 ? 8 : 4;
    const int64_t stride = (rod_n + 63) / 64 * 64;
    if ((size_t)(stride * rods.size() * esz * (prec == ge::kFP32C ? 2 : 1)) > ubytes) return -1;
    const ge::SchemeCoef sc = ge::scheme_coef(2.0);
    for (size_t i = 0; i < rods.size(); ++i)
        rods[i] = BatchRod{(int64_t)i * stride, rod_n, sc.c1, sc.c2, sc.cs, 0.25, -0.5, -1};
    for (int t = 0; t < ntasks; ++t) {
        memset(&tasks[t], 0, sizeof(BatchTask));
        tasks[t].k = k;
        tasks[t].halo = (halo && !walls) ? 1 : 0;   // one-wave rods never run as halo tasks
        for (int w = 0; w < kBatchWaves; ++w) {
            tasks[t].wave_rod[w] = walls ? t * rods_per_task + w : t;
            tasks[t].wave_idx[w] = walls ? 0 : w;
        }
    }
    if (hipMemcpyAsync(d_rods, rods.data(), rods.size() * sizeof(BatchRod),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d_tasks, tasks.data(), tasks.size() * sizeof(BatchTask),
                       hipMemcpyHostToDevice, st) != hipSuccess)
        return -1;
    ge::BatchArgs a{};
    a.u = u;
    a.rods = d_rods;
    a.tasks = d_tasks;
    a.counter = counter;
    a.estride = stride * (int64_t)rods.size();
    a.step0 = 0;
    a.nsteps = nsteps;
    a.ntasks = ntasks;
    a.sync = sync;
    a.wait_polls = kDefaultWaitPolls;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    double best = 1e300;
    for (int rep = 0; rep < 3; ++rep) {
        (void)hipEventRecord(e0, st);
        if (ge::launch_batch(prec, a, grid, st) != hipSuccess) {
            best = -1;
            break;
        }
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) best = std::min(best, (double)ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best < 0) return -1;
    // every workgroup runs ntasks/grid = 2 tasks of nsteps levels
    return best * 1e3 / (2.0 * nsteps);
}

ge_status tune_device(int prec, int sync, CostModel &m)
{
    const int grid = device_grid();
    const int kmax = ge::batch_max_k(prec);
    const int nsteps = 200;
    // enough for 2*grid tasks of 16 waves x 64 lanes x kmax points, pair-sized
    const size_t ubytes = (size_t)2 * grid * kBatchWaves * 64 * kmax * 8 + (1 << 20);
    void *u = nullptr;
    int *counter = nullptr;
    BatchRod *d_rods = nullptr;
    BatchTask *d_tasks = nullptr;
    hipStream_t st = nullptr;
    ge_status rc = GE_OK;
    if (hipMalloc(&u, ubytes) != hipSuccess || hipMalloc((void **)&counter, 256) != hipSuccess ||
        hipMalloc((void **)&d_rods, sizeof(BatchRod) * 2 * grid * kBatchWaves) != hipSuccess ||
        hipMalloc((void **)&d_tasks, sizeof(BatchTask) * 2 * grid) != hipSuccess ||
        hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        rc = fail(GE_ERR_NOMEM, "ge_batch_plan: tuning buffers could not be allocated");
    } else if (hipMemsetAsync(u, 0, ubytes, st) != hipSuccess) {
        rc = fail(GE_ERR_HIP, "ge_batch_plan: tuning buffer clear failed");
    } else {
        for (int i = 0; i < kNK && rc == GE_OK; ++i) {
            if (kKs[i] > kmax) {
                m.k[i].base = 1e9;   // not built
                m.k[i].wall = 0;
                continue;
            }
            const double base = time_tasks(prec, sync, kKs[i], false, grid, u, ubytes, counter,
                                           d_rods, d_tasks, nsteps, st);
            const double all = time_tasks(prec, sync, kKs[i], true, grid, u, ubytes, counter,
                                          d_rods, d_tasks, nsteps, st);
            if (base <= 0 || all <= 0) {
                rc = fail(GE_ERR_HIP, "ge_batch_plan: tuning run failed");
                break;
            }
            m.k[i].base = base;
            m.k[i].wall = std::max(0.0, all - base);
        }
        m.measured = (rc == GE_OK);
    }
    if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    if (u) (void)hipFree(u);
    if (counter) (void)hipFree(counter);
    if (d_rods) (void)hipFree(d_rods);
    if (d_tasks) (void)hipFree(d_tasks);
    return rc;
}

}  // namespace

extern "C" {

ge_status ge_batch_plan(ge_batch_t *out, const ge_batch_desc *d)
{
    if (!out)
        return fail(GE_ERR_INVALID, "ge_batch_plan: out is NULL");
    *out = nullptr;
    if (!d)
        return fail(GE_ERR_INVALID, "ge_batch_plan: desc is NULL");
    if (d->nrods < 1 || d->nrods > (1 << 24))
        return fail(GE_ERR_INVALID, "ge_batch_plan: nrods = %lld out of range",
                    (long long)d->nrods);
    if (!d->n || !d->offsets || !d->r || !d->g_left || !d->g_right)
        return fail(GE_ERR_INVALID, "ge_batch_plan: a rod table pointer is NULL");
    if (d->precision < GE_FP64 || d->precision > GE_FP32_COMP)
        return fail(GE_ERR_INVALID, "ge_batch_plan: unknown precision %d", d->precision);
    if (d->sync < 0 || d->sync > 3)
        return fail(GE_ERR_INVALID, "ge_batch_plan: sync %d unknown", d->sync);
    const int prec = d->precision;
    // library choice, measured on the 4096-rod batch: halo lanes (+23% FP32,
    // +21% pair, +26% FP64 over neighbour flags)
    const int sync = d->sync != 0 ? d->sync : 3;
    for (int64_t i = 0; i < d->nrods; ++i) {
        if (d->n[i] < 1)
            return fail(GE_ERR_INVALID, "ge_batch_plan: rod %lld has n = %lld", (long long)i,
                        (long long)d->n[i]);
        if (d->offsets[i] < 0 || d->offsets[i] % 4 != 0)
            return fail(GE_ERR_INVALID, "ge_batch_plan: offsets[%lld] must be >= 0 and a multiple of 4",
                        (long long)i);
        if (d->offsets[i + 1] < d->offsets[i] + d->n[i])
            return fail(GE_ERR_INVALID, "ge_batch_plan: rod %lld overlaps the next one", (long long)i);
        if (!std::isfinite(d->r[i]) || !std::isfinite(d->g_left[i]) || !std::isfinite(d->g_right[i]))
            return fail(GE_ERR_NONFINITE, "ge_batch_plan: rod %lld has a non-finite parameter",
                        (long long)i);
        if (!(d->r[i] > 0))
            return fail(GE_ERR_INVALID, "ge_batch_plan: rod %lld has r = %g", (long long)i, d->r[i]);
    }

    CostModel cm;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_cache_locked();
        const std::string key = device_key(prec, sync);
        auto it = g_tune.find(key);
        if (d->tune || it == g_tune.end() || !it->second.measured) {
            if (d->tune) {
                CostModel m;
                ge_status rc = tune_device(prec, sync, m);
                if (rc != GE_OK) return rc;
                g_tune[key] = m;
                save_cache_locked();
                cm = m;
            } else {
                cm = default_model(prec, sync);
            }
        } else {
            cm = it->second;
        }
    }

    ge_batch_s *b = new (std::nothrow) ge_batch_s();
    if (!b)
        return fail(GE_ERR_NOMEM, "ge_batch_plan: out of host memory");
    b->prec = prec;
    b->sync = sync;
    b->nrods = d->nrods;
    b->total = d->offsets[d->nrods];
    b->estride = prec == ge::kFP32C ? ge::comp_offset(b->total) : 0;
    b->n.assign(d->n, d->n + d->nrods);
    b->grid = device_grid();

    // rods above the on-chip limit get their second level buffers back to
    // back in u2, each starting on a 256-byte boundary
    std::vector<BatchRod> rods(d->nrods);
    int64_t woff = 0;
    for (int64_t i = 0; i < d->nrods; ++i) {
        const ge::SchemeCoef sc = ge::scheme_coef(d->r[i]);
        const bool lng = d->n[i] > on_chip_cap(prec);
        rods[i] = BatchRod{d->offsets[i], d->n[i], sc.c1, sc.c2, sc.cs, d->g_left[i],
                           d->g_right[i], lng ? woff : -1};
        if (lng) woff += (d->n[i] + 63) / 64 * 64;
    }
    b->long_elems = woff;
    b->estride2 = prec == ge::kFP32C ? woff : 0;
    Plan P = make_plan(b->n, prec, cm, 1, b->grid, sync == 3);
    b->rod_k = P.rod_k;
    b->ntasks = (int)P.tasks.size();
    b->est_us = P.est_us;
    b->has_long = P.has_long;
    b->wait_polls = kDefaultWaitPolls;
    hipError_t e;
    if ((e = hipMalloc((void **)&b->d_rods, sizeof(BatchRod) * rods.size())) != hipSuccess ||
        (e = hipMalloc((void **)&b->d_tasks, sizeof(BatchTask) * P.tasks.size())) != hipSuccess) {
        free_batch(b);
        return fail(GE_ERR_NOMEM, "ge_batch_plan: device tables: %s", hipGetErrorString(e));
    }
    if ((e = hipMemcpy(b->d_rods, rods.data(), sizeof(BatchRod) * rods.size(),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(b->d_tasks, P.tasks.data(), sizeof(BatchTask) * P.tasks.size(),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess) {
        free_batch(b);
        return hip_fail(e, "ge_batch_plan: setup");
    }
    if (!ge::status_alloc(b->status)) {
        free_batch(b);
        return fail(GE_ERR_NOMEM, "ge_batch_plan: status words could not be allocated");
    }
    *out = b;
    return GE_OK;
}

void ge_batch_destroy(ge_batch_t b) { free_batch(b); }

size_t ge_batch_workspace_bytes(ge_batch_t b)
{
    if (!b) return 0;
    if (!b->has_long) return 256;
    const size_t u2 = (size_t)b->long_elems * (b->prec == ge::kFP32C ? 2 : 1) *
                      (b->prec == ge::kFP64 ? 8 : 4);
    return 256 + (u2 + 255) / 256 * 256;
}

ge_status ge_batch_set_wait_polls(ge_batch_t b, int64_t polls)
{
    if (!b)
        return fail(GE_ERR_INVALID, "ge_batch_set_wait_polls: batch is NULL");
    if (polls < 0 || polls > (1 << 30))
        return fail(GE_ERR_INVALID, "ge_batch_set_wait_polls: polls = %lld out of range",
                    (long long)polls);
    if (polls != b->wait_polls) {
        drop_graphs(b);
        b->wait_polls = (int)polls;
    }
    return GE_OK;
}

ge_status ge_batch_check(ge_batch_t b, void *stream)
{
    if (!b)
        return fail(GE_ERR_INVALID, "ge_batch_check: batch is NULL");
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail(e, "ge_batch_check: stream synchronize");
    return take_status(b, "ge_batch_check");
}

}  // extern "C"

bool ge::batch_shape(ge_batch_t b, int64_t *nrods, const int64_t **n, int *prec)
{
    if (!b) return false;
    *nrods = b->nrods;
    *n = b->n.data();
    *prec = b->prec;
    return true;
}

namespace {

// Kernel arguments of one run of the plan with queue head and second level
// buffers at `work` (256-byte aligned: the head, then u2 from byte 256).
ge::BatchArgs run_args(const ge_batch_s *b, void *u, void *work, int64_t step0, int64_t nsteps)
{
    ge::BatchArgs a{};
    a.u = u;
    a.rods = b->d_rods;
    a.tasks = b->d_tasks;
    a.counter = static_cast<int *>(work);
    a.estride = b->estride;
    a.step0 = step0 & 1;   // only the parity of the first level matters
    a.nsteps = (int32_t)nsteps;
    a.ntasks = b->ntasks;
    a.sync = b->sync;
    a.wait_polls = b->wait_polls;
    a.status = b->status.dev;
    a.u2 = b->has_long ? static_cast<char *>(work) + 256 : nullptr;
    a.estride2 = b->estride2;
    a.long_depth = kLongDepth;
    a.long_halo = long_halo(b->prec);
    return a;
}

// Checks shared by both run entry points; reports what earlier runs raised.
ge_status check_run(ge_batch_s *b, void *u, int64_t step0, int64_t nsteps, const char *who)
{
    if (!b)
        return fail(GE_ERR_INVALID, "%s: batch is NULL", who);
    if (!u)
        return fail(GE_ERR_INVALID, "%s: u must be given", who);
    if ((uintptr_t)u & 15)
        return fail(GE_ERR_INVALID, "%s: u must be 16-byte aligned", who);
    if (step0 < 0 || nsteps < 0 || nsteps > (1 << 30))
        return fail(GE_ERR_INVALID, "%s: step0/nsteps out of range", who);
    return take_status(b, who);
}

}  // namespace

extern "C" {

int64_t ge_batch_state_elems(ge_batch_t b)
{
    if (!b) return -1;
    return b->prec == ge::kFP32C ? 2 * b->estride : b->total;
}

ge_status ge_batch_info(ge_batch_t b, int32_t *ntasks, int32_t *grid, double *est_us_per_level,
                        int32_t *rod_k)
{
    if (!b)
        return fail(GE_ERR_INVALID, "ge_batch_info: batch is NULL");
    if (ntasks) *ntasks = b->ntasks;
    if (grid) *grid = b->grid;
    if (est_us_per_level) *est_us_per_level = b->est_us;
    if (rod_k)
        for (int64_t i = 0; i < b->nrods; ++i) rod_k[i] = b->rod_k[i];
    return GE_OK;
}

ge_status ge_solve_batch(ge_batch_t b, void *u, void *workspace, int64_t step0, int64_t nsteps,
                         void *stream)
{
    if (b && !workspace)
        return fail(GE_ERR_INVALID, "ge_solve_batch: workspace must be given");
    if ((uintptr_t)workspace & 255)
        return fail(GE_ERR_INVALID, "ge_solve_batch: workspace must be 256-byte aligned");
    {
        const ge_status rs = check_run(b, u, step0, nsteps, "ge_solve_batch");
        if (rs != GE_OK) return rs;
    }
    if (nsteps == 0)
        return GE_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int parity = (int)(step0 & 1);
    ge_batch_s::Graph *slot = nullptr;
    for (int i = 0; i < b->ngraphs; ++i) {
        ge_batch_s::Graph &g = b->graphs[i];
        if (g.u == u && g.ws == workspace && g.parity == parity && g.nsteps == nsteps) slot = &g;
    }
    if (!slot) {
        const ge::BatchArgs a = run_args(b, u, workspace, parity, nsteps);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "ge_solve_batch: begin capture");
        hipError_t le = ge::launch_batch(b->prec, a, b->grid, b->cap);
        e = hipStreamEndCapture(b->cap, &g);
        if (le != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(le, "ge_solve_batch: capture launch");
        }
        if (e != hipSuccess) return hip_fail(e, "ge_solve_batch: end capture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "ge_solve_batch: instantiate");
        if (b->ngraphs < ge_batch_s::kGraphs) {
            slot = &b->graphs[b->ngraphs++];
        } else {
            slot = &b->graphs[0];
            for (int i = 1; i < b->ngraphs; ++i)
                if (b->graphs[i].used < slot->used) slot = &b->graphs[i];
            // the replaced graph may still be queued on a stream: wait for it
            (void)hipDeviceSynchronize();
            (void)hipGraphExecDestroy(slot->exec);
        }
        *slot = ge_batch_s::Graph{exec, u, workspace, parity, nsteps, 0};
    }
    slot->used = ++b->clock;
    hipError_t e = hipGraphLaunch(slot->exec, st);
    return e == hipSuccess ? GE_OK : hip_fail(e, "ge_solve_batch: graph launch");
}

}  // extern "C"

extern "C" {

ge_status ge_solve_batch_static(ge_batch_t b, void *u, int64_t step0, int64_t nsteps,
                                void *stream)
{
    {
        const ge_status rs = check_run(b, u, step0, nsteps, "ge_solve_batch_static");
        if (rs != GE_OK) return rs;
    }
    const size_t need = ge_batch_workspace_bytes(b);
    if (need > ge::kBatchScratchBytes)
        return fail(GE_ERR_UNSUPPORTED,
                    "ge_solve_batch_static: the plan needs %zu bytes of scratch (its rods above "
                    "the on-chip limit), the library's static scratch holds %zu",
                    need, ge::kBatchScratchBytes);
    if (nsteps == 0)
        return GE_OK;
    hipError_t e = hipSuccess;
    void *work = ge::batch_scratch(&e);
    if (!work)
        return hip_fail(e, "ge_solve_batch_static: scratch address");
    const ge::BatchArgs a = run_args(b, u, work, step0, nsteps);
    e = ge::launch_batch(b->prec, a, b->grid, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GE_OK : hip_fail(e, "ge_solve_batch_static: launch");
}

}  // extern "C"
