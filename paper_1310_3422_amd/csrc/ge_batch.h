// Internal interface of the persistent batch sweep (ge_batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ge {

constexpr int kBatchWaves = 16;   // waves per workgroup of the batch kernel

// One rod, as the device sees it.
struct BatchRod {
    int64_t off;              // element offset of the rod's first point in u
    int64_t n;                // interior points
    double c1, c2, cs;        // (r+r^2)/(1+2r), r^2/(1+2r), r/(1+r)
    double gl, gr;            // constant wall values
    int64_t woff;             // rod above the on-chip limit: element offset of
                              // its second level buffer in u2; else -1
};

// One unit of work for a workgroup: rods sharing points-per-lane k, each
// owning a contiguous range of the workgroup's waves (-1: wave idle).
// halo = 1: the rods' waves overlap by one lane on each side and exchange
// those lanes every k-1 levels; halo = 0: adjacent waves exchange their edge
// values every level; halo = 2: one rod too long for the workgroup's
// registers (wave_rod[0]), swept in passes of at most BatchArgs::long_depth
// levels over single-wave windows of 64k points with halos, ping-ponging
// between u and the workspace's second level buffer.
struct BatchTask {
    int32_t k;
    int32_t halo;
    int32_t wave_rod[kBatchWaves];   // rod index per wave
    int32_t wave_idx[kBatchWaves];   // wave index within its rod
};

struct BatchArgs {
    void *u;                  // packed state (s block; e block at estride)
    const BatchRod *rods;
    const BatchTask *tasks;   // largest first
    int *counter;             // queue head, reset by a kernel before each run
    int64_t estride;          // FP32C: element offset of the e block
    int64_t step0;
    int32_t nsteps;
    int32_t ntasks;
    int32_t sync;             // 1: workgroup barrier per level; 2: neighbour flags;
                              // 3: halo lanes (tasks with halo = 0 use flags)
    int32_t wait_polls;       // polls before a neighbour wait gives up
    int *status;              // host-mapped status words (StatusWord), or null
    void *u2;                 // second level buffers of the long rods (s block,
                              // then the e block at estride2 for FP32C)
    int64_t estride2;
    int32_t long_depth;       // levels per pass of a long-rod task
    int32_t long_halo;        // window points each side of its cores
};

// Points per lane of the single-wave windows of long-rod tasks.
constexpr int batch_long_k(int prec) { return prec == 1 ? 32 : 16; }

// Waves a rod of n points needs at k points per lane when neighbouring
// waves overlap by one lane (halo tasks): 64k points for the first wave and
// 62k new points for each further one.
__host__ __device__ inline int halo_waves(int64_t n, int k)
{
    const int64_t w = 64 * (int64_t)k, c = 62 * (int64_t)k;
    return n <= w ? 1 : (int)(1 + (n - w + c - 1) / c);
}

// Where the waves of a halo task's rod start: wave j at 62 k j, except the
// last, which ends at the right wall node rounded up to a 16-byte boundary
// (so its start stays even and aligned).  `fits`: the rod has two or more
// waves and the last window does not reach into its neighbour's duplicated
// lane; only such rods go to halo tasks.
struct HaloLayout {
    int64_t n;
    int k, m;
    int64_t last;
    bool fits;
    __host__ __device__ HaloLayout(int64_t n_, int k_) : n(n_), k(k_), m(halo_waves(n_, k_))
    {
        last = (int64_t)(m - 1) * 62 * k;
        fits = false;
        if (m >= 2) {
            const int64_t r = (n - 64 * (int64_t)k + 3) / 4 * 4;
            const int64_t need = m == 2 ? 0 : (int64_t)(m - 2) * 62 * k + k;
            if (r >= need) {
                last = r;
                fits = true;
            }
        }
    }
    __host__ __device__ int64_t start(int j) const
    {
        return j == m - 1 ? last : (int64_t)j * 62 * k;
    }
};

hipError_t launch_batch(int prec, const BatchArgs &a, int grid, hipStream_t stream);

// Library-owned scratch of the allocation-free entry point: a file-scope
// device array of kBatchScratchBytes per GPU (the queue head at byte 0, the
// long rods' second level buffers from byte 256).  batch_scratch returns its
// device address on the current device, looked up once per device.
constexpr size_t kBatchScratchBytes = (size_t)32 << 20;
void *batch_scratch(hipError_t *err);
int batch_max_k(int prec);

}  // namespace ge
