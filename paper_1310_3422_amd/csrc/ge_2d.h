// Two-dimensional extension (ge_2d.hip): one launch per level, each the
// x-level of every row then the y-level of every column, ping-ponging
// between u and work; after an odd number of levels the result is copied
// back into u.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ge {

struct Grid2dArgs {
    void *u;                 // ny rows of nx values; holds the result
    void *work;              // same size, distinct from u
    int64_t nx, ny, step0, nsteps;
    double rx, ry;           // tau/hx^2, tau/hy^2
    double gw, ge, gs, gn;   // constant walls: west, east, south, north
};

hipError_t launch_2d(int prec, const Grid2dArgs &a, hipStream_t stream);

}  // namespace ge
