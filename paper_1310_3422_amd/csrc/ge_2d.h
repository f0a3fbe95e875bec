// Two-dimensional extension (ge_2d.hip): launches of `depth` levels (then
// single levels for the rest), each level the x-level of every row then the
// y-level of every column, ping-ponging between u and work; after an odd
// number of launches the result is copied back into u.
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
    int depth;               // levels per launch: 1, 2 or 4
};

hipError_t launch_2d(int prec, const Grid2dArgs &a, hipStream_t stream);

}  // namespace ge
