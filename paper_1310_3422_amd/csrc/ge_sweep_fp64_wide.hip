// The per-tile sweep kernels in FP64 at 32 and 64 points per lane.
#include "ge_sweep_kernels.h"

namespace ge {

hipError_t launch_tiles_fp64_wide(int k, int nw, bool src, const TileArgs &a,
                                  hipStream_t stream, const SideStream *side)
{
    if (k == 32) return launch_nw<double, 32, false>(nw, src, a, stream, side);
    if (k == 64) return launch_nw<double, 64, false>(nw, src, a, stream, side);
    return hipErrorInvalidValue;
}

}  // namespace ge
