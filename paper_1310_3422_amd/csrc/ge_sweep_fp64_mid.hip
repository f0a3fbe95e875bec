// The per-tile sweep kernels in FP64 at 24 and 28 points per lane.
#include "ge_sweep_kernels.h"

namespace ge {

hipError_t launch_tiles_fp64_mid(int k, int nw, bool src, const TileArgs &a,
                                 hipStream_t stream, const SideStream *side)
{
    if (k == 24) return launch_nw<double, 24, false>(nw, src, a, stream, side);
    if (k == 28) return launch_nw<double, 28, false>(nw, src, a, stream, side);
    return hipErrorInvalidValue;
}

}  // namespace ge
