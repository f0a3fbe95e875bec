// The per-tile sweep kernels in FP64 at 2 to 20 points per lane.
#include "ge_sweep_kernels.h"

namespace ge {

hipError_t launch_tiles_fp64_narrow(int k, int nw, bool src, const TileArgs &a,
                                    hipStream_t stream, const SideStream *side)
{
    if (k == 2) return launch_nw<double, 2, false>(nw, src, a, stream, side);
    if (k == 4) return launch_nw<double, 4, false>(nw, src, a, stream, side);
    if (k == 8) return launch_nw<double, 8, false>(nw, src, a, stream, side);
    if (k == 16) return launch_nw<double, 16, false>(nw, src, a, stream, side);
    if (k == 20) return launch_nw<double, 20, false>(nw, src, a, stream, side);
    return hipErrorInvalidValue;
}

}  // namespace ge
