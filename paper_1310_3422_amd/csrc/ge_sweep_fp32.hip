// The per-tile sweep kernels in FP32 and in the compensated FP32 pair.
#include "ge_sweep_kernels.h"

namespace ge {

hipError_t launch_tiles_fp32(bool comp, int k, int nw, bool src, const TileArgs &a,
                             hipStream_t stream, const SideStream *side)
{
    if (comp) {
        if (k == 4) return launch_nw<float, 4, true>(nw, src, a, stream, side);
        if (k == 8) return launch_nw<float, 8, true>(nw, src, a, stream, side);
        if (k == 16) return launch_nw<float, 16, true>(nw, src, a, stream, side);
        return hipErrorInvalidValue;
    }
    if (k == 4) return launch_nw<float, 4, false>(nw, src, a, stream, side);
    if (k == 8) return launch_nw<float, 8, false>(nw, src, a, stream, side);
    if (k == 16) return launch_nw<float, 16, false>(nw, src, a, stream, side);
    if (k == 32) return launch_nw<float, 32, false>(nw, src, a, stream, side);
    return hipErrorInvalidValue;
}

}  // namespace ge
