// Instantiations of the restart-residual and Richardson products, both value types.
#include "krylov_tiled.hpp"

namespace ipi {
void tiled_other(int var, bool fp32, const tiled::TileParams& p, int lanes, int vec, int nb, hipStream_t st) {
    using namespace tiled;
    if (var == kResid) {
        if (fp32) {
            if (vec >= 4) launch_tiled_lanes<float, 4, kResid>(p, lanes, nb, 1, st);
            else if (vec >= 2) launch_tiled_lanes<float, 2, kResid>(p, lanes, nb, 1, st);
            else launch_tiled_lanes<float, 1, kResid>(p, lanes, nb, 1, st);
        } else {
            if (vec >= 2) launch_tiled_lanes<double, 2, kResid>(p, lanes, nb, 1, st);
            else launch_tiled_lanes<double, 1, kResid>(p, lanes, nb, 1, st);
        }
    } else if (var == kApply) {
        if (fp32) {
            if (vec >= 4) launch_tiled_lanes<float, 4, kApply>(p, lanes, nb, 2, st);
            else if (vec >= 2) launch_tiled_lanes<float, 2, kApply>(p, lanes, nb, 2, st);
            else launch_tiled_lanes<float, 1, kApply>(p, lanes, nb, 2, st);
        } else {
            if (vec >= 2) launch_tiled_lanes<double, 2, kApply>(p, lanes, nb, 2, st);
            else launch_tiled_lanes<double, 1, kApply>(p, lanes, nb, 2, st);
        }
    } else {
        if (fp32) {
            if (vec >= 4) launch_tiled_lanes<float, 4, kRich>(p, lanes, nb, 1, st);
            else if (vec >= 2) launch_tiled_lanes<float, 2, kRich>(p, lanes, nb, 1, st);
            else launch_tiled_lanes<float, 1, kRich>(p, lanes, nb, 1, st);
        } else {
            if (vec >= 2) launch_tiled_lanes<double, 2, kRich>(p, lanes, nb, 1, st);
            else launch_tiled_lanes<double, 1, kRich>(p, lanes, nb, 1, st);
        }
    }
}
}  // namespace ipi
