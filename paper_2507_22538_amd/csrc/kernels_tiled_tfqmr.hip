// Instantiations of the two fused TFQMR products (kTfqW: J q with the w, d, x
// updates; kTfqV: J u with the v update), both value types.
#include "krylov_tiled.hpp"

namespace ipi {
void tiled_tfqmr(int var, bool fp32, const tiled::TileParams& p, int lanes, int vec, int nb, hipStream_t st) {
    using namespace tiled;
    if (var == kTfqW) {
        if (fp32) {
            if (vec >= 4) launch_tiled_lanes<float, 4, kTfqW>(p, lanes, nb, 2, st);
            else if (vec >= 2) launch_tiled_lanes<float, 2, kTfqW>(p, lanes, nb, 2, st);
            else launch_tiled_lanes<float, 1, kTfqW>(p, lanes, nb, 2, st);
        } else {
            if (vec >= 2) launch_tiled_lanes<double, 2, kTfqW>(p, lanes, nb, 2, st);
            else launch_tiled_lanes<double, 1, kTfqW>(p, lanes, nb, 2, st);
        }
    } else {
        if (fp32) {
            if (vec >= 4) launch_tiled_lanes<float, 4, kTfqV>(p, lanes, nb, 1, st);
            else if (vec >= 2) launch_tiled_lanes<float, 2, kTfqV>(p, lanes, nb, 1, st);
            else launch_tiled_lanes<float, 1, kTfqV>(p, lanes, nb, 1, st);
        } else {
            if (vec >= 2) launch_tiled_lanes<double, 2, kTfqV>(p, lanes, nb, 1, st);
            else launch_tiled_lanes<double, 1, kTfqV>(p, lanes, nb, 1, st);
        }
    }
}
}  // namespace ipi
