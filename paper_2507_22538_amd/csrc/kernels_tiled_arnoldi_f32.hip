// Instantiations of the fused Arnoldi product (J_pi v_j with the Gram-Schmidt dots), float32 P_pi values.
#include "krylov_tiled.hpp"

namespace ipi {
void tiled_arnoldi_f32(const tiled::TileParams& p, int lanes, int vec, int nb, int mj, hipStream_t st) {
    using namespace tiled;
    if (vec >= 4) launch_tiled_lanes<float, 4, kArnoldi>(p, lanes, nb, mj, st);
    else if (vec >= 2) launch_tiled_lanes<float, 2, kArnoldi>(p, lanes, nb, mj, st);
    else launch_tiled_lanes<float, 1, kArnoldi>(p, lanes, nb, mj, st);
}
}  // namespace ipi
