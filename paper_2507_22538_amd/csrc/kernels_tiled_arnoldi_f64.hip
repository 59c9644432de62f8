// Instantiations of the fused Arnoldi product (J_pi v_j with the Gram-Schmidt dots), FP64 P_pi values.
#include "krylov_tiled.hpp"

namespace ipi {
void tiled_arnoldi_f64(const tiled::TileParams& p, int lanes, int vec, int nb, int mj, hipStream_t st) {
    using namespace tiled;
    if (vec >= 2) launch_tiled_lanes<double, 2, kArnoldi>(p, lanes, nb, mj, st);
    else launch_tiled_lanes<double, 1, kArnoldi>(p, lanes, nb, mj, st);
}
}  // namespace ipi
