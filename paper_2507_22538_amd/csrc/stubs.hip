// temporary: pieces not yet written
#include "internal.hpp"
namespace ipi {
int default_spmv_lanes(const ipi_mdp_s*, bool) { return 1; }
int default_spmv_spt(const ipi_mdp_s*, int) { return 256; }
ipi_status solve_single(ipi_mdp_s*, const ipi_solve_opts&, double*, int32_t*, ipi_solve_info*, hipStream_t) {
    throw Error(IPI_E_INVALID_ARG, "not implemented");
}
ipi_status solve_batch(int, ipi_mdp_s* const*, const ipi_solve_opts*, double* const*, int32_t* const*,
                       ipi_solve_info*, ipi_status*, hipStream_t) {
    throw Error(IPI_E_INVALID_ARG, "not implemented");
}
ipi_status autotune(ipi_mdp_s*, bool, const char*, hipStream_t) { throw Error(IPI_E_INVALID_ARG, "not implemented"); }
}
