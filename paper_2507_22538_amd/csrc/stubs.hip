// temporary: pieces not yet written
#include "internal.hpp"
namespace ipi {
ipi_status autotune(ipi_mdp_s*, bool, const char*, hipStream_t) { throw Error(IPI_E_INVALID_ARG, "not implemented"); }
}
