// Kernels of the dSMC combine tree for state dimensions padded to 32, fp64.
#include "dsmc_kernels_impl.h"

namespace dsmc {
DSMC_INSTANTIATE(32, double, _f64)
}  // namespace dsmc
