// Kernels of the dSMC combine tree for state dimensions padded to 16, fp32 and fp64.
#include "dsmc_kernels_impl.h"

namespace dsmc {
DSMC_INSTANTIATE(16, float, _f32)
DSMC_INSTANTIATE(16, double, _f64)
}  // namespace dsmc
