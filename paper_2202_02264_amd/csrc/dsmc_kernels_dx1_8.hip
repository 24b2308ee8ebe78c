// Kernels of the dSMC combine tree for state dimensions padded to 1, 2, 4, 8, fp32 and fp64.
#include "dsmc_kernels_impl.h"

namespace dsmc {
DSMC_INSTANTIATE(1, float, _f32)
DSMC_INSTANTIATE(1, double, _f64)
DSMC_INSTANTIATE(2, float, _f32)
DSMC_INSTANTIATE(2, double, _f64)
DSMC_INSTANTIATE(4, float, _f32)
DSMC_INSTANTIATE(4, double, _f64)
DSMC_INSTANTIATE(8, float, _f32)
DSMC_INSTANTIATE(8, double, _f64)
}  // namespace dsmc
