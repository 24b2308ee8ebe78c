// Kernels of the dSMC combine tree for state dimensions padded to 32, fp32.
#include "dsmc_kernels_impl.h"

namespace dsmc {
DSMC_INSTANTIATE(32, float, _f32)
}  // namespace dsmc
