// Kernels and launchers of the mixture-size templates for K = 1.
#include "cog_kern.h"

namespace cog {
COG_INSTANTIATE_K(1)
}  // namespace cog
