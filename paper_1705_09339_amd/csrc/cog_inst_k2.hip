// Kernels and launchers of the mixture-size templates for K = 2.
#include "cog_kern.h"

namespace cog {
COG_INSTANTIATE_K(2)
}  // namespace cog
