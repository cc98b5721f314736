// Kernels and launchers of the mixture-size templates for K = 3.
#include "cog_kern.h"

namespace cog {
COG_INSTANTIATE_K(3)
}  // namespace cog
