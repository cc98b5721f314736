// Kernels and launchers of the mixture-size templates for K = 8.
#include "cog_kern.h"

namespace cog {
COG_INSTANTIATE_K(8)
}  // namespace cog
