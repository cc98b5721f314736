// Kernels and launchers of the mixture-size templates for K = 6.
#include "cog_kern.h"

namespace cog {
COG_INSTANTIATE_K(6)
}  // namespace cog
