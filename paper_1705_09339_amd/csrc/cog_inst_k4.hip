// Kernels and launchers of the mixture-size templates for K = 4.
#include "cog_kern.h"

namespace cog {
COG_INSTANTIATE_K(4)
}  // namespace cog
