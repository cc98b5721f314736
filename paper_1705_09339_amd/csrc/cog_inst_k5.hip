// Kernels and launchers of the mixture-size templates for K = 5.
#include "cog_kern.h"

namespace cog {
COG_INSTANTIATE_K(5)
}  // namespace cog
