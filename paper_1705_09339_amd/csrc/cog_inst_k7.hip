// Kernels and launchers of the mixture-size templates for K = 7.
#include "cog_kern.h"

namespace cog {
COG_INSTANTIATE_K(7)
}  // namespace cog
