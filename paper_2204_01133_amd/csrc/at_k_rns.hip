// Tile-kernel instantiations of one kernel kind (compiled as its own unit).
#include "at_kernels.hpp"
AT_DEFINE_LAUNCHER(launch_rns, AT_VARIANTS_RNS64)
