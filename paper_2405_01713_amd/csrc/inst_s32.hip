// Integrator kernels for mechanisms padded to S = 32 species (groups of 32 lanes).
#include "bdf_kernels.h"

BDFX_DEFINE_SIZE(32, 32)
