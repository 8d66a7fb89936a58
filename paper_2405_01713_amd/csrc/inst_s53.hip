// Integrator kernels for mechanisms padded to S = 53 species (groups of 64 lanes).
#include "bdf_kernels.h"

BDFX_DEFINE_SIZE(53, 64)
