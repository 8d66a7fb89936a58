// Integrator kernels for mechanisms padded to S = 64 species (groups of 64 lanes).
#include "bdf_kernels.h"

BDFX_DEFINE_SIZE(64, 64)
