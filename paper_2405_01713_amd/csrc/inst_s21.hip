// Integrator kernels for mechanisms padded to S = 21 species (groups of 32 lanes).
#include "bdf_kernels.h"

BDFX_DEFINE_SIZE(21, 32)
