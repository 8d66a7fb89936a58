// Integrator kernels for mechanisms padded to S = 16 species (groups of 16 lanes).
#include "bdf_kernels.h"

BDFX_DEFINE_SIZE(16, 16)
