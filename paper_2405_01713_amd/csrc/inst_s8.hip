// Integrator kernels for mechanisms padded to S = 8 species (groups of 8 lanes).
#include "bdf_kernels.h"

BDFX_DEFINE_SIZE(8, 8)
