// Integrator kernels for mechanisms padded to S = 4 species (groups of 4 lanes).
#include "bdf_kernels.h"

BDFX_DEFINE_SIZE(4, 4)
