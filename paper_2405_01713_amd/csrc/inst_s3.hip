// Integrator kernels for mechanisms padded to S = 3 species (groups of 4 lanes).
#include "bdf_kernels.h"

BDFX_DEFINE_SIZE(3, 4)
