// Integrator kernels for mechanisms padded to S = 9 species (groups of 16 lanes).
#include "bdf_kernels.h"

BDFX_DEFINE_SIZE(9, 16)
