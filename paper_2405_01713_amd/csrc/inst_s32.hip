// Integrator kernels for mechanisms padded to S = 32 species.
#include "bdf_kernels.h"

BDFX_DEFINE_SIZE(32)
