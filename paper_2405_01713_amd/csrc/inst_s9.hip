// Integrator kernels for mechanisms padded to S = 9 species.
#include "bdf_kernels.h"

BDFX_DEFINE_SIZE(9)
