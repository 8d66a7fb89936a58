// Both bins of a batch that mixes a 53-species and a 9-species mechanism in
// one persistent launch.
#include "bdf_kernels.h"

BDFX_DEFINE_PAIR(53, 9)
