// bdf_kernels.h -- kernels of the batched BDF integrator and their launchers.
//
// k_integrate: one lane group per cell.  In grid mode every group takes the
// cell of its grid index; in queue mode (persistent waves) a group pops cell
// indices from a global atomic counter until the list is exhausted, so lanes
// whose cell finished early take new work instead of idling while other
// cells of the same wave are still stepping (the lock-step limitation of the
// paper's batches, Sec. 2 and Sec. 3.3).
#pragma once

#include "bdf_device.h"

namespace bdfx {

template <int S, int G, typename LT>
__global__ void __launch_bounds__(256) k_integrate(Params P) {
  extern __shared__ double smem[];
  const int grp = threadIdx.x / G;
  const int li = threadIdx.x & (G - 1);
  const int gpb = blockDim.x / G;
  double *lds = smem + static_cast<int64_t>(grp) * P.lds_doubles;
  // grid mode: one pass with the group's own index; queue mode: pop `chunk`
  // consecutive list entries at a time until the list is exhausted
  int64_t next = 0, stop = 0;
  if (!P.use_queue) {
    next = static_cast<int64_t>(blockIdx.x) * gpb + grp;
    stop = next + 1;
  }
  for (;;) {
    if (next >= stop) {
      if (!P.use_queue) break;
      unsigned int base = 0;
      if (li == 0) base = atomicAdd(P.queue, static_cast<unsigned int>(P.chunk));
      next = __shfl(base, 0, G);
      stop = next + P.chunk;
    }
    if (next >= P.n_list) break;
    const int64_t cell = P.list ? P.list[next] : next;
    ++next;
    integrate_cell<S, G, LT>(P, cell, li, lds);
  }
}

struct LaunchCfg {
  int grid, block;
  size_t lds_bytes;
};

template <int S, int G>
hipError_t launch_integrate(const Params &P, bool fp32, const LaunchCfg &c, hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL((k_integrate<S, G, float>), dim3(c.grid), dim3(c.block), c.lds_bytes, s, P);
  else
    hipLaunchKernelGGL((k_integrate<S, G, double>), dim3(c.grid), dim3(c.block), c.lds_bytes, s, P);
  return hipGetLastError();
}

template <int S, int G>
hipError_t occupancy_integrate(bool fp32, int block, size_t lds_bytes, int *blocks_per_cu) {
  if (fp32)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks_per_cu, reinterpret_cast<const void *>(&k_integrate<S, G, float>), block, lds_bytes);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks_per_cu, reinterpret_cast<const void *>(&k_integrate<S, G, double>), block, lds_bytes);
}

}  // namespace bdfx

// One translation unit per species size (compiled in parallel).
#define BDFX_DEFINE_SIZE(S, G)                                                                   \
  hipError_t bdfx_launch_s##S(const bdfx::Params &P, bool fp32, const bdfx::LaunchCfg &c,       \
                              hipStream_t s) {                                                   \
    return bdfx::launch_integrate<S, G>(P, fp32, c, s);                                          \
  }                                                                                              \
  hipError_t bdfx_occupancy_s##S(bool fp32, int block, size_t lds, int *out) {                   \
    return bdfx::occupancy_integrate<S, G>(fp32, block, lds, out);                               \
  }

#define BDFX_DECLARE_SIZE(S)                                                                     \
  hipError_t bdfx_launch_s##S(const bdfx::Params &P, bool fp32, const bdfx::LaunchCfg &c,       \
                              hipStream_t s);                                                    \
  hipError_t bdfx_occupancy_s##S(bool fp32, int block, size_t lds, int *out);
