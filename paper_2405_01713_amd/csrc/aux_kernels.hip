// aux_kernels.hip -- small kernels around the integrator: the outer-step
// perturbation of the split state and a fill kernel used to reset work-queue
// counters (a kernel rather than a memset, so that it can live in a captured
// graph).
#include "bdf_kernels.h"

namespace bdfx {

// SplitMix64 output for generator state x (Steele, Lea & Flood 2014): add the
// golden gamma, then the variant-13 mixer.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// y_i <- max(0, y_i (1 + amp u_i)), u uniform in [-1, 1) keyed by
// (seed, step, cell, species); then a common factor restores sum_i w_i y_i.
// Plain (non-contracted) IEEE operations in a fixed order so the result is
// reproducible bit for bit.  One thread per cell.
__global__ void __launch_bounds__(256) k_perturb(Params P, uint64_t seed, int64_t step, double amp) {
#pragma clang fp contract(off)
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= P.n_list) return;
  const int64_t cell = P.list ? P.list[idx] : idx;
  double *yc = P.y + cell * P.ldy;
  const double *w = P.mech.w;
  const int S = P.mech.S;  // species only (a temperature entry is not perturbed)
  const uint64_t key = splitmix64(seed);
  double before = 0.0, after = 0.0;
  for (int i = 0; i < S; ++i) before = before + w[i] * yc[i];
  for (int i = 0; i < S; ++i) {
    const uint64_t ctr = (static_cast<uint64_t>(step) << 40) + (static_cast<uint64_t>(cell) << 8) +
                         static_cast<uint64_t>(i);
    const uint64_t v = splitmix64(key ^ ctr);
    const double u01 = static_cast<double>(v >> 11) * (1.0 / 9007199254740992.0);
    const double u = 2.0 * u01 - 1.0;
    const double y = yc[i] * (1.0 + amp * u);
    yc[i] = y > 0.0 ? y : 0.0;
    after = after + w[i] * yc[i];
  }
  if (after > 0.0) {
    const double s = before / after;
    for (int i = 0; i < S; ++i) yc[i] = yc[i] * s;
  }
}

// out[r] = sum over the cells of list (length n) of pbar[cell][r]; one block
// per reaction, fixed summation order (deterministic).
__global__ void __launch_bounds__(256) k_sum_cells(const double *pbar, int ldp, const int32_t *list,
                                                   int64_t n, int R, double *out) {
  __shared__ double part[256];
  const int r = blockIdx.x;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const int64_t c = list ? list[i] : i;
    acc += pbar[c * ldp + r];
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = part[0];
}

__global__ void k_fill_u32(uint32_t *p, int n, uint32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace bdfx

hipError_t bdfx_launch_perturb(const bdfx::Params &P, uint64_t seed, int64_t step, double amp,
                               hipStream_t s) {
  const int block = 256;
  const int64_t grid = (P.n_list + block - 1) / block;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(bdfx::k_perturb, dim3(static_cast<unsigned>(grid)), dim3(block), 0, s, P,
                     seed, step, amp);
  return hipGetLastError();
}

hipError_t bdfx_launch_sum_cells(const double *pbar, int ldp, const int32_t *list, int64_t n, int R,
                                 double *out, hipStream_t s) {
  hipLaunchKernelGGL(bdfx::k_sum_cells, dim3(R), dim3(256), 0, s, pbar, ldp, list, n, R, out);
  return hipGetLastError();
}

// dst[i][0..S) <- y[list[i]][0..S) (save) or the reverse (restore), i < n.
__global__ void __launch_bounds__(256) k_copy_rows(double *y, int ldy, const int32_t *list, int64_t n,
                                                   int S, double *dst, bool restore) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n * S) return;
  const int64_t i = idx / S;
  const int k = static_cast<int>(idx - i * S);
  const int64_t cell = list ? list[i] : i;
  if (restore)
    y[cell * ldy + k] = dst[i * S + k];
  else
    dst[i * S + k] = y[cell * ldy + k];
}

hipError_t bdfx_launch_copy_rows(double *y, int ldy, const int32_t *list, int64_t n, int S,
                                 double *dst, bool restore, hipStream_t s) {
  const int64_t total = n * S;
  if (total <= 0) return hipSuccess;
  const int64_t blocks = (total + 255) / 256;
  hipLaunchKernelGGL(k_copy_rows, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, y, ldy, list,
                     n, S, dst, restore);
  return hipGetLastError();
}

hipError_t bdfx_launch_fill_u32(uint32_t *p, int n, uint32_t v, hipStream_t s) {
  hipLaunchKernelGGL(bdfx::k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
