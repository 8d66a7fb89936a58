// typical.hip -- typical-value absolute tolerances (Sec. 4.1.3, Eq. (9)):
// atol_i = eta * (min_c y_ci + max_c y_ci) / 2 over the cells of a mechanism.
//
// Two kernels per call.  k_extremes streams the state rows of one mechanism
// once (the HBM-bound part): a wave covers floor(64 / S) cells per pass, lane
// l holding species l mod S of cell l / S, so the rows of consecutive cells
// are read as one contiguous run; each block (16 waves, at most 256 blocks per
// mechanism) leaves its per-species extremes in a partial array.  k_typical
// combines the partials of every mechanism and writes the tolerances.  Minimum
// and maximum are exact, so the result does not depend on the order in which
// cells are visited.  A NaN entry makes both extremes NaN (as a plain minimum
// over the values would).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bdf_device.h"
#include "bdfx.h"

namespace bdfx {

constexpr int kExtBlock = 1024;  // threads per k_extremes block
constexpr int kExtUnroll = 8;   // passes per loop iteration (loads in flight)

__device__ __forceinline__ double lo_of(double a, double v) { return (v < a || v != v) ? v : a; }
__device__ __forceinline__ double hi_of(double a, double v) { return (v > a || v != v) ? v : a; }

// part[block][0][i] = min, part[block][1][i] = max over this block's cells.
__global__ void __launch_bounds__(kExtBlock) k_extremes(const double *y, int ldy, const int32_t *list,
                                                        int64_t n, int S, double *part) {
  __shared__ double lo_s[kExtBlock], hi_s[kExtBlock];
  const int lane = threadIdx.x & (kWave - 1);
  const int wib = threadIdx.x / kWave;
  const int per = kWave / S;  // cells per wave pass
  const int sub = lane / S, sp = lane - sub * S;
  const bool act = sub < per;
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (kExtBlock / kWave);
  const int64_t w0 = static_cast<int64_t>(blockIdx.x) * (kExtBlock / kWave) + wib;
  const int64_t passes = (n + per - 1) / per;
  double lo = __builtin_huge_val(), hi = -__builtin_huge_val();
  for (int64_t p0 = w0; p0 < passes; p0 += waves * kExtUnroll) {
    double v[kExtUnroll];
#pragma unroll
    for (int u = 0; u < kExtUnroll; ++u) {
      const int64_t idx = (p0 + u * waves) * per + sub;
      v[u] = __builtin_nan("");
      if (act && p0 + u * waves < passes && idx < n) {
        const int64_t c = list ? list[idx] : idx;
        v[u] = y[c * ldy + sp];
      }
    }
#pragma unroll
    for (int u = 0; u < kExtUnroll; ++u) {
      const int64_t idx = (p0 + u * waves) * per + sub;
      if (act && p0 + u * waves < passes && idx < n) {
        lo = lo_of(lo, v[u]);
        hi = hi_of(hi, v[u]);
      }
    }
  }
  lo_s[threadIdx.x] = lo;
  hi_s[threadIdx.x] = hi;
  __syncthreads();
  // Two-level combine.  First thread t < (waves per block) S takes wave
  // t / S, species t mod S, over that wave's lanes holding the species
  // (sp, sp + S, ...); then thread t < S takes species t over the waves.
  constexpr int kExtWaves = kExtBlock / kWave;
  __shared__ double lo_w[kExtWaves * kWave], hi_w[kExtWaves * kWave];
  if (threadIdx.x < kExtWaves * S) {
    const int w = threadIdx.x / S, s = threadIdx.x - w * S;
    double l = __builtin_huge_val(), h = -__builtin_huge_val();
    for (int k = 0; k < per; ++k) {
      l = lo_of(l, lo_s[w * kWave + k * S + s]);
      h = hi_of(h, hi_s[w * kWave + k * S + s]);
    }
    lo_w[threadIdx.x] = l;
    hi_w[threadIdx.x] = h;
  }
  __syncthreads();
  if (threadIdx.x < S) {
    double l = __builtin_huge_val(), h = -__builtin_huge_val();
    for (int w = 0; w < kExtWaves; ++w) {
      l = lo_of(l, lo_w[w * S + threadIdx.x]);
      h = hi_of(h, hi_w[w * S + threadIdx.x]);
    }
    part[(static_cast<int64_t>(blockIdx.x) * 2) * kWave + threadIdx.x] = l;
    part[(static_cast<int64_t>(blockIdx.x) * 2 + 1) * kWave + threadIdx.x] = h;
  }
}

struct TypicalArgs {
  int32_t n_mech, ldt;               // mechanisms; row length of the outputs
  int32_t S[BDFX_MAX_MECH];          // species of each mechanism
  int32_t nblk[BDFX_MAX_MECH];       // k_extremes blocks that ran (0: no cells)
  int64_t part_off[BDFX_MAX_MECH];   // offset (doubles) of its partials
};

// One block per mechanism of kTypThreads threads: thread t takes species
// t mod S and every (kTypThreads / S)-th partial block from t / S on, so all
// threads work whatever S is; the chunks' extremes are combined in LDS in two
// levels, then typ = 0.5 (min + max), atol = (typ > 0 ? typ : 1) eta.  Entries
// beyond the mechanism's species (and all of a mechanism without cells) get
// typ = 0, atol = eta.  Minimum and maximum are exact: the partition changes no bit.
constexpr int kTypThreads = 1024;

__global__ void __launch_bounds__(kTypThreads) k_typical(TypicalArgs a, const double *part,
                                                         double eta, double *atol, double *typ) {
#pragma clang fp contract(off)
  __shared__ double lo_s[kTypThreads], hi_s[kTypThreads];
  const int m = blockIdx.x;
  const int S = a.S[m];
  const int t = threadIdx.x;
  const int nchunk = kTypThreads / S;  // S <= 64: at least 16 chunks
  const int i = t % S, g = t / S;
  const double *pm = part + a.part_off[m];
  double l = __builtin_huge_val(), h = -__builtin_huge_val();
  if (g < nchunk) {
#pragma unroll 4
    for (int b = g; b < a.nblk[m]; b += nchunk) {
      l = lo_of(l, pm[(static_cast<int64_t>(b) * 2) * kWave + i]);
      h = hi_of(h, pm[(static_cast<int64_t>(b) * 2 + 1) * kWave + i]);
    }
  }
  lo_s[t] = l;
  hi_s[t] = h;
  __syncthreads();
  // two-level combine: thread t < nq S takes species t mod S over chunks
  // 8q .. 8q + 7 (q = t / S), then thread t < S over the nq groups
  constexpr int kTypGroup = 8;
  const int nq = (nchunk + kTypGroup - 1) / kTypGroup;  // nq S <= 1024 / 8 + 64
  __shared__ double lo_q[kTypThreads / kTypGroup + kWave], hi_q[kTypThreads / kTypGroup + kWave];
  if (t < nq * S) {
    const int q = t / S, s = t - q * S;
    const int k1 = (q + 1) * kTypGroup < nchunk ? (q + 1) * kTypGroup : nchunk;
    double lq = __builtin_huge_val(), hq = -__builtin_huge_val();
    for (int k = q * kTypGroup; k < k1; ++k) {
      lq = lo_of(lq, lo_s[k * S + s]);
      hq = hi_of(hq, hi_s[k * S + s]);
    }
    lo_q[t] = lq;
    hi_q[t] = hq;
  }
  __syncthreads();
  if (t < a.ldt) {  // ldt <= 64: thread t writes entry t
    double tv = 0.0, at = eta;
    if (t < S && a.nblk[m] > 0) {
      double lt = lo_q[t], ht = hi_q[t];
      for (int q = 1; q < nq; ++q) {
        lt = lo_of(lt, lo_q[q * S + t]);
        ht = hi_of(ht, hi_q[q * S + t]);
      }
      tv = 0.5 * (lt + ht);
      at = (tv > 0.0 ? tv : 1.0) * eta;
    }
    atol[static_cast<int64_t>(m) * a.ldt + t] = at;
    if (typ) typ[static_cast<int64_t>(m) * a.ldt + t] = tv;
  }
}

}  // namespace bdfx

// blocks of k_extremes for n cells of S species (at most max_blocks)
int bdfx_extremes_blocks(int64_t n, int S, int max_blocks) {
  if (n <= 0 || S < 1 || S > bdfx::kWave) return 0;
  const int per = bdfx::kWave / S;
  const int64_t passes = (n + per - 1) / per;
  const int64_t waves_needed = (passes + bdfx::kExtUnroll - 1) / bdfx::kExtUnroll;
  const int64_t blocks = (waves_needed + bdfx::kExtBlock / bdfx::kWave - 1) / (bdfx::kExtBlock / bdfx::kWave);
  return static_cast<int>(blocks < max_blocks ? blocks : max_blocks);
}

hipError_t bdfx_launch_extremes(const double *y, int ldy, const int32_t *list, int64_t n, int S,
                                int blocks, double *part, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(bdfx::k_extremes, dim3(blocks), dim3(bdfx::kExtBlock), 0, s, y, ldy, list, n,
                     S, part);
  return hipGetLastError();
}

hipError_t bdfx_launch_typical(int n_mech, int ldt, const int32_t *S, const int32_t *nblk,
                               const int64_t *part_off, const double *part, double eta, double *atol,
                               double *typ, hipStream_t s) {
  bdfx::TypicalArgs a{};
  a.n_mech = n_mech;
  a.ldt = ldt;
  for (int m = 0; m < n_mech && m < BDFX_MAX_MECH; ++m) {
    a.S[m] = S[m];
    a.nblk[m] = nblk[m];
    a.part_off[m] = part_off[m];
  }
  hipLaunchKernelGGL(bdfx::k_typical, dim3(n_mech), dim3(bdfx::kTypThreads), 0, s, a,
                     part, eta, atol, typ);
  return hipGetLastError();
}
