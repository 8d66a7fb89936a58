// bdf_kernels.h -- kernels of the batched BDF integrator and their launchers.
//
// k_integrate: one wavefront per cell.  In grid mode every wave takes the
// cell of its grid index; in queue mode (persistent waves) a wave pops cell
// indices from a global atomic counter until the list is exhausted, so waves
// whose cells finish early take new work instead of leaving their SIMD slot
// to the tail (the load imbalance of lock-step batches, Sec. 2 and 4.1.1).
#pragma once

#include "bdf_device.h"

namespace bdfx {

// MINW: minimum resident waves per SIMD the register allocation must allow
// (1 = compiler's choice; 3 = at most 168 VGPRs, 4 = at most 128, 5 = at
// most 96, spilling if needed).  TAB: placement of the reaction tables
// (kTab*).  G: cells per wave (2: each half-wave integrates its own cell,
// S <= 32); each group has its own LDS area of P.lds_doubles and pops its
// own cells.  With the tables
// in global memory, wave w of the grid owns rate-constant slot w (the host
// guarantees that the grid's waves fit the slot array).  ABC: every reaction
// is A + B <=> C (see rhs_reaction).  TH: non-isothermal cells (temperature
// as the last state entry, rates re-evaluated from it).  LIN: linear solver
// of the Newton iteration (kLin*: Newton matrix from the analytic Jacobian or
// from difference quotients, or matrix-free GMRES; LT is unused by GMRES).
// LOCK: lock-step batches (the paper's batches, Sec. 2): block k integrates
// batch k of P.batch consecutive list entries, one wave per cell, with one
// step size and one WRMS norm over the batch (BatchRed); the work queue then
// hands out batches.  Blocks of up to kMaxBatch waves.
template <int S, typename LT, int MINW, int TAB, int G, bool ABC, bool TH,
          int LIN = kLinAnalytic, bool LOCK = false>
__global__ void __launch_bounds__(LOCK ? kWave * kMaxBatch : 256, MINW) k_integrate(Params P) {
  extern __shared__ double smem[];
  const int wib = threadIdx.x / kWave;
  const Grp<G> W(threadIdx.x & (kWave - 1));
  const int wpb = blockDim.x / kWave;
  double *lds = smem + static_cast<int64_t>(wib * G + W.grp) * P.lds_doubles;
  if constexpr (LOCK) {
    static_assert(G == 1 && TAB == kTabLds, "lock-step batches: one cell per wave, tables in LDS");
    // the batch slots follow the waves' areas; slot 2 kMaxBatch holds the popped batch index
    double *slots = smem + static_cast<int64_t>(wpb) * P.lds_doubles;
    const int64_t n_batches = (P.n_list + wpb - 1) / wpb;
    int64_t b = P.use_queue ? -1 : blockIdx.x;
    for (;;) {
      __syncthreads();
      if (P.use_queue) {
        if (threadIdx.x == 0) slots[2 * kMaxBatch] = static_cast<double>(atomicAdd(P.queue, 1u));
        __syncthreads();
        b = static_cast<int64_t>(slots[2 * kMaxBatch]);
      }
      if (b >= n_batches) break;
      const int64_t first = b * wpb;
      const int nb = static_cast<int>(P.n_list - first < wpb ? P.n_list - first : wpb);
      BatchRed<true> br;
      br.slots = slots;
      br.wid = wib;
      br.nw = wpb;
      br.active = wib < nb;
      const int64_t idx = first + (br.active ? wib : 0);
      const int64_t cell = P.list ? P.list[idx] : idx;
      integrate_cell<S, LT, TAB, G, ABC, TH, LIN, true>(P, cell, W, lds, nullptr, br, nb);
      if (!P.use_queue) break;
    }
    return;
  }
  double *kk_slot = nullptr;
  if constexpr (TAB == kTabGlobal)
    kk_slot = P.kk_slots + ((static_cast<int64_t>(blockIdx.x) * wpb + wib) * G + W.grp) * (2 * P.mech.R);
  int64_t next = 0, stop = 0;
  if (!P.use_queue) {
    next = (static_cast<int64_t>(blockIdx.x) * wpb + wib) * G + W.grp;
    stop = next + 1;
  }
  for (;;) {
    if (next >= stop) {
      if (!P.use_queue) break;
      unsigned int base = 0;
      if (W.lane == 0) base = atomicAdd(P.queue, static_cast<unsigned int>(P.chunk));
      next = W.from_lane0(static_cast<int>(base));
      stop = next + P.chunk;
    }
    if (next >= P.n_list) break;
    const int64_t cell = P.list ? P.list[next] : next;
    ++next;
    integrate_cell<S, LT, TAB, G, ABC, TH, LIN>(P, cell, W, lds, kk_slot);
  }
}

// Two mechanism bins in one persistent launch (several mechanism sizes in one
// grid).  Each block holds PA.pair_waves waves for the larger mechanism (bin A,
// padded size SA, table placement TABA) followed by the rest of its waves for
// the smaller one (bin B, padded size SB, tables in LDS), each wave with an
// LDS area for its own bin.  A-waves pop cells of bin A and, once its queue is
// exhausted, cells of bin B (an A area holds a B cell); B-waves pop cells of
// bin B only.  The large cells start first; the small ones run beside them,
// in the issue slots the A-waves leave while they wait, and then in the tail
// of bin A.  Every cell runs the integrate_cell code of its own bin's launch
// (one cell per wave, A + B <=> C mechanisms, isothermal, direct solver with
// the analytic Jacobian), so results do not depend on the launch.
template <int SA, int SB, typename LT, int MINW, int TABA>
__global__ void __launch_bounds__(256, MINW) k_integrate_pair(Params PA, Params PB) {
  extern __shared__ double smem[];
  const int wib = threadIdx.x / kWave;
  const Grp<1> W(threadIdx.x & (kWave - 1));
  const int wa = PA.pair_waves;
  const bool is_a = wib < wa;
  double *lds = is_a ? smem + static_cast<int64_t>(wib) * PA.lds_doubles
                     : smem + static_cast<int64_t>(wa) * PA.lds_doubles +
                           static_cast<int64_t>(wib - wa) * PB.lds_doubles;
  double *kk_slot = nullptr;
  if constexpr (TABA == kTabGlobal)
    if (is_a) kk_slot = PA.kk_slots + (static_cast<int64_t>(blockIdx.x) * wa + wib) * (2 * PA.mech.R);
  int64_t next = 0, stop = 0;
  if (is_a) {
    for (;;) {
      if (next >= stop) {
        unsigned int base = 0;
        if (W.lane == 0) base = atomicAdd(PA.queue, static_cast<unsigned int>(PA.chunk));
        next = W.from_lane0(static_cast<int>(base));
        stop = next + PA.chunk;
      }
      if (next >= PA.n_list) break;
      const int64_t cell = PA.list ? PA.list[next] : next;
      ++next;
      integrate_cell<SA, LT, TABA, 1, true, false, kLinAnalytic>(PA, cell, W, lds, kk_slot);
    }
  }
  next = stop = 0;
  for (;;) {
    if (next >= stop) {
      unsigned int base = 0;
      if (W.lane == 0) base = atomicAdd(PB.queue, static_cast<unsigned int>(PB.chunk));
      next = W.from_lane0(static_cast<int>(base));
      stop = next + PB.chunk;
    }
    if (next >= PB.n_list) break;
    const int64_t cell = PB.list ? PB.list[next] : next;
    ++next;
    integrate_cell<SB, LT, kTabLds, 1, true, false, kLinAnalytic>(PB, cell, W, lds, nullptr);
  }
}

template <int SA, int SB>
const void *pair_kernel(bool fp32, int minw, int taba) {
  using F = const void *;
  if (minw >= 5) return nullptr;  // built for the budgets 0, 3 and 4
  const int w = minw >= 4 ? 2 : minw >= 3 ? 1 : 0;
  static const F t64[3][3] = {
      {F(&k_integrate_pair<SA, SB, double, 1, kTabRxGlobal>), F(&k_integrate_pair<SA, SB, double, 1, kTabLds>),
       F(&k_integrate_pair<SA, SB, double, 1, kTabGlobal>)},
      {F(&k_integrate_pair<SA, SB, double, 3, kTabRxGlobal>), F(&k_integrate_pair<SA, SB, double, 3, kTabLds>),
       F(&k_integrate_pair<SA, SB, double, 3, kTabGlobal>)},
      {F(&k_integrate_pair<SA, SB, double, 4, kTabRxGlobal>), F(&k_integrate_pair<SA, SB, double, 4, kTabLds>),
       F(&k_integrate_pair<SA, SB, double, 4, kTabGlobal>)}};
  static const F t32[3][3] = {
      {F(&k_integrate_pair<SA, SB, float, 1, kTabRxGlobal>), F(&k_integrate_pair<SA, SB, float, 1, kTabLds>),
       F(&k_integrate_pair<SA, SB, float, 1, kTabGlobal>)},
      {F(&k_integrate_pair<SA, SB, float, 3, kTabRxGlobal>), F(&k_integrate_pair<SA, SB, float, 3, kTabLds>),
       F(&k_integrate_pair<SA, SB, float, 3, kTabGlobal>)},
      {F(&k_integrate_pair<SA, SB, float, 4, kTabRxGlobal>), F(&k_integrate_pair<SA, SB, float, 4, kTabLds>),
       F(&k_integrate_pair<SA, SB, float, 4, kTabGlobal>)}};
  if (taba < 0 || taba > 2) return nullptr;
  return fp32 ? t32[w][taba] : t64[w][taba];
}

// Adjoint sweep over a full record: one wave per cell.
template <int S>
__global__ void __launch_bounds__(256) k_adjoint(Params P) {
  extern __shared__ double smem[];
  const int wib = threadIdx.x / kWave;
  const int li = threadIdx.x & (kWave - 1);
  const int64_t w = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + wib;
  if (w >= P.n_list) return;
  const int64_t cell = P.list ? P.list[w] : w;
  const RecView rv{P.rec + cell * P.rec_cap * P.rec_stride, 1, P.rec_stride};
  adjoint_steps<S>(P, cell, li, smem + static_cast<int64_t>(wib) * P.lds_doubles, rv,
                   uni(P.rec_n[cell]), 1, true);
}

// Pass j of the sweep over checkpointed records, as two launches: k_adj_rerun
// reruns the pass's segment of every cell (the forward step code, with the
// registers of that code alone), k_adj_sweep sweeps it (with the sweep's).  One
// wave per cell of the list; a cell without a segment in this pass returns at
// once.  (A persistent loop over cells costs these kernels 20-35 % more
// registers.)  ABC as in k_integrate.
template <int S, bool ABC>
__global__ void __launch_bounds__(256) k_adj_rerun(Params P, int j) {
  extern __shared__ double smem[];
  const int wib = threadIdx.x / kWave;
  const Grp<1> W(threadIdx.x & (kWave - 1));
  const int64_t w = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + wib;
  if (w >= P.n_list) return;
  rerun_segment<S, ABC>(P, P.list ? P.list[w] : w, W, smem + static_cast<int64_t>(wib) * P.lds_doubles, j);
}

template <int S>
__global__ void __launch_bounds__(256) k_adj_sweep(Params P, int j) {
  extern __shared__ double smem[];
  const int wib = threadIdx.x / kWave;
  const int li = threadIdx.x & (kWave - 1);
  const int64_t w = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + wib;
  if (w >= P.n_list) return;
  sweep_segment<S>(P, P.list ? P.list[w] : w, li, smem + static_cast<int64_t>(wib) * P.lds_doubles, j);
}

// kind 0: full-record sweep; 1: segment rerun; 2: segment sweep
template <int S>
const void *adjoint_kernel(int kind, bool abc) {
  if (kind == 0) return (const void *)&k_adjoint<S>;
  if (kind == 2) return (const void *)&k_adj_sweep<S>;
  return abc ? (const void *)&k_adj_rerun<S, true> : (const void *)&k_adj_rerun<S, false>;
}

struct LaunchCfg {
  int grid, block;
  size_t lds_bytes;
};

// the three register budgets of one kernel configuration
// lock-step kernels: one register budget (the block of up to 16 waves caps
// the registers anyway), one cell per wave, tables in LDS
template <int S>
const void *lock_kernel(bool fp32, bool abc) {
  if (abc)
    return fp32 ? (const void *)&k_integrate<S, float, 1, kTabLds, 1, true, false, kLinAnalytic, true>
                : (const void *)&k_integrate<S, double, 1, kTabLds, 1, true, false, kLinAnalytic, true>;
  return fp32 ? (const void *)&k_integrate<S, float, 1, kTabLds, 1, false, false, kLinAnalytic, true>
              : (const void *)&k_integrate<S, double, 1, kTabLds, 1, false, false, kLinAnalytic, true>;
}

template <int S, typename LT, int TAB, int G, bool ABC, bool TH = false, int LIN = kLinAnalytic>
const void *by_budget(int w) {
  using F = const void *;
  static const F t[4] = {F(&k_integrate<S, LT, 1, TAB, G, ABC, TH, LIN>),
                         F(&k_integrate<S, LT, 3, TAB, G, ABC, TH, LIN>),
                         F(&k_integrate<S, LT, 4, TAB, G, ABC, TH, LIN>),
                         F(&k_integrate<S, LT, 5, TAB, G, ABC, TH, LIN>)};
  return t[w];
}

// difference-quotient and GMRES kernels: one cell per wave, tables in LDS;
// GMRES forms no matrix, so it has only the FP64 instance
template <int S, bool TH, int LIN>
const void *lin_kernel(bool fp32, int w, bool abc) {
  if constexpr (LIN == kLinGmres) {
    return abc ? by_budget<S, double, kTabLds, 1, true, TH, LIN>(w)
               : by_budget<S, double, kTabLds, 1, false, TH, LIN>(w);
  } else {
    if (abc)
      return fp32 ? by_budget<S, float, kTabLds, 1, true, TH, LIN>(w)
                  : by_budget<S, double, kTabLds, 1, true, TH, LIN>(w);
    return fp32 ? by_budget<S, float, kTabLds, 1, false, TH, LIN>(w)
                : by_budget<S, double, kTabLds, 1, false, TH, LIN>(w);
  }
}

template <int S, bool ABC>
const void *integrate_kernel_abc(bool fp32, int w, int tab, int cells_per_wave) {
  if (cells_per_wave == 2) {
    if constexpr (S <= 32) {
      if (tab != kTabLds) return nullptr;
      return fp32 ? by_budget<S, float, kTabLds, 2, ABC>(w) : by_budget<S, double, kTabLds, 2, ABC>(w);
    }
    return nullptr;
  }
  if (cells_per_wave != 1) return nullptr;
  switch (tab) {
    case kTabRxGlobal:
      return fp32 ? by_budget<S, float, kTabRxGlobal, 1, ABC>(w)
                  : by_budget<S, double, kTabRxGlobal, 1, ABC>(w);
    case kTabLds:
      return fp32 ? by_budget<S, float, kTabLds, 1, ABC>(w) : by_budget<S, double, kTabLds, 1, ABC>(w);
    case kTabGlobal:
      if constexpr (S >= 32)
        return fp32 ? by_budget<S, float, kTabGlobal, 1, ABC>(w)
                    : by_budget<S, double, kTabGlobal, 1, ABC>(w);
      return nullptr;
    default:
      return nullptr;
  }
}

// the integrator kernel for (LU precision, register budget, table placement,
// cells per wave, A + B <=> C mechanism, non-isothermal, linear solver);
// nullptr where no such variant is built (two cells per wave only with the
// tables in LDS; tables in global memory only for sizes whose LDS can limit
// the resident waves; non-isothermal cells, difference quotients and GMRES
// one cell per wave with the tables in LDS)
template <int S>
const void *integrate_kernel(bool fp32, int minw, int tab, int cells_per_wave, bool abc,
                             bool thermal, int lin, bool lock = false) {
  const int w = minw >= 5 ? 3 : minw >= 4 ? 2 : minw >= 3 ? 1 : 0;
  if (lock) {
    if (tab != kTabLds || cells_per_wave != 1 || thermal || lin != kLinAnalytic) return nullptr;
    return lock_kernel<S>(fp32, abc);
  }
  if (lin != kLinAnalytic) {
    if (tab != kTabLds || cells_per_wave != 1) return nullptr;
    if (lin == kLinDq)
      return thermal ? lin_kernel<S, true, kLinDq>(fp32, w, abc)
                     : lin_kernel<S, false, kLinDq>(fp32, w, abc);
    if (lin == kLinGmres)
      return thermal ? lin_kernel<S, true, kLinGmres>(fp32, w, abc)
                     : lin_kernel<S, false, kLinGmres>(fp32, w, abc);
    return nullptr;
  }
  if (thermal) {
    if (tab != kTabLds || cells_per_wave != 1) return nullptr;
    if (abc)
      return fp32 ? by_budget<S, float, kTabLds, 1, true, true>(w)
                  : by_budget<S, double, kTabLds, 1, true, true>(w);
    return fp32 ? by_budget<S, float, kTabLds, 1, false, true>(w)
                : by_budget<S, double, kTabLds, 1, false, true>(w);
  }
  return abc ? integrate_kernel_abc<S, true>(fp32, w, tab, cells_per_wave)
             : integrate_kernel_abc<S, false>(fp32, w, tab, cells_per_wave);
}

template <int S>
hipError_t launch_integrate(const Params &P, bool fp32, int minw, int tab, int cells_per_wave,
                            bool abc, bool thermal, int lin, bool lock, const LaunchCfg &c,
                            hipStream_t s) {
  const void *f = integrate_kernel<S>(fp32, minw, tab, cells_per_wave, abc, thermal, lin, lock);
  if (!f) return hipErrorInvalidDeviceFunction;
  Params arg = P;
  void *args[] = {&arg};
  return hipLaunchKernel(f, dim3(c.grid), dim3(c.block), args, c.lds_bytes, s);
}

template <int S>
hipError_t launch_adjoint(const Params &P, int kind, int pass, bool abc, const LaunchCfg &c,
                          hipStream_t s) {
  Params arg = P;
  int j = pass;
  void *args[] = {&arg, &j};
  return hipLaunchKernel(adjoint_kernel<S>(kind, abc), dim3(c.grid), dim3(c.block), args,
                         c.lds_bytes, s);
}

template <int S>
hipError_t occupancy_integrate(bool fp32, int minw, int tab, int cells_per_wave, bool abc,
                               bool thermal, int lin, bool lock, int block, size_t lds_bytes,
                               int *blocks_per_cu) {
  const void *f = integrate_kernel<S>(fp32, minw, tab, cells_per_wave, abc, thermal, lin, lock);
  if (!f) {
    *blocks_per_cu = 0;
    return hipSuccess;
  }
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, block, lds_bytes);
}

}  // namespace bdfx

// One translation unit per species size (compiled in parallel).  The
// kernel flags are passed packed: bit 0 A + B <=> C, bit 1 non-isothermal,
// bit 2 difference-quotient Jacobian, bit 3 GMRES, bit 4 lock-step batches.
#define BDFX_LIN_OF_FLAGS(f) \
  ((f) & 8 ? bdfx::kLinGmres : (f) & 4 ? bdfx::kLinDq : bdfx::kLinAnalytic)
#define BDFX_DEFINE_SIZE(S)                                                                      \
  hipError_t bdfx_launch_s##S(const bdfx::Params &P, bool fp32, int minw, int tab, int cpw,      \
                              int flags, const bdfx::LaunchCfg &c, hipStream_t s) {              \
    return bdfx::launch_integrate<S>(P, fp32, minw, tab, cpw, flags & 1, flags & 2,              \
                                     BDFX_LIN_OF_FLAGS(flags), flags & 16, c, s);                \
  }                                                                                              \
  hipError_t bdfx_occupancy_s##S(bool fp32, int minw, int tab, int cpw, int flags, int block,    \
                                 size_t lds, int *out) {                                         \
    return bdfx::occupancy_integrate<S>(fp32, minw, tab, cpw, flags & 1, flags & 2,              \
                                        BDFX_LIN_OF_FLAGS(flags), flags & 16, block, lds, out);  \
  }                                                                                              \
  hipError_t bdfx_adjoint_s##S(const bdfx::Params &P, int kind, int pass, bool abc,            \
                                const bdfx::LaunchCfg &c, hipStream_t s) {                       \
    return bdfx::launch_adjoint<S>(P, kind, pass, abc, c, s);                                    \
  }

// Both bins of a two-mechanism batch in one launch (k_integrate_pair).
#define BDFX_DEFINE_PAIR(SA, SB)                                                                 \
  hipError_t bdfx_launch_pair_s##SA##_s##SB(const bdfx::Params &PA, const bdfx::Params &PB,      \
                                            bool fp32, int minw, int taba,                       \
                                            const bdfx::LaunchCfg &c, hipStream_t s) {           \
    const void *f = bdfx::pair_kernel<SA, SB>(fp32, minw, taba);                                 \
    if (!f) return hipErrorInvalidDeviceFunction;                                                \
    bdfx::Params a = PA, b = PB;                                                                 \
    void *args[] = {&a, &b};                                                                     \
    return hipLaunchKernel(f, dim3(c.grid), dim3(c.block), args, c.lds_bytes, s);                \
  }                                                                                              \
  /* blocks per CU for this block size and LDS; lds above 64 KiB is first allowed for the     */ \
  /* kernel (the device's per-block maximum bounds it)                                         */ \
  hipError_t bdfx_occupancy_pair_s##SA##_s##SB(bool fp32, int minw, int taba, int block,         \
                                               size_t lds, int *out) {                           \
    const void *f = bdfx::pair_kernel<SA, SB>(fp32, minw, taba);                                 \
    *out = 0;                                                                                    \
    if (!f) return hipSuccess;                                                                   \
    if (lds > 65536) {                                                                           \
      const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,    \
                                               static_cast<int>(lds));                           \
      if (e != hipSuccess) return e;                                                             \
    }                                                                                            \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, f, block, lds);                     \
  }

#define BDFX_DECLARE_PAIR(SA, SB)                                                                \
  hipError_t bdfx_launch_pair_s##SA##_s##SB(const bdfx::Params &PA, const bdfx::Params &PB,      \
                                            bool fp32, int minw, int taba,                       \
                                            const bdfx::LaunchCfg &c, hipStream_t s);            \
  hipError_t bdfx_occupancy_pair_s##SA##_s##SB(bool fp32, int minw, int taba, int block,         \
                                               size_t lds, int *out);

#define BDFX_DECLARE_SIZE(S)                                                                     \
  hipError_t bdfx_launch_s##S(const bdfx::Params &P, bool fp32, int minw, int tab, int cpw,      \
                              int flags, const bdfx::LaunchCfg &c, hipStream_t s);               \
  hipError_t bdfx_occupancy_s##S(bool fp32, int minw, int tab, int cpw, int flags, int block,    \
                                 size_t lds, int *out);                                          \
  hipError_t bdfx_adjoint_s##S(const bdfx::Params &P, int kind, int pass, bool abc,            \
                                const bdfx::LaunchCfg &c, hipStream_t s);
