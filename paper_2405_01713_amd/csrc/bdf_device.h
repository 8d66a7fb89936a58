// bdf_device.h -- gfx950 device code of the per-cell variable-order BDF
// integrator for mass-action kinetics.
//
// Method (arXiv 2405.01713, Balos et al.): for every grid cell the split
// chemistry ODE y' = R(y) + F (Sec. 3.1, Eq. (7)) is integrated by CVODE-style
// variable-order, variable-step BDF (Sec. 2, Eq. (1)) with WRMS local error
// control (Sec. 2, Eq. (3)), modified Newton stopped by Sec. 2, Eq. (4)
// (c_eps = 0.1, c_r = 0.3), Newton matrix I - gamma J from the analytic
// Jacobian and dense LU with partial pivoting (Table 1, approach 2A/2B).
// Unlike the paper's host-driven lock-step batches (Sec. 2), step size and
// order are chosen per cell, entirely on the device.
//
// Mapping: one wavefront (64 lanes) per cell.  Lane i owns species i: its
// Nordsieck entries z_j[i], Newton correction, error weight and, during a
// setup, row i of the Newton matrix in registers.  Everything that is a
// property of the cell (t, h, q, counters, Newton rate, ...) is wave-uniform:
// reductions are DPP row operations plus row broadcasts, broadcasts are
// v_readlane, branches are scalar, so the integrator's control flow never
// diverges inside a wave.  Per-cell data that is gathered by index (current
// state, rate constants, the right-hand side accumulator, the control block
// and the LU factors) lives in LDS.  Reactions are distributed over lanes;
// their rates are scattered into f with LDS FP64 atomics.
//
// Readings of the paper where it is silent are the same as the CPU oracle's
// (which shares no code with this file): Nordsieck variable-coefficient BDF
// with Lambda(x) = prod (1 + x/xi_i), error constant 1/(l_1 xi_{q+1}),
// interpolation-preserving order changes, next step size chosen after every
// accepted step and the order every q+1 steps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdfx {

constexpr int kWave = 64;
constexpr int kQmax = 5;
constexpr int kMaxS = 64;
// slot byte of an empty reaction slot: indexes a 1.0 kept after the 64 state
// entries, so that a rate is a product over all three slots without branches
constexpr int kEmptySlot = 64;
constexpr double kUround = 2.220446049250313e-16;

constexpr int kSuccess = 0;
constexpr int kTooMuchWork = -1;
constexpr int kErrFailure = -3;
constexpr int kConvFailure = -4;
constexpr int kSetupFailure = -6;
constexpr int kNonfinite = -9;
constexpr int kRecordFull = -10;

struct CellStats {
  int32_t status, nst, nfe, nni, nsetups, netf, ncfn, q_last, nli, ncfl;
  double h_last, t_reached;
};

// Linear solver of the Newton iteration: modified Newton with a direct solve
// of the Newton matrix from the analytic Jacobian (Table 1, approaches 2A/2B)
// or from difference quotients (3A/3B), or inexact Newton with matrix-free
// GMRES (1A/1B).
enum : int { kLinAnalytic = 0, kLinDq = 1, kLinGmres = 2 };
constexpr int kGmresMaxl = 10;

// Device-resident mechanism tables (built on the host from the
// stoichiometry; see the host runtime for the encodings).
struct MechDev {
  int32_t S, R;
  int32_t reversible;
  const int32_t *rx;       // [R][2]: species of the reactant / product slots, one byte each (kEmptySlot = empty)
  const double *lnA;       // [R]
  const double *EaR;       // [R]
  const double *lnK;       // [R] (reversible only)
  const double *w;           // [S] species weights (perturbation rescale)
  // non-isothermal cells (nullptr: isothermal): temperature is state entry S,
  // species energies u_i(T) = u0_i + cv_i T, adiabatic at constant volume
  const double *cv;        // [S]
  const double *u0;        // [S]
};

struct Params {
  MechDev mech;
  int64_t n_list;         // cells handled by this launch
  const int32_t *list;    // their indices (nullptr = 0..n_list-1)
  double *y;
  int32_t ldy;
  int32_t ldk;
  const double *T;
  const double *kscale;
  const double *F;
  int32_t *status;
  CellStats *stats;
  double t0, tout, rtol;
  int32_t atol_len, max_order, max_steps;
  int32_t max_netf, max_ncf;  // failures within one step that fail the cell
  int32_t n_sp;           // species of the mechanism (<= template S)
  int32_t gmres_maxl;     // Krylov vectors per GMRES solve (GMRES kernels only)
  int32_t lds_doubles;    // LDS per wave
  int32_t pair_waves;     // k_integrate_pair: waves per block of the larger mechanism
  int32_t use_queue;      // 0: one cell per wave from the grid index; 1: work queue
  uint32_t *queue;
  int32_t chunk;
  double *kk_slots;       // [waves][2R] rate constants of each wave's cell (tables in global memory)
  int64_t kk_nslots;      // waves the slot array can hold
  // accepted-step records for the adjoint (rec == nullptr: off)
  double *rec;            // [N][cap][stride]: y (n_sp), h, q | rebuild << 8
  int32_t rec_cap, rec_stride;
  int32_t *rec_n;         // [N]
  double *rec_hpad;       // [N]
  double *rec_y0;         // [N][rec_stride]
  // checkpointed records (ckpt != nullptr: no per-step states; at every
  // ckpt_every-th accepted step the integrator's whole state is saved, and the
  // adjoint recomputes the steps in between from it with this same code)
  double *ckpt;           // [N][ckpt_cap][Ckpt::stride(ckpt_vs)]
  double *ckpt_setup;     // [N][ckpt_vs]: predicted state of the cell's last Newton-matrix setup
  int32_t ckpt_every, ckpt_cap, ckpt_vs;
  int32_t seg_rows;       // adjoint: rows of a rerun segment (ckpt_every + kQmax + 1)
  double *seg;            // adjoint: [N][seg_rows][rec_stride], each cell's current segment
  double *adj;            // adjoint: [N][kQmax + 2][ckpt_vs], sweep state between segments
  const double *atol;     // [atol_len] (device)
  // adjoint (bdfx_adjoint only)
  const double *ybar;     // [N][ldy] dL/dy(t_out)
  double *y0bar;          // [N][ldy] out
  double *pbar;           // [N][ldp] out: dL/dlnA_r contributions of each cell
  int32_t ldp;
};

// ---------------------------------------------------------------------------
// wavefront primitives (all 64 lanes active, uniform control flow)
// ---------------------------------------------------------------------------

// Orders this wave's LDS accesses: the compiler may not move memory
// operations across it, and LDS instructions of one wave execute in order.
__device__ __forceinline__ void wave_lds_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ double uni(double v) {
  const int2 p = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_readfirstlane(p.x);
  r.y = __builtin_amdgcn_readfirstlane(p.y);
  return __builtin_bit_cast(double, r);
}

// value of lane `lane` (wave-uniform index)
__device__ __forceinline__ double lane_bcast(double v, int lane) {
  const int2 p = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_readlane(p.x, lane);
  r.y = __builtin_amdgcn_readlane(p.y, lane);
  return __builtin_bit_cast(double, r);
}

__device__ __forceinline__ float lane_bcast(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// value of lane `src` (per-lane index, taken mod 64) by ds_bpermute
__device__ __forceinline__ double lane_pull(double v, int src) {
  const int2 p = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_ds_bpermute(src << 2, p.x);
  r.y = __builtin_amdgcn_ds_bpermute(src << 2, p.y);
  return __builtin_bit_cast(double, r);
}

// One 32-bit DPP move.  With every row enabled the permutations used here
// read a valid source lane everywhere, so no old value is needed (and none
// is materialised); rows a row mask disables read 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp32(int x) {
  if constexpr (ROWMASK == 0xf) return __builtin_amdgcn_mov_dpp(x, CTRL, 0xf, 0xf, false);
  else return __builtin_amdgcn_update_dpp(0, x, CTRL, ROWMASK, 0xf, false);
}

template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp(double v) {
  const int2 p = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = dpp32<CTRL, ROWMASK>(p.x);
  r.y = dpp32<CTRL, ROWMASK>(p.y);
  return __builtin_bit_cast(double, r);
}

template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ uint64_t dpp(uint64_t v) {
  const int2 p = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = dpp32<CTRL, ROWMASK>(p.x);
  r.y = dpp32<CTRL, ROWMASK>(p.y);
  return __builtin_bit_cast(uint64_t, r);
}

// DPP controls: quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror,
// row_mirror (full 16-lane row), then row_bcast:15 into rows 1 and 3 and
// row_bcast:31 into rows 2 and 3: lane 63 ends with the whole wave.
constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E, kHalfMirror = 0x141, kMirror = 0x140,
              kBcast15 = 0x142, kBcast31 = 0x143;

// sum over the 64 lanes (wave-uniform result)
__device__ __forceinline__ double wsum(double v) {
  v += dpp<kQuadXor1>(v);
  v += dpp<kQuadXor2>(v);
  v += dpp<kHalfMirror>(v);
  v += dpp<kMirror>(v);
  v += dpp<kBcast15, 0xa>(v);
  v += dpp<kBcast31, 0xc>(v);
  return lane_bcast(v, 63);
}

// max over the 64 lanes of non-negative values (masked rows read 0)
__device__ __forceinline__ double wmax(double v) {
  v = fmax(v, dpp<kQuadXor1>(v));
  v = fmax(v, dpp<kQuadXor2>(v));
  v = fmax(v, dpp<kHalfMirror>(v));
  v = fmax(v, dpp<kMirror>(v));
  v = fmax(v, dpp<kBcast15, 0xa>(v));
  v = fmax(v, dpp<kBcast31, 0xc>(v));
  return lane_bcast(v, 63);
}

__device__ __forceinline__ uint32_t wmax_u32(uint32_t v) {
  auto step = [](uint32_t a, uint32_t b) { return a > b ? a : b; };
  v = step(v, __builtin_amdgcn_update_dpp(0u, v, kQuadXor1, 0xf, 0xf, false));
  v = step(v, __builtin_amdgcn_update_dpp(0u, v, kQuadXor2, 0xf, 0xf, false));
  v = step(v, __builtin_amdgcn_update_dpp(0u, v, kHalfMirror, 0xf, 0xf, false));
  v = step(v, __builtin_amdgcn_update_dpp(0u, v, kMirror, 0xf, 0xf, false));
  v = step(v, __builtin_amdgcn_update_dpp(0u, v, kBcast15, 0xa, 0xf, false));
  v = step(v, __builtin_amdgcn_update_dpp(0u, v, kBcast31, 0xc, 0xf, false));
  return __builtin_amdgcn_readlane(v, 63);
}

// 1/x for finite, normal, nonzero x: the hardware estimate refined by two
// Newton-Raphson steps r <- r + r (1 - x r) (within about one ulp).
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// lowest lane whose predicate holds (-1 if none); wave-uniform
__device__ __forceinline__ int wfirst(bool pred) {
  return uni(static_cast<int>(__ffsll(static_cast<long long>(__ballot(pred)))) - 1);
}

__device__ __forceinline__ bool wany(bool pred) { return __ballot(pred) != 0ull; }

// The lanes that integrate one cell: the whole wave (G = 1) or one half-wave
// (G = 2, two cells per wave for S <= 32).  Reductions, broadcasts and
// "uniform" values are per group: for G = 1 they are wave-uniform (scalar
// registers, scalar branches); for G = 2 they are uniform within each half
// and the two halves follow their own control flow under the exec mask.  The
// reductions run over 16-lane rows and then combine rows 0+1 (and 2+3), so a
// half-wave sum of S <= 32 species uses the same operations as the full-wave
// one, whose rows 2 and 3 only add zeros.
template <int G>
struct Grp {
  static_assert(G == 1 || G == 2, "one or two cells per wave");
  static constexpr int kLanes = kWave / G;
  int lane;  // lane within the group (species index)
  int grp;   // group index within the wave
  __device__ explicit Grp(int li) : lane(li % kLanes), grp(li / kLanes) {}

  __device__ double uni(double v) const {
    if constexpr (G == 1) return bdfx::uni(v);
    else return v;
  }
  __device__ int uni(int v) const {
    if constexpr (G == 1) return bdfx::uni(v);
    else return v;
  }
  // the value of lane 0 of the group
  __device__ int from_lane0(int v) const {
    if constexpr (G == 1) return bdfx::uni(v);
    else return grp ? __builtin_amdgcn_readlane(v, 32) : __builtin_amdgcn_readlane(v, 0);
  }
  // the value of the group's lane p (p uniform within the group)
  template <typename T>
  __device__ T bcast(T v, int p) const {
    if constexpr (G == 1) {
      return lane_bcast(v, p);
    } else {
      const int p0 = __builtin_amdgcn_readlane(p, 0), p1 = __builtin_amdgcn_readlane(p, 32);
      const T a = lane_bcast(v, p0), b = lane_bcast(v, 32 + p1);
      return grp ? b : a;
    }
  }
  // Reductions over the group.  NROW: 16-lane rows that can hold nonzero
  // data (the first ceil(S/16) of each group); the rounds that would only
  // combine zero rows are left out, which changes no result bit.
  static constexpr int rows(int nrow) { return nrow < kLanes / 16 ? nrow : kLanes / 16; }
  // the group-uniform result from the lane that holds it
  template <int NROW, typename T>
  __device__ T last(T v) const {
    constexpr int l = 16 * rows(NROW) - 1;  // 15, 31 or 63 within the group
    if constexpr (G == 1) {
      return lane_bcast(v, l);
    } else {
      const T a = lane_bcast(v, l), b = lane_bcast(v, 32 + l);
      return grp ? b : a;
    }
  }
  template <int NROW = 4>
  __device__ double sum(double v) const {
    v += dpp<kQuadXor1>(v);
    v += dpp<kQuadXor2>(v);
    v += dpp<kHalfMirror>(v);
    v += dpp<kMirror>(v);
    if constexpr (rows(NROW) >= 2) v += dpp<kBcast15, 0xa>(v);
    if constexpr (rows(NROW) >= 3) v += dpp<kBcast31, 0xc>(v);
    return last<NROW>(v);
  }
  // max of non-negative values (masked rows read 0)
  template <int NROW = 4>
  __device__ double max(double v) const {
    v = fmax(v, dpp<kQuadXor1>(v));
    v = fmax(v, dpp<kQuadXor2>(v));
    v = fmax(v, dpp<kHalfMirror>(v));
    v = fmax(v, dpp<kMirror>(v));
    if constexpr (rows(NROW) >= 2) v = fmax(v, dpp<kBcast15, 0xa>(v));
    if constexpr (rows(NROW) >= 3) v = fmax(v, dpp<kBcast31, 0xc>(v));
    return last<NROW>(v);
  }
  template <int NROW = 4>
  __device__ uint32_t max_u32(uint32_t v) const {
    auto step = [](uint32_t a, uint32_t b) { return a > b ? a : b; };
    v = step(v, __builtin_amdgcn_update_dpp(0u, v, kQuadXor1, 0xf, 0xf, false));
    v = step(v, __builtin_amdgcn_update_dpp(0u, v, kQuadXor2, 0xf, 0xf, false));
    v = step(v, __builtin_amdgcn_update_dpp(0u, v, kHalfMirror, 0xf, 0xf, false));
    v = step(v, __builtin_amdgcn_update_dpp(0u, v, kMirror, 0xf, 0xf, false));
    if constexpr (rows(NROW) >= 2)
      v = step(v, __builtin_amdgcn_update_dpp(0u, v, kBcast15, 0xa, 0xf, false));
    if constexpr (rows(NROW) >= 3)
      v = step(v, __builtin_amdgcn_update_dpp(0u, v, kBcast31, 0xc, 0xf, false));
    constexpr int l = 16 * rows(NROW) - 1;
    if constexpr (G == 1) {
      return __builtin_amdgcn_readlane(v, l);
    } else {
      const uint32_t a = __builtin_amdgcn_readlane(v, l), b = __builtin_amdgcn_readlane(v, 32 + l);
      return grp ? b : a;
    }
  }
  // lowest lane of the group whose predicate holds (-1 if none)
  __device__ int first(bool pred) const {
    const uint64_t b = __ballot(pred);
    if constexpr (G == 1) {
      return bdfx::uni(static_cast<int>(__ffsll(static_cast<long long>(b))) - 1);
    } else {
      const uint32_t h = grp ? static_cast<uint32_t>(b >> 32) : static_cast<uint32_t>(b);
      return h ? __ffs(static_cast<int>(h)) - 1 : -1;
    }
  }
  __device__ bool any(bool pred) const {
    const uint64_t b = __ballot(pred);
    if constexpr (G == 1) return b != 0ull;
    else return (grp ? (b >> 32) : (b & 0xffffffffull)) != 0ull;
  }
};

// ---------------------------------------------------------------------------
// Nordsieck array operations (z_j = h^j y^(j) / j!)
// ---------------------------------------------------------------------------

// The integrator keeps z_j = 0 for every j > q (columns start at zero, an
// order decrease zeroes z_q, an order increase writes z_{q+1}, a restart
// zeroes z_2..), so the operations below run over all kQmax columns with no
// per-order selects: the extra terms add or scale exact zeros.

// z <- z * Pascal: Taylor shift by one step (predictor).
__device__ __forceinline__ void nd_predict(double (&z)[kQmax + 1]) {
#pragma unroll
  for (int k = 1; k <= kQmax; ++k)
#pragma unroll
    for (int j = kQmax; j >= k; --j) z[j - 1] += z[j];
}

// exact inverse of nd_predict (restore after a rejected attempt)
__device__ __forceinline__ void nd_unpredict(double (&z)[kQmax + 1]) {
#pragma unroll
  for (int k = 1; k <= kQmax; ++k)
#pragma unroll
    for (int j = kQmax; j >= k; --j) z[j - 1] -= z[j];
}

// h -> eta h: z_j <- eta^j z_j
__device__ __forceinline__ void nd_rescale(double (&z)[kQmax + 1], double eta) {
  double f = 1.0;
#pragma unroll
  for (int j = 1; j <= kQmax; ++j) {
    f *= eta;
    z[j] *= f;
  }
}

// a[k] for a small register array and a run-time k, as bitwise masks on the
// IEEE bit patterns (a compare-and-select chain can be turned into an indexed
// load, which would force the array into scratch memory)
template <int N>
__device__ __forceinline__ double pick(const double (&a)[N], int k) {
  uint64_t v = 0;
#pragma unroll
  for (int j = 0; j < N; ++j)
    v |= __builtin_bit_cast(uint64_t, a[j]) & (0ull - static_cast<uint64_t>(j == k));
  return __builtin_bit_cast(double, v);
}

__device__ __forceinline__ double nd_get(const double (&z)[kQmax + 1], int q) { return pick(z, q); }

// l_j of Lambda(x) = prod_{i=1}^{q} (1 + x/xi_i); Cerr = 1/(l_1 xi_{q+1}).
__device__ __forceinline__ void bdf_coeffs(int q, const double (&xi)[kQmax + 2],
                                           double (&l)[kQmax + 2], double &Cerr) {
  l[0] = 1.0;
#pragma unroll
  for (int j = 1; j <= kQmax + 1; ++j) l[j] = 0.0;
#pragma unroll
  for (int i = 1; i <= kQmax; ++i)
    if (i <= q) {
      const double rxi = rcp(xi[i]);
#pragma unroll
      for (int j = i; j >= 1; --j) l[j] = fma(l[j - 1], rxi, l[j]);
    }
  Cerr = rcp(l[1] * pick(xi, q + 1));
}

// H_k = 1 + 1/2 + ... + 1/k and k! for k = 0..6
// (a switch on the wave-uniform order: scalar branches, no table in registers)
__device__ __forceinline__ double harmonic(int k) {
  switch (k) {
    case 1: return 1.0;
    case 2: return 1.5;
    case 3: return 11.0 / 6.0;
    case 4: return 25.0 / 12.0;
    case 5: return 137.0 / 60.0;
    case 6: return 49.0 / 20.0;
    default: return 0.0;
  }
}

__device__ __forceinline__ double factorial(int k) {
  switch (k) {
    case 2: return 2.0;
    case 3: return 6.0;
    case 4: return 24.0;
    case 5: return 120.0;
    case 6: return 720.0;
    default: return 1.0;
  }
}

// x^(1/p) for x >= 0 and p in 1..14.  With x = u 2^(p k) (k from the binary
// exponent, u in about [2^-1, 2^(p+1)), exact power-of-two scaling) the root
// is 2^k u^(1/p); u^(1/p) starts from the FP32 hardware log2/exp2 estimate
// (relative error below 1e-6) and takes one Newton step on y^p = u in FP64
// (relative error below 1e-12).
__device__ __forceinline__ double root_p(double x, int p) {
  if (p == 1 || !(x > 0.0) || !(x < __builtin_huge_val())) return x;
  const int e = __builtin_amdgcn_frexp_exp(x);
  const double m = __builtin_amdgcn_frexp_mant(x);  // x = m 2^e, m in [0.5, 1)
  const float rp = __builtin_amdgcn_rcpf(static_cast<float>(p));
  const int k = static_cast<int>(__builtin_floorf(static_cast<float>(e) * rp));
  const double u = __builtin_ldexp(m, e - k * p);  // any integer k keeps x = u 2^(p k) exact
  double y = static_cast<double>(
      __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(static_cast<float>(u)) * rp));
  double yp1 = 1.0;  // y^(p-1)
  for (int i = 1; i < p; ++i) yp1 *= y;
  y = fma(fma(-y, yp1, u), __builtin_amdgcn_rcp(p * yp1), y);
  return __builtin_ldexp(y, k);
}

// eta = 1 / ((bias err)^(1/p) + 1e-6), from the squared error err2 = err^2:
// 1 / ((bias^2 err2)^(1/(2p)) + 1e-6)
__device__ __forceinline__ double eta_from2(double bias, double err2, int p) {
  return rcp(root_p(bias * bias * err2, 2 * p) + 1.0e-6);
}

// eta_from2(6, err2, p) >= 1.5 needs (36 err2)^(1/(2p)) <= 2/3 - 1e-6, i.e.
// 36 err2 <= (2/3 - 1e-6)^(2p).  hold_bound(p) is that bound raised by 1e-9
// relative (far above the rounding of either side): above it, eta < 1.5 for
// certain and the root need not be taken.
__device__ __forceinline__ double hold_bound(int p) {
  constexpr double c = 2.0 / 3.0 - 1.0e-6;
  constexpr double c2 = c * c, c4 = c2 * c2, c8 = c4 * c4;
  double b = (p & 1) ? c2 : 1.0;
  if (p & 2) b *= c4;
  if (p & 4) b *= c8;
  return b * (1.0 + 1.0e-9);
}

__device__ __forceinline__ double ipow(double x, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

// ---------------------------------------------------------------------------
// per-wave LDS
// ---------------------------------------------------------------------------

// Control block: cell-uniform values needed once per attempt or per
// accepted step, kept in LDS instead of registers.
struct Ctl {
  static constexpr int kHist = 0;    // [6] accepted step sizes, most recent first
  static constexpr int kXi = 6;      // [7] xi_i of the current attempt
  static constexpr int kL = 13;      // [7] l_j of the current attempt
  static constexpr int kEtaMax = 20;
  static constexpr int kHprev = 21;  // step size that produced e_prev
  static constexpr int kGammaBar = 22;
  static constexpr int kTn = 23;
  static constexpr int kSize = 24;
};

// One checkpoint (doubles): the integrator's state at the top of its step
// loop after nst accepted steps, everything the steps after it read.  Scalars
// (lane 0): t, h, q, nst, the order-change countdown, the step of the last
// Newton-matrix setup, the squared convergence rate, the setup/e_prev flags,
// the step sizes h_nst .. h_{nst-kQmax}, the step-growth limit, the step size
// of e_prev, the gamma of the last setup and the order step nst was taken
// with.  Lane vectors, vs apart (the kernel's padded size, so that their
// offsets are constants): the Nordsieck array z_0 .. z_kQmax, e_prev and the
// predicted state the last setup formed its Newton matrix at (the inverse is
// rebuilt from it, bit for bit).  Checkpoints of a cell lie stride(vs_max)
// apart, vs_max the largest padded size of the batch.
struct Ckpt {
  static constexpr int kT = 0, kH = 1, kQ = 2, kNst = 3, kQwait = 4, kNstSetup = 5, kR2 = 6,
                       kNeedSetup = 7, kHaveEprev = 8, kHist = 9 /* [kQmax + 1] */,
                       kEtaMax = kHist + kQmax + 1, kHprev = kEtaMax + 1, kGammaBar = kHprev + 1,
                       kQtaken = kGammaBar + 1, kScalars = 20;
  static_assert(kQtaken < kScalars, "checkpoint scalars overlap the vectors");
  // lane vectors: z_j is vector j, then e_prev and the setup state
  static constexpr int kVecEprev = kQmax + 1, kVecSetup = kQmax + 2;
  __host__ __device__ static constexpr int vec(int j, int vs) { return kScalars + j * vs; }
  __host__ __device__ static constexpr int stride(int vs) { return vec(kVecSetup + 1, vs); }
};

// A resumed integration (the adjoint's recomputation of one segment): start
// from checkpoint `ck` instead of the cell's input state, stop once `stop`
// steps are accepted, record accepted step s into row s - first of `rows`
// (n_rows rows of P.rec_stride; steps outside are not recorded) and write none
// of the cell's outputs.
struct Resume {
  const double *ck;
  double *rows;
  int first, stop, n_rows;
};

struct Lds {
  double *yb;   // [64 + 8] state for gathers (also the right-hand side of a solve); yb[kEmptySlot] = 1
  double *fb;   // [64] right-hand-side accumulator
  double *C;    // [Ctl::kSize]
  int *perm;    // [64] pivot row of each elimination step
  double *kk;   // [2R]: k_f at 2r, -k_r at 2r+1 (LDS, or the wave's slot in global memory)
  const int2 *rx;  // [R]: reactant / product slot words (an LDS copy, or the mechanism's table)
  void *fac;    // [S][S] inverse Newton matrix (LT), column-major: (r, c) at c*S + r
  double *kry;  // GMRES kernels, in place of fac: Krylov basis and Hessenberg data (KryLayout)
  double *uT;   // non-isothermal: [64 + 8] u_i(T) at the setup state (uT[kEmptySlot] = 0)
  double *uj;   // non-isothermal: [64 + 8] sum_r dU_r dq_r/dx_c per column c (Jacobian T row)
};

// Where a wave keeps the tables its inner loops read: the reaction slot words
// (copied per cell, or read from the mechanism's table) and the cell's rate
// constants (LDS, or the wave's own slot of a global array, which each lane
// writes and reads back for its own reactions only).  Placements that leave
// tables in global memory free LDS where LDS limits the resident waves.
enum : int {
  kTabRxGlobal = 0,  // slot words in global memory, rate constants in LDS
  kTabLds = 1,       // both in LDS
  kTabGlobal = 2,    // both in global memory (persistent waves only)
};

// GMRES area of a wave's LDS (doubles) for S state entries and at most maxl
// Krylov vectors: the basis of the scaled space ([maxl + 1][S]), the
// Hessenberg matrix (column-major, maxl + 1 rows; rotated in place), the
// rotations, the rotated right-hand side and the solution coefficients.
struct KryLayout {
  int V, H, cs, sn, g, c, size;
  __host__ __device__ constexpr KryLayout(int S, int maxl)
      : V(0), H((maxl + 1) * S), cs(H + (maxl + 1) * maxl), sn(cs + maxl), g(sn + maxl),
        c(g + maxl + 1), size(c + maxl) {}
};

// Slots of the inverse Newton matrix a wave keeps in registers instead of
// LDS (inv_tail columns of S entries).  At 53 species with the FP64 matrix
// (analytic Jacobian, one isothermal cell per wave, not lock-step) the last 9
// pivot slots: with the tables in global memory the wave then needs 20,192
// bytes of LDS, so 8 waves fit a CU's 160 KiB instead of 6, for 18 more VGPRs.
__host__ __device__ constexpr int inv_tail(int S, int lt_bytes, bool thermal, int lin, bool lock,
                                           int cells_per_wave) {
  return S == 53 && lt_bytes == 8 && !thermal && lin == kLinAnalytic && !lock && cells_per_wave == 1
             ? 9
             : 0;
}

// doubles of LDS per wave for S state entries, R reactions, factor type
// size, table placement and non-isothermal cells; gmres_maxl > 0: GMRES
// kernels, whose Krylov area replaces the Newton matrix and the
// non-isothermal Jacobian rows; tail: inverse slots held in registers
// (inv_tail)
__host__ __device__ constexpr int lds_doubles(int S, int R, int lt_bytes, int tab = kTabLds,
                                              bool thermal = false, int gmres_maxl = 0,
                                              int tail = 0) {
  return 2 * kWave + 8 + Ctl::kSize + kWave / 2 + (tab == kTabLds ? R : 0) +
         (tab == kTabGlobal ? 0 : 2 * R) +
         (gmres_maxl > 0 ? KryLayout(S, gmres_maxl).size
                         : ((S - tail) * S * lt_bytes + 7) / 8 + (thermal ? 2 * (kWave + 8) : 0));
}

// Inverse slots held in registers (lane r: M^{-1}(r, perm[S - T + t])).
template <int T, typename LT>
struct InvTail {
  LT v[T];
};
template <typename LT>
struct InvTail<0, LT> {};

template <int TAB, bool TH = false, bool KRY = false>
__device__ __forceinline__ Lds carve(double *base, int R, const int32_t *mech_rx, double *kk_slot,
                                     int S = 0, int lt_bytes = 8) {
  Lds L;
  L.yb = base;
  L.fb = base + kWave + 8;
  L.C = L.fb + kWave;
  L.perm = reinterpret_cast<int *>(L.C + Ctl::kSize);
  double *next = L.C + Ctl::kSize + kWave / 2;
  if constexpr (TAB == kTabGlobal) {
    L.kk = kk_slot;
  } else {
    L.kk = next;
    next += 2 * R;
  }
  if constexpr (TAB == kTabLds) {
    L.rx = reinterpret_cast<const int2 *>(next);
    next += R;
  } else {
    L.rx = reinterpret_cast<const int2 *>(mech_rx);
  }
  L.fac = next;
  L.kry = next;
  if constexpr (KRY) {
    L.fac = nullptr;
    L.uT = L.uj = nullptr;
  } else if constexpr (TH) {
    L.uT = next + (S * S * lt_bytes + 7) / 8;
    L.uj = L.uT + kWave + 8;
  } else {
    L.uT = L.uj = nullptr;
  }
  return L;
}

// ---------------------------------------------------------------------------
// kinetics
// ---------------------------------------------------------------------------

__device__ __forceinline__ int slot_species(int word, int s) { return (word >> (8 * s)) & 0xff; }

// f_i = F_i + sum_r nu_ir q_r: reaction r is handled by lane r mod 64, its
// net rate q_r = k_f prod y_reac - k_r prod y_prod is scattered into the LDS
// accumulator with FP64 atomics.  Two passes of 64 reactions are processed
// per loop iteration so that their LDS round trips overlap; lanes past R take
// an all-empty slot word.  Lane i passes y_i, F_i and gets f_i.
//
// ABC: every reaction of the mechanism has the form A + B <=> C (reactant
// slots 0 and 1 and product slot 0 occupied, the others empty), so the empty
// slots are neither gathered nor tested.  The products and sums are formed in
// the generic path's order (the empty slots there multiply by exactly 1) and
// the atomics land in its order, so both paths give the same bits.
//
// Non-isothermal cells (TH) pass the rate constants at the current
// temperature (kf and -kr); otherwise they come from the table of the cell.
template <bool ABC>
__device__ __forceinline__ void rhs_reaction(const Lds &L, int r, int2 w, double kf, double krn) {
  if constexpr (ABC) {
#pragma clang fp contract(off)
    const int a0 = slot_species(w.x, 0), a1 = slot_species(w.x, 1), b0 = slot_species(w.y, 0);
    const double pf = kf * L.yb[a0] * L.yb[a1];
    const double pr = krn * L.yb[b0];
    const double q = pf + pr;
    atomicAdd(&L.fb[a0], -q);
    atomicAdd(&L.fb[b0], q);
    atomicAdd(&L.fb[a1], -q);
    return;
  }
  double pf = kf, pr = krn;
  // empty slots read the 1.0 at yb[kEmptySlot]: the six gathers issue together
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    pf *= L.yb[slot_species(w.x, s)];
    pr *= L.yb[slot_species(w.y, s)];
  }
  const double q = pf + pr;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int a = slot_species(w.x, s), b = slot_species(w.y, s);
    if (a != kEmptySlot) atomicAdd(&L.fb[a], -q);
    if (b != kEmptySlot) atomicAdd(&L.fb[b], q);
  }
}

// Rate constants of reaction r at temperature 1 / rT for a non-isothermal
// cell: the table holds ln k_f0 (ln A plus the log of the cell's scale) and
// -exp(-ln K); k_f = exp(ln k_f0 - EaR rT).
__device__ __forceinline__ void thermal_rates(const MechDev &m, const Lds &L, int r, double rT,
                                              double &kf, double &krn) {
  kf = exp(L.kk[2 * r] - m.EaR[r] * rT);
  krn = kf * L.kk[2 * r + 1];
}

// Non-isothermal cells (TH): lane ns (= the species count) holds the
// temperature; the rate constants are evaluated at it, and that lane gets
// dT/dt = F_T - sum_i u_i(T) f_i / sum_i cv_i y_i.
template <bool ABC, bool TH = false, int G>
__device__ __forceinline__ double rhs(const MechDev &m, const Lds &L, const Grp<G> &W, double yi,
                                      double Fi, int ns = 0) {
  wave_lds_sync();
  L.yb[W.lane] = yi;
  L.fb[W.lane] = Fi;
  wave_lds_sync();
  const int R = m.R;
  double rT = 0.0;
  if constexpr (TH) rT = W.uni(rcp(W.bcast(yi, ns)));
  const int2 none = make_int2(0x40404040, 0x40404040);  // every slot empty
  for (int r0 = 0; r0 < R; r0 += 2 * W.kLanes) {
    const int ra = r0 + W.lane, rb = ra + W.kLanes;
    const int2 wa = ra < R ? L.rx[ra] : none;
    const int2 wb = rb < R ? L.rx[rb] : none;
    if constexpr (TH) {
      if (ra < R) {
        double kf, krn;
        thermal_rates(m, L, ra, rT, kf, krn);
        rhs_reaction<ABC>(L, ra, wa, kf, krn);
      }
      if (rb < R) {
        double kf, krn;
        thermal_rates(m, L, rb, rT, kf, krn);
        rhs_reaction<ABC>(L, rb, wb, kf, krn);
      }
    } else {
      if (ra < R) rhs_reaction<ABC>(L, ra, wa, L.kk[2 * ra], L.kk[2 * ra + 1]);
      if (rb < R) rhs_reaction<ABC>(L, rb, wb, L.kk[2 * rb], L.kk[2 * rb + 1]);
    }
  }
  wave_lds_sync();
  if constexpr (TH) {
    const double f = L.fb[W.lane];
    const bool sp = W.lane < ns;
    const double T = W.uni(W.bcast(yi, ns));
    const double cv = sp ? m.cv[W.lane] : 0.0, u = sp ? fma(cv, T, m.u0[W.lane]) : 0.0;
    const double N = W.uni(W.sum(u * f)), D = W.uni(W.sum(cv * yi));
    return W.lane == ns ? f - N / D : f;
  }
  return L.fb[W.lane];
}

// Row li of M = I - gamma J (or of M^T when `transposed`) at the state y held
// by the lanes (lane i passes y_i).  M is assembled in LDS, in the area that
// afterwards holds the inverse, column-major ((i, c) at c*S + i): starting
// from the identity, lane r mod 64 takes reaction r, forms d q_r / d y_c for
// every occupied slot c (the side's rate constant times the other slots of
// that side; the reverse constant is stored negated) and adds
// -gamma nu_ir d q_r / d y_c to M(i, c) for every occupied slot i of the
// reaction (reactant slots count -1, product slots +1) with LDS atomics.
// Each lane then reads its row (its column for M^T).  Terms are rounded to LT
// before they are summed.  T > 0 (an inverse with T slots in registers,
// whose LDS area holds S - T columns): two passes over the reactions, columns
// 0 .. S-T-1 and then the last T, each entry with the same terms in the same
// order as in one pass.
template <int S, typename LT, bool ABC = false, int T = 0, int G>
__device__ __forceinline__ void newton_matrix(LT (&a)[S], const MechDev &m, const Lds &L, const Grp<G> &W,
                                              double yi, double gamma, bool transposed) {
  static_assert(T == 0 || G == 1, "an inverse tail needs one cell per wave");
  LT *M = reinterpret_cast<LT *>(L.fac);
  const int lr = W.lane < S ? W.lane : 0;
  wave_lds_sync();
  L.yb[W.lane] = yi;
#pragma unroll
  for (int pass = 0; pass < (T > 0 ? 2 : 1); ++pass) {
    // columns c0 .. c0 + nc - 1, column c at (c - c0) * S
    const int c0 = pass == 0 ? 0 : S - T, nc = T == 0 ? S : (pass == 0 ? S - T : T);
    if (pass > 0) wave_lds_sync();
    for (int e = W.lane; e < nc * S; e += W.kLanes)
      M[e] = e % S == c0 + e / S ? static_cast<LT>(1) : static_cast<LT>(0);
    wave_lds_sync();
    for (int r = W.lane; r < m.R; r += W.kLanes) {
      const int2 w = L.rx[r];
      if constexpr (ABC) {
        // columns A, B (forward side) and C (reverse side), each scattered
        // into rows A, C, B: the generic path's terms in its order
        const int a0 = slot_species(w.x, 0), a1 = slot_species(w.x, 1), b0 = slot_species(w.y, 0);
        const double kf = L.kk[2 * r];
        const int col[3] = {a0, a1, b0};
        const double d[3] = {kf * L.yb[a1], kf * L.yb[a0], L.kk[2 * r + 1]};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (c == 2 && !m.reversible) break;
          if constexpr (T > 0) {
            if (col[c] < c0 || col[c] >= c0 + nc) continue;
          }
          const LT g = static_cast<LT>(gamma * d[c]);
          LT *Mc = M + (col[c] - c0) * S;
          atomicAdd(Mc + a0, g);
          atomicAdd(Mc + b0, -g);
          atomicAdd(Mc + a1, g);
        }
        continue;
      }
      int sp[2][3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sp[0][k] = slot_species(w.x, k);
        sp[1][k] = slot_species(w.y, k);
      }
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        if (side == 1 && !m.reversible) break;
        const double kside = L.kk[2 * r + side];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int col = sp[side][c];
          if (col == kEmptySlot) continue;
          if constexpr (T > 0) {
            if (col < c0 || col >= c0 + nc) continue;
          }
          double d = kside;
#pragma unroll
          for (int o = 0; o < 3; ++o)
            if (o != c) d *= L.yb[sp[side][o]];  // empty slots multiply by 1
          const LT g = static_cast<LT>(gamma * d);
          LT *Mc = M + (col - c0) * S;
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            if (sp[0][i] != kEmptySlot) atomicAdd(Mc + sp[0][i], g);
            if (sp[1][i] != kEmptySlot) atomicAdd(Mc + sp[1][i], -g);
          }
        }
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < S; ++j) {
      if (j < c0 || j >= c0 + nc) continue;
      const LT v = (T == 0 && transposed) ? M[lr * S + j] : M[(j - c0) * S + lr];
      a[j] = W.lane < S ? v : static_cast<LT>(0);
    }
  }
  wave_lds_sync();
}

// Row li of M = I - gamma J for a non-isothermal cell (state: ns species,
// then the temperature T at entry ns).  As newton_matrix for the species
// columns, with the rate constants at T; in the same pass over the reactions
// each lane also scatters
//   the T column: d q_r / dT = q_r EaR_r / T^2 (both rate constants carry
//     exp(-EaR_r / T)) into the rows of the reaction's species,
//   the species rates f_i (for the energy balance), and
//   sum_r dU_r d q_r / dx_c for every column c, with dU_r = sum_i nu_ir u_i(T)
//     the reaction's energy change, into L.uj,
// and the T row follows from the energy balance dT/dt = F_T - N / D,
// N = sum_i u_i f_i, D = sum_i cv_i y_i:
//   M(T, j) = gamma (sum_r dU_r dq_r/dy_j - N cv_j / D) / D,
//   M(T, T) = 1 + gamma (sum_i cv_i f_i + sum_r dU_r dq_r/dT) / D.
template <int S, typename LT, int G>
__device__ __forceinline__ void newton_matrix_thermal(LT (&a)[S], const MechDev &m, const Lds &L,
                                                   const Grp<G> &W, double yi, double Fi,
                                                   double gamma, int ns) {
  LT *M = reinterpret_cast<LT *>(L.fac);
  const double T = W.uni(W.bcast(yi, ns));
  const double rT = W.uni(rcp(T));
  const bool sp = W.lane < ns;
  const double cv = sp ? m.cv[W.lane] : 0.0;
  const double u = sp ? fma(cv, T, m.u0[W.lane]) : 0.0;
  wave_lds_sync();
  L.yb[W.lane] = yi;
  L.fb[W.lane] = sp ? Fi : 0.0;
  L.uT[W.lane] = u;  // 0 past the species
  if (W.lane == 0) L.uT[kEmptySlot] = 0.0;
  L.uj[W.lane] = 0.0;
  for (int e = W.lane; e < S * S; e += W.kLanes)
    M[e] = e % (S + 1) == 0 ? static_cast<LT>(1) : static_cast<LT>(0);
  wave_lds_sync();
  for (int r = W.lane; r < m.R; r += W.kLanes) {
    const int2 w = L.rx[r];
    double kf, krn;
    thermal_rates(m, L, r, rT, kf, krn);
    int sp2[2][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      sp2[0][k] = slot_species(w.x, k);
      sp2[1][k] = slot_species(w.y, k);
    }
    double dU = 0.0, pf = kf, pr = krn;
#pragma unroll
    for (int k = 0; k < 3; ++k) {  // empty slots read u = 0 and y = 1
      dU += L.uT[sp2[1][k]] - L.uT[sp2[0][k]];
      pf *= L.yb[sp2[0][k]];
      pr *= L.yb[sp2[1][k]];
    }
    const double q = pf + pr;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (sp2[0][k] != kEmptySlot) atomicAdd(&L.fb[sp2[0][k]], -q);
      if (sp2[1][k] != kEmptySlot) atomicAdd(&L.fb[sp2[1][k]], q);
    }
#pragma unroll
    for (int side = 0; side < 3; ++side) {  // 0, 1: species columns of each side; 2: T
      if (side == 1 && !m.reversible) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (side == 2 && c > 0) break;
        int col;
        double d;
        if (side == 2) {
          col = ns;
          d = q * m.EaR[r] * rT * rT;
        } else {
          col = sp2[side][c];
          if (col == kEmptySlot) continue;
          d = side == 0 ? kf : krn;
#pragma unroll
          for (int o = 0; o < 3; ++o)
            if (o != c) d *= L.yb[sp2[side][o]];
        }
        const LT g = static_cast<LT>(gamma * d);
        LT *Mc = M + col * S;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          if (sp2[0][i] != kEmptySlot) atomicAdd(Mc + sp2[0][i], g);
          if (sp2[1][i] != kEmptySlot) atomicAdd(Mc + sp2[1][i], -g);
        }
        atomicAdd(&L.uj[col], d * dU);
      }
    }
  }
  wave_lds_sync();
  const double f = L.fb[W.lane];
  const double N = W.uni(W.sum(u * f)), cf = W.uni(W.sum(cv * f));
  const double D = W.uni(W.sum(cv * yi));
  const double rD = 1.0 / D;
  if (W.lane <= ns) {
    const double v = W.lane < ns ? gamma * (L.uj[W.lane] - N * cv * rD) * rD
                                 : 1.0 + gamma * (cf + L.uj[ns]) * rD;
    M[W.lane * S + ns] = static_cast<LT>(v);
  }
  wave_lds_sync();
  const int lr = W.lane < S ? W.lane : 0;
#pragma unroll
  for (int j = 0; j < S; ++j) {
    const LT v = M[j * S + lr];
    a[j] = W.lane < S ? v : static_cast<LT>(0);
  }
  wave_lds_sync();
}

// squared WRMS norm of Eq. (3); inv_n = 1 / (species of the cell).  The
// integrator compares and raises squared norms, so no square root is taken.
template <int S, int G>
__device__ __forceinline__ double wrms2(const Grp<G> &W, double v, double w, double inv_n) {
  const double t = v * w;  // w = 0 on lanes without a species
  return W.uni(W.template sum<(S + 15) / 16>(t * t) * inv_n);
}

// Row li of M = I - gamma J with J by forward difference quotients, one
// right-hand side per state entry (Table 1, approaches 3A/3B; increments of
// the dense difference-quotient scheme documented for CVODE): f0 = f(y),
// min_inc = 1000 |h| u n ||f0|| (1 if ||f0|| = 0), inc_j = max(sqrt(u) |y_j|,
// min_inc / w_j), column j = (f(y + inc_j e_j) - f0) / inc_j.  Columns are
// written to the LDS matrix area (padding entries keep the identity), then
// each lane reads its row.  Costs n + 1 right-hand sides.
template <int S, typename LT, bool ABC, bool TH, int G>
__device__ __forceinline__ void dq_matrix(LT (&a)[S], const MechDev &m, const Lds &L, const Grp<G> &W,
                                          double y, double Fi, double gamma, double h, double ewt,
                                          int ns, int n, double inv_n) {
  LT *M = reinterpret_cast<LT *>(L.fac);
  constexpr double kSrur = 1.4901161193847656e-08;  // sqrt(kUround) = 2^-26
  double f0 = 0.0, min_inc = 1.0;
  // pass j = -1 evaluates f0; pass j >= 0 column j (one right-hand-side body)
  for (int j = -1; j < n; ++j) {
    double inc = 1.0, yp = y;
    if (j >= 0) {
      const double yj = W.uni(W.bcast(y, j)), wj = W.uni(W.bcast(ewt, j));
      const double sy = kSrur * fabs(yj), sm = min_inc / wj;
      inc = W.uni(sy > sm ? sy : sm);
      if (W.lane == j) yp = yj + inc;
    }
    const double f = rhs<ABC, TH>(m, L, W, yp, Fi, ns);
    if (j < 0) {
      f0 = f;
      const double fnorm = W.uni(sqrt(wrms2<S>(W, f0, ewt, inv_n)));
      min_inc = fnorm != 0.0 ? 1000.0 * fabs(h) * kUround * n * fnorm : 1.0;
      wave_lds_sync();
      for (int e = W.lane; e < S * S; e += W.kLanes)
        M[e] = e % (S + 1) == 0 ? static_cast<LT>(1) : static_cast<LT>(0);
    } else {
      const double col = (f - f0) / inc;
      wave_lds_sync();
      if (W.lane < n) M[j * S + W.lane] = static_cast<LT>((W.lane == j ? 1.0 : 0.0) - gamma * col);
    }
  }
  wave_lds_sync();
  const int lr = W.lane < S ? W.lane : 0;
#pragma unroll
  for (int j = 0; j < S; ++j) {
    const LT v = M[j * S + lr];
    a[j] = W.lane < S ? v : static_cast<LT>(0);
  }
  wave_lds_sync();
}

// ---------------------------------------------------------------------------
// dense LU with partial pivoting, one row per lane
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t abs_key(double v) {
  return (__builtin_bit_cast(uint64_t, v) & 0x7FFFFFFFFFFFFFFFull) + 1ull;
}
__device__ __forceinline__ uint64_t abs_key(float v) {
  return static_cast<uint64_t>(__builtin_bit_cast(uint32_t, v) & 0x7FFFFFFFu) + 1ull;
}

// Four in-place updates a_j <- ng * b_j + a_j whose broadcast operands b_j
// sit in scalar registers just written by v_readlane: one pair of wait states
// at the top covers all four FMAs (the first one may read the last register
// written).
__device__ __forceinline__ void fmac4s(double &a0, double &a1, double &a2, double &a3, double ng,
                                       double b0, double b1, double b2, double b3) {
  asm("s_nop 1\n\tv_fmac_f64 %0, %4, %8\n\tv_fmac_f64 %1, %5, %8\n\t"
      "v_fmac_f64 %2, %6, %8\n\tv_fmac_f64 %3, %7, %8"
      : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3)
      : "s"(b0), "s"(b1), "s"(b2), "s"(b3), "v"(ng));
}
__device__ __forceinline__ void fmac4s(float &a0, float &a1, float &a2, float &a3, float ng, float b0,
                                       float b1, float b2, float b3) {
  asm("s_nop 1\n\tv_fmac_f32 %0, %4, %8\n\tv_fmac_f32 %1, %5, %8\n\t"
      "v_fmac_f32 %2, %6, %8\n\tv_fmac_f32 %3, %7, %8"
      : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3)
      : "s"(b0), "s"(b1), "s"(b2), "s"(b3), "v"(ng));
}
// Slot updated i-th by an in-place Gauss-Jordan step on slot E: slot E + 1
// first (the next step's column, so that its pivot search can start while
// the rest of the row is updated), then the others in ascending order.
template <int S, int E>
constexpr int gj_slot(int i) {
  if (E + 1 < S) {
    if (i == 0) return E + 1;
    --i;
  }
  for (int j = 0;; ++j) {
    if (j == E || j == E + 1) continue;
    if (i-- == 0) return j;
  }
}

// In-place update a_j += ng * a_pj of the S - 1 slots other than E, from the
// I-th in gj_slot order; four per asm block where one wave holds one cell.
template <int S, int E, int I, typename LT, int G>
__device__ __forceinline__ void gj_update(LT (&a)[S], const Grp<G> &W, int p, LT ng) {
  constexpr int N = S - 1;
  if constexpr (G == 1 && I + 4 <= N) {
    constexpr int j0 = gj_slot<S, E>(I), j1 = gj_slot<S, E>(I + 1), j2 = gj_slot<S, E>(I + 2),
                  j3 = gj_slot<S, E>(I + 3);
    const LT b0 = W.bcast(a[j0], p), b1 = W.bcast(a[j1], p), b2 = W.bcast(a[j2], p),
             b3 = W.bcast(a[j3], p);
    fmac4s(a[j0], a[j1], a[j2], a[j3], ng, b0, b1, b2, b3);
    gj_update<S, E, I + 4>(a, W, p, ng);
  } else if constexpr (I < N) {
    constexpr int j = gj_slot<S, E>(I);
    a[j] = fma(ng, W.bcast(a[j], p), a[j]);
    gj_update<S, E, I + 1>(a, W, p, ng);
  }
}

// One Gauss-Jordan step on the cell's S x S Newton matrix (row i in lane i's
// registers): eliminates the column held in slot E.  Its pivot is the largest
// |a_iE| among rows not yet used, lowest row on ties (the pivot sequence of an
// LU factorisation with partial pivoting); every other row is updated as
// row_i -= (a_iE / p) row_p and slot E becomes that column of the
// accumulated inverse.  Pivot rows stay unscaled (all later updates are linear
// in them): the owner of a pivot keeps 1/p and divides its row at the end, so
// each entry costs one FMA per step and large pivots cause no cancellation.
// SH = 0 updates the slots in place; SH > 0 (the last step of a block, E =
// SH - 1) also rotates the row by SH slots: slot j goes to j - SH and slots
// 0..SH-1 to S-SH..S-1, so that the next block again eliminates slots 0, 1, ...
template <int S, int E, int SH, typename LT, int G>
__device__ __forceinline__ void gj_step(LT (&a)[S], const Grp<G> &W, int k, int &piv, LT &dinv,
                                        int &info) {
  int p;
  bool zero_pivot;
  if constexpr (sizeof(LT) == 4) {
    const uint32_t key = piv < 0 ? static_cast<uint32_t>(abs_key(a[E])) : 0u;
    const uint32_t kmax = W.template max_u32<(S + 15) / 16>(key);
    p = W.first(key == kmax);
    zero_pivot = kmax <= 1u;
  } else {
    // exact 64-bit maximum in two 32-bit passes: high words, then the low
    // words of the lanes that tie on the high word.  With one cell per wave
    // and S > 16, a high word held by one lane only decides alone (the
    // low-word pass would return that lane, and its key is not zero); ties,
    // the all-zero column among them, take the second pass.  (The smallest
    // kernels, whose elimination is a minor cost, stay without the extra
    // branch: it costs them spilled registers.)
    constexpr bool kShortcut = G == 1 && S > 16;
    const uint64_t key = piv < 0 ? abs_key(a[E]) : 0ull;
    const uint32_t hi = static_cast<uint32_t>(key >> 32), lo = static_cast<uint32_t>(key);
    const uint32_t hmax = W.template max_u32<(S + 15) / 16>(hi);
    uint64_t tie = 0;
    if constexpr (kShortcut) tie = __ballot(hi == hmax);
    if (kShortcut && __builtin_popcountll(tie) == 1) {
      p = __builtin_ctzll(tie);
      zero_pivot = false;
    } else {
      const uint32_t lmax = W.template max_u32<(S + 15) / 16>(hi == hmax ? lo : 0u);
      p = W.first(hi == hmax && lo == lmax);
      zero_pivot = hmax == 0u && lmax <= 1u;
    }
  }
  if (zero_pivot && info == 0) info = k + 1;
  const bool is_p = W.lane == p;
  const LT pk = W.bcast(a[E], p);
  const LT rp = rcp(pk);
  const LT ng = is_p ? static_cast<LT>(0) : -(a[E] * rp);
  if constexpr (S > 16) {
    // selects, not a branch: a block of steps stays one basic block
    piv = is_p ? k : piv;
    dinv = is_p ? rp : dinv;
  } else if (is_p) {
    piv = k;
    dinv = rp;
  }
  const LT col = is_p ? static_cast<LT>(1) : ng;  // new column of the inverse
  if constexpr (SH == 0) {
    gj_update<S, E, 0>(a, W, p, ng);
    a[E] = col;
  } else {
    static_assert(E == SH - 1, "a block rotates on its last step");
    gj_update<S, E, 0>(a, W, p, ng);
    a[E] = col;
    LT t[SH];
#pragma unroll
    for (int u = 0; u < SH; ++u) t[u] = a[u];
#pragma unroll
    for (int j = SH; j < S; ++j) a[j - SH] = a[j];
#pragma unroll
    for (int u = 0; u < SH; ++u) a[S - SH + u] = t[u];
  }
}

// steps E = 0 .. B-1 of a block of B steps starting at step k0
template <int S, int B, int E, typename LT, int G>
__device__ __forceinline__ void gj_block(LT (&a)[S], const Grp<G> &W, int k0, int &piv, LT &dinv,
                                         int &info) {
  if constexpr (E < B) {
    gj_step<S, E, (E == B - 1 ? B : 0)>(a, W, k0 + E, piv, dinv, info);
    gj_block<S, B, E + 1>(a, W, k0, piv, dinv, info);
  }
}

// Inverts the cell's S x S Newton matrix M (row i in lane i's registers) by
// Gauss-Jordan elimination with partial pivoting (gj_step), in blocks of four
// (eight above 32 species) steps whose slot indices are static, so the block
// loop need not be unrolled (at S = 53 the unrolled form would not fit the
// instruction cache) and only the last step of a block writes its row to
// rotated slots.  After S steps slot k
// holds the inverse column of step k, i.e. column p_k.  M^{-1} is written to
// LDS in natural order, column-major (entry (r, c) at c*S + r), so that a
// solve is one lane-parallel matrix-vector product.  T > 0: M^{-1} is kept in
// slot order instead ((r, k) at k*S + r holds M^{-1}(r, p_k)), slots 0 .. S-T-1
// in LDS and the last T in registers of lane r (moved there from the lane
// that computed row r by ds_bpermute), so the LDS area is (S - T) S entries.
// Returns 0, or k+1 for the first column k without a nonzero pivot (the
// elimination then runs on garbage).
template <int S, typename LT, int T = 0, int G>
__device__ __forceinline__ int gj_invert(LT (&a)[S], const Grp<G> &W, const Lds &L,
                                         InvTail<T, LT> *tail = nullptr) {
  static_assert(T == 0 || (G == 1 && sizeof(LT) == 8), "an inverse tail: FP64, one cell per wave");
  // steps per block (one register rotation per block): eight above 32
  // species, where the rotation's S moves are a larger share; sixteen
  // steps made the 53-species FP64 kernels' loop too large for the
  // instruction cache (27 % slower), eight at 21 species gained nothing
  constexpr int B = S > 32 ? 8 : 4;
  int piv = W.lane < S ? -1 : 1 << 20;
  int info = 0;
  LT dinv = static_cast<LT>(1);  // 1 / own pivot
  for (int k0 = 0; k0 + B <= S; k0 += B) gj_block<S, B, 0>(a, W, k0, piv, dinv, info);
  constexpr int BT = S % B;
  if constexpr (BT > 0) gj_block<S, BT, 0>(a, W, S - BT, piv, dinv, info);
  // lane i holds row piv(i) of M^{-1} (times its pivot); slot k is column
  // perm[k], the row that was the pivot of step k
  int *perm = L.perm;
  LT *inv = reinterpret_cast<LT *>(L.fac);
  wave_lds_sync();
  if (W.lane < S) perm[piv] = W.lane;
  wave_lds_sync();
  if constexpr (T == 0) {
    if (W.lane < S) {
#pragma unroll
      for (int k = 0; k < S; ++k) inv[perm[k] * S + piv] = a[k] * dinv;
    }
  } else {
    if (W.lane < S) {
#pragma unroll
      for (int k = 0; k < S - T; ++k) inv[k * S + piv] = a[k] * dinv;
    }
    // lane r takes row r from the lane whose pivot step put it there
    const int src = W.lane < S ? perm[W.lane] : W.lane;
#pragma unroll
    for (int t = 0; t < T; ++t) tail->v[t] = lane_pull(a[S - T + t] * dinv, src);
  }
  wave_lds_sync();
  return info;
}

// x = M^{-1} b with the inverse in LDS; lane i passes b_i and gets x_i.
// SPLIT: three partial sums (FP32 inverse of isothermal kernels, see below).
// T > 0 (gj_invert's slot order with a register tail): the sum runs over the
// slots k, b_{p_k} gathered to lane k first.
template <int S, typename LT, bool SPLIT, int T = 0, int G>
__device__ __forceinline__ double inv_solve(const Lds &L, const Grp<G> &W, double b,
                                            const InvTail<T, LT> *tail = nullptr) {
  const LT *inv = reinterpret_cast<const LT *>(L.fac);
  LT *bb = reinterpret_cast<LT *>(L.yb);
  if constexpr (T > 0) {
    static_assert(!SPLIT && sizeof(LT) == 8, "an inverse tail: FP64, one chain");
    wave_lds_sync();
    const double bk = lane_pull(b, W.lane < S ? L.perm[W.lane] : W.lane);
    if (W.lane < S) bb[W.lane] = bk;
    wave_lds_sync();
    const int lr = W.lane < S ? W.lane : 0;
    LT acc = 0;
#pragma unroll
    for (int k = 0; k < S - T; ++k) acc = fma(inv[k * S + lr], bb[k], acc);
#pragma unroll
    for (int t = 0; t < T; ++t) acc = fma(tail->v[t], bb[S - T + t], acc);
    return W.lane < S ? static_cast<double>(acc) : 0.0;
  }
  wave_lds_sync();
  if (W.lane < S) bb[W.lane] = static_cast<LT>(b);
  wave_lds_sync();
  const int lr = W.lane < S ? W.lane : 0;
  if constexpr (SPLIT) {
    // three partial sums (column c into sum c mod 3, added in a fixed order)
    // shorten the dependent FMA chain, and the unrolled loop issues the LDS
    // reads early: -2.6 % time at 21 species, -3.7 % at 53 with the FP32
    // inverse.  With the FP64 inverse, or in the non-isothermal kernels, the
    // same form raises register pressure and runs slower.
    LT acc0 = 0, acc1 = 0, acc2 = 0;
#pragma unroll
    for (int c = 0; c < S; c += 3) {
      acc0 = fma(inv[c * S + lr], bb[c], acc0);
      if (c + 1 < S) acc1 = fma(inv[(c + 1) * S + lr], bb[c + 1], acc1);
      if (c + 2 < S) acc2 = fma(inv[(c + 2) * S + lr], bb[c + 2], acc2);
    }
    return W.lane < S ? static_cast<double>((acc0 + acc1) + acc2) : 0.0;
  } else {
    LT acc = 0;
#pragma unroll
    for (int c = 0; c < S; ++c) acc = fma(inv[c * S + lr], bb[c], acc);
    return W.lane < S ? static_cast<double>(acc) : 0.0;
  }
}

// ---------------------------------------------------------------------------
// per-cell integration
// ---------------------------------------------------------------------------


// Lock-step batches (the paper's batches, Sec. 2): the waves of a block
// integrate the cells of one batch with one step size and order and one WRMS
// norm over the batch vector.  Every decision of the step control then rests
// on batch reductions: each wave puts its wave-uniform partial value into its
// LDS slot, one block barrier, and every wave combines all slots in slot
// order, so every wave computes the same value and takes the same branch
// (the barriers need exactly that).  Slots alternate between two halves, so
// one barrier per reduction suffices: a half is written again only after
// every wave has passed the barrier of the reduction in between.  A wave
// without a cell (the last batch can be short) repeats the first cell's work
// and contributes 0.  LOCK = false: every reduction is the identity.
constexpr int kMaxBatch = 16;

template <bool LOCK>
struct BatchRed {
  double *slots = nullptr;  // [2][kMaxBatch] in the block's LDS
  int wid = 0, nw = 1;      // this wave's slot, waves of the block
  int half = 0;
  bool active = true;       // the wave integrates a cell of the batch
  __device__ double sum(double v) {
    if constexpr (!LOCK) {
      return v;
    } else {
      double *h = slots + half * kMaxBatch;
      half ^= 1;
      if (threadIdx.x % kWave == 0) h[wid] = active ? v : 0.0;
      __syncthreads();
      double t = 0.0;
      for (int k = 0; k < nw; ++k) t += h[k];
      return uni(t);
    }
  }
  __device__ double max(double v) {  // of non-negative values
    if constexpr (!LOCK) {
      return v;
    } else {
      double *h = slots + half * kMaxBatch;
      half ^= 1;
      if (threadIdx.x % kWave == 0) h[wid] = active ? v : 0.0;
      __syncthreads();
      double t = 0.0;
      for (int k = 0; k < nw; ++k) t = fmax(t, h[k]);
      return uni(t);
    }
  }
  __device__ bool any(bool p) { return LOCK ? max(p ? 1.0 : 0.0) != 0.0 : p; }
};

// Linear solve of the inexact Newton iteration (Table 1, approaches 1A/1B):
// GMRES on the system scaled by the error weights (Sec. 2, Eq. (5),
// S1 = S2 = diag(w), no preconditioner) for (I - gamma J(y)) x = b, with J v
// the difference quotient (f(y + sigma v) - f(y)) / sigma, sigma =
// 1 / ||v||_wrms, and fy = f(y).  Initial guess 0; modified Gram-Schmidt
// Arnoldi; Givens rotations reduce the Hessenberg matrix to triangular form
// and give the residual norm of the scaled system as the magnitude of the
// last rotated right-hand-side entry (Sec. 2, after Eq. (6)).
// Stops at maxl basis vectors or when that norm is at most delta (the
// 2-norm of Eq. (6)).  Lane i holds entry i of y, fy, w and b (w = 0
// past the state); the basis and the Hessenberg data live in the wave's LDS
// (KryLayout), so the loop is not unrolled and the right-hand side is
// inlined once.  Returns 0 when converged, 1 when the residual was reduced
// but not to delta, 2 otherwise; x receives the lane's solution entry and
// nli the iterations (one right-hand side each).
template <int S, bool ABC, bool TH, int G>
__device__ int gmres(const MechDev &m, const Lds &L, const Grp<G> &W, double y, double fy,
                     double Fi, double ewt, double gamma, double b, int maxl, double delta,
                     int ns, int n, double inv_n, double &x, int &nli) {
  constexpr int NR = (S + 15) / 16;
  const KryLayout K(S, maxl);
  double *const kb = L.kry;
  const int ld = maxl + 1;  // Hessenberg column stride
  const bool own = W.lane < n;
  const int li = own ? W.lane : 0;
  const double rw = own ? 1.0 / ewt : 0.0;  // S2^{-1} (one division per solve)
  const double r0 = own ? ewt * b : 0.0;  // b~ = S1 b, the residual of x = 0
  const double beta = W.uni(sqrt(W.template sum<NR>(r0 * r0)));
  x = 0.0;
  if (beta <= delta) return 0;
  wave_lds_sync();
  if (own) kb[K.V + li] = r0 * W.uni(rcp(beta));
  double gl = beta;  // last entry of the rotated right-hand side
  double rho = beta;
  int k = 0;
  // every basis vector has unit 2-norm in the scaled space, so v = S2^{-1} V_l
  // has ||v||_wrms = 1 / sqrt(n): sigma = sqrt(n) without a reduction
  const double vn = W.uni(sqrt(inv_n));
  const double sigma = W.uni(sqrt(static_cast<double>(n)));
  for (int l = 0; l < maxl; ++l) {
    wave_lds_sync();
    // w = A~ V_l = S1 (v - gamma J v) with v = S2^{-1} V_l; sigma = 1 / ||v||
    // and J v = (f(y + sigma v) - f(y)) ||v||
    const double vl = own ? kb[K.V + l * S + li] : 0.0;
    const double v = vl * rw;
    const double fp = rhs<ABC, TH>(m, L, W, y + sigma * v, Fi, ns);
    nli++;
    double w = own ? ewt * (v - gamma * ((fp - fy) * vn)) : 0.0;
    // modified Gram-Schmidt: column l of the Hessenberg matrix
    for (int j = 0; j <= l; ++j) {
      const double vj = own ? kb[K.V + j * S + li] : 0.0;
      const double d = W.uni(W.template sum<NR>(w * vj));
      if (W.lane == 0) kb[K.H + l * ld + j] = d;
      w -= d * vj;
    }
    const double hn = W.uni(sqrt(W.template sum<NR>(w * w)));
    wave_lds_sync();
    // the earlier rotations, then the one that zeroes the subdiagonal entry
    // (each store goes to an entry no later read of the loop touches)
    double a = kb[K.H + l * ld];
    for (int j = 0; j < l; ++j) {
      const double c = kb[K.cs + j], sn = kb[K.sn + j], a1 = kb[K.H + l * ld + j + 1];
      const double top = c * a + sn * a1;
      a = -sn * a + c * a1;
      if (W.lane == 0) kb[K.H + l * ld + j] = top;
    }
    const double r = W.uni(sqrt(fma(a, a, hn * hn)));  // a and hn are O(beta): no overflow
    if (!(r > 0.0)) break;  // singular Hessenberg column: keep k columns
    const double c = W.uni(a / r), sn = W.uni(hn / r);
    wave_lds_sync();
    if (W.lane == 0) {
      kb[K.H + l * ld + l] = r;
      kb[K.cs + l] = c;
      kb[K.sn + l] = sn;
      kb[K.g + l] = c * gl;
    }
    gl = W.uni(-sn * gl);
    rho = fabs(gl);
    k = l + 1;
    if (rho <= delta) break;
    if (l + 1 < maxl) {
      if (!(hn > 0.0)) break;
      if (own) kb[K.V + (l + 1) * S + li] = w * W.uni(rcp(hn));
    }
  }
  // back substitution for the coefficients, then x = S2^{-1} sum_j c_j V_j
  wave_lds_sync();
  for (int i = k - 1; i >= 0; --i) {
    double t = kb[K.g + i];
    for (int j = i + 1; j < k; ++j) t -= kb[K.H + j * ld + i] * kb[K.c + j];
    const double ci = W.uni(t / kb[K.H + i * ld + i]);
    wave_lds_sync();
    if (W.lane == 0) kb[K.c + i] = ci;
    wave_lds_sync();
  }
  double t = 0.0;
  for (int j = 0; j < k; ++j) t += kb[K.c + j] * (own ? kb[K.V + j * S + li] : 0.0);
  x = t * rw;
  wave_lds_sync();
  if (rho <= delta) return 0;
  return rho < beta ? 1 : 2;
}

// RES: a resumed integration (Resume); its Newton matrix is the analytic one
// in FP64, one cell per wave.
template <int S, typename LT, int TAB, int G, bool ABC, bool TH, int LIN, bool LOCK = false,
          bool RES = false>
__device__ __forceinline__ void integrate_cell(const Params &P, int64_t cell, const Grp<G> &W,
                                               double *lds, double *kk_slot,
                                               BatchRed<LOCK> br = BatchRed<LOCK>{},
                                               int batch_cells = 1, const Resume *rs = nullptr) {
  static_assert(!RES || (G == 1 && !LOCK && !TH && LIN == kLinAnalytic && sizeof(LT) == 8),
                "resumed integrations: FP64 direct solver, analytic Jacobian, one cell per wave");
  constexpr bool KRY = LIN == kLinGmres;
  const MechDev &m = P.mech;
  const int R = m.R;
  const int ns = m.S;  // species; a non-isothermal state also holds T at entry ns
  const Lds L = carve<TAB, TH, KRY>(lds, R, m.rx, kk_slot, S, static_cast<int>(sizeof(LT)));
  if (W.lane == 0) L.yb[kEmptySlot] = 1.0;  // empty reaction slots multiply by 1
  double *const C = L.C;
  const int n = P.n_sp;
  const double inv_n = 1.0 / n;
  const bool own = W.lane < n;
  // squared WRMS norm of Eq. (3) over the cell, or over the lock-step batch
  // vector (batch_cells n entries)
  const double inv_bn = 1.0 / (static_cast<double>(batch_cells) * n);
  auto norm2 = [&](double v, double w) {
    if constexpr (LOCK) {
      const double t = v * w;  // w = 0 on lanes without a species
      return W.uni(br.sum(W.uni(W.template sum<(S + 15) / 16>(t * t))) * inv_bn);
    } else {
      return wrms2<S>(W, v, w, inv_n);
    }
  };
  const double rtol = P.rtol, t0 = P.t0, tout = P.tout;
  const int qmax = P.max_order < 1 ? 1 : (P.max_order > kQmax ? kQmax : P.max_order);

  // rate constants (Arrhenius, frozen T); a non-isothermal cell keeps
  // ln k_f0 and -exp(-ln K) and evaluates them at its temperature later
  const double T = (P.T && !TH) ? P.T[cell] : 1.0;
  wave_lds_sync();
  for (int r = W.lane; r < R; r += W.kLanes) {
    if constexpr (TH) {
      double lk = m.lnA[r];
      if (P.kscale) lk += log(P.kscale[cell * P.ldk + r]);
      L.kk[2 * r] = lk;
      L.kk[2 * r + 1] = m.reversible ? -exp(-m.lnK[r]) : -0.0;
      if constexpr (TAB == kTabLds) const_cast<int2 *>(L.rx)[r] = reinterpret_cast<const int2 *>(m.rx)[r];
      continue;
    }
    double lk = m.lnA[r];
    lk -= m.EaR[r] / T;
    double kf = exp(lk);
    if (P.kscale) kf *= P.kscale[cell * P.ldk + r];
    L.kk[2 * r] = kf;
    L.kk[2 * r + 1] = m.reversible ? -(kf * exp(-m.lnK[r])) : -0.0;
    if constexpr (TAB == kTabLds) const_cast<int2 *>(L.rx)[r] = reinterpret_cast<const int2 *>(m.rx)[r];
  }

  const double Fi = (own && P.F) ? P.F[cell * P.ldy + W.lane] : 0.0;
  const double atol_i = own ? (P.atol_len == 1 ? P.atol[0] : P.atol[W.lane]) : 1.0;
  const bool keep = (P.rec || P.ckpt) && !RES;  // this run records its steps for the adjoint
  // inverse slots in registers (kept from one setup to the next)
  constexpr int TL = inv_tail(S, static_cast<int>(sizeof(LT)), TH, LIN, LOCK, G);
  InvTail<TL, LT> itail;

  int status = kSuccess;
  int nst = 0, nfe = 0, nni = 0, nsetups = 0, netf = 0, ncfn = 0, nli = 0, ncfl = 0;
  int q = 1, qstep = 1;  // qstep: the order the last accepted step was taken with
  double t = t0, h = 0.0;
  double z[kQmax + 1];
#pragma unroll
  for (int j = 0; j <= kQmax; ++j) z[j] = 0.0;
  bool write_y = !RES;
  int qwait = 2, nst_setup = 0;
  double R2 = 1.0;  // squared Newton convergence rate
  bool need_setup = true, have_eprev = false, rebuilt = false;
  double e = 0.0, eprev = 0.0;
  double f = 0.0, ewt = 0.0;

  if constexpr (RES) {
    // the state after ck[kNst] accepted steps, as the step loop left it
    const double *ck = rs->ck;
#pragma unroll
    for (int j = 0; j <= kQmax; ++j) z[j] = own ? ck[Ckpt::vec(j, S) + W.lane] : 0.0;
    eprev = own ? ck[Ckpt::vec(Ckpt::kVecEprev, S) + W.lane] : 0.0;
    t = uni(ck[Ckpt::kT]);
    h = uni(ck[Ckpt::kH]);
    q = static_cast<int>(uni(ck[Ckpt::kQ]));
    nst = static_cast<int>(uni(ck[Ckpt::kNst]));
    qwait = static_cast<int>(uni(ck[Ckpt::kQwait]));
    nst_setup = static_cast<int>(uni(ck[Ckpt::kNstSetup]));
    R2 = uni(ck[Ckpt::kR2]);
    need_setup = uni(ck[Ckpt::kNeedSetup]) != 0.0;
    have_eprev = uni(ck[Ckpt::kHaveEprev]) != 0.0;
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k <= kQmax; ++k) C[Ctl::kHist + k] = ck[Ckpt::kHist + k];
    C[Ctl::kEtaMax] = ck[Ckpt::kEtaMax];
    C[Ctl::kHprev] = ck[Ckpt::kHprev];
    C[Ctl::kGammaBar] = ck[Ckpt::kGammaBar];
    if (!need_setup) {
      // the inverse the run held: the same matrix at the same state and gamma
      const double zs = own ? ck[Ckpt::vec(Ckpt::kVecSetup, S) + W.lane] : 0.0;
      LT a[S];
      newton_matrix<S, LT, ABC, TL>(a, m, L, W, zs, uni(ck[Ckpt::kGammaBar]), false);
      gj_invert<S, LT, TL>(a, W, L, &itail);
    }
  } else {
    const double yin = own ? P.y[cell * P.ldy + W.lane] : 0.0;
    if (keep && own) P.rec_y0[cell * P.rec_stride + W.lane] = yin;
    if (br.any(W.any(!isfinite(T) || (own && !isfinite(yin))))) {
      status = kNonfinite;
      write_y = false;
    }
    if (status == kSuccess) {
      z[0] = yin;
      f = rhs<ABC, TH>(m, L, W, yin, Fi, ns);
      nfe = 1;
      if (br.any(W.any(own && !isfinite(f)))) {
        status = kNonfinite;
        write_y = false;
      }
    }
    if (status == kSuccess) {
      // initial step (same reading as the oracle)
      ewt = own ? 1.0 / (rtol * fabs(yin) + atol_i) : 0.0;
      const double tdist = fabs(tout - t0);
      const double hlb = 100.0 * kUround * fmax(fabs(t0), fabs(tout));
      double hub = 0.1 * tdist;
      const double hub_inv = br.max(
          W.uni(W.template max<(S + 15) / 16>(own ? fabs(f) / (0.1 * fabs(yin) + atol_i) : 0.0)));
      if (hub * hub_inv > 1.0) hub = 1.0 / hub_inv;
      if (hub < hlb) {
        h = hub;
      } else {
        double hg = sqrt(hlb * hub), hnew = hg;
        bool at_ub = false;
        for (int it = 0; it < 4; ++it) {
          const double ft = rhs<ABC, TH>(m, L, W, yin + hg * f, Fi, ns);
          nfe++;
          const double ydd = (ft - f) / hg;
          const double yddnrm = sqrt(norm2(ydd, ewt));
          if (!(yddnrm > 0.0)) {
            at_ub = true;
            break;
          }
          hnew = W.uni(sqrt(2.0 / yddnrm));
          const double ratio = hnew / hg;
          hg = hnew;
          if (ratio >= 0.5 && ratio <= 2.0) break;
        }
        if (at_ub) {
          h = hub;
        } else {
          h = 0.5 * hnew;
          if (h < hlb) h = hlb;
          if (h > hub) h = hub;
        }
      }
      h = W.uni(h);
      z[1] = h * f;
    }

    wave_lds_sync();
#pragma unroll
    for (int k = 0; k <= kQmax; ++k) C[Ctl::kHist + k] = h;
    C[Ctl::kEtaMax] = 1.0e4;
    C[Ctl::kHprev] = h;
    C[Ctl::kGammaBar] = 0.0;
    if (keep && W.lane == 0) P.rec_hpad[cell] = h;
  }

  // step loop (same structure as the oracle: steps, attempts, Newton iterations)
  while (status == kSuccess && t < tout) {
    if constexpr (RES) {
      if (nst >= rs->stop) break;
    }
    if (nst >= P.max_steps) {
      status = kTooMuchWork;
      break;
    }
    if (keep && nst >= P.rec_cap) {
      // the record is full and time is left: stop at the last recorded step,
      // so that the returned state is the end point of the recorded map
      status = kRecordFull;
      break;
    }
    if (!RES && P.ckpt && nst % P.ckpt_every == 0) {
      // checkpoint nst / ckpt_every (nst < rec_cap <= ckpt_cap ckpt_every)
      // (vectors S apart: constant offsets from one address per lane)
      double *ck = P.ckpt + (cell * P.ckpt_cap + nst / P.ckpt_every) * Ckpt::stride(P.ckpt_vs);
      if (own) {
#pragma unroll
        for (int j = 0; j <= kQmax; ++j) ck[Ckpt::vec(j, S) + W.lane] = z[j];
        ck[Ckpt::vec(Ckpt::kVecEprev, S) + W.lane] = eprev;
      }
      wave_lds_sync();
      if (W.lane == 0) {
        ck[Ckpt::kT] = t;
        ck[Ckpt::kH] = h;
        ck[Ckpt::kQ] = q;
        ck[Ckpt::kNst] = nst;
        ck[Ckpt::kQwait] = qwait;
        ck[Ckpt::kNstSetup] = nst_setup;
        ck[Ckpt::kR2] = R2;
        ck[Ckpt::kNeedSetup] = need_setup ? 1.0 : 0.0;
        ck[Ckpt::kHaveEprev] = have_eprev ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k <= kQmax; ++k) ck[Ckpt::kHist + k] = C[Ctl::kHist + k];
        ck[Ckpt::kEtaMax] = C[Ctl::kEtaMax];
        ck[Ckpt::kHprev] = C[Ctl::kHprev];
        ck[Ckpt::kGammaBar] = C[Ctl::kGammaBar];
        ck[Ckpt::kQtaken] = qstep;
      }
      if (!need_setup && own)
        ck[Ckpt::vec(Ckpt::kVecSetup, S) + W.lane] = P.ckpt_setup[cell * P.ckpt_vs + W.lane];
    }
    ewt = own ? rcp(rtol * fabs(z[0]) + atol_i) : 0.0;  // from y^{n-1}, Eq. (3)
    int nef_step = 0, ncf_step = 0, nsf_step = 0;
    double dsm2 = 0.0, Cerr = 0.5;
    for (;;) {  // attempts of this step
      bool landing = false;
      if (t + h >= tout * (1.0 - 4.0 * kUround)) {
        const double hnew = W.uni(tout - t);
        nd_rescale(z, hnew / h);
        h = hnew;
        landing = true;
      }
      if (h <= 4.0 * kUround * fabs(t)) {
        status = kErrFailure;
        break;
      }
      nd_predict(z);
      double l1;
      {
        // xi_i = (t_n - t_{n-i}) / h and the coefficients of this attempt
        double xi[kQmax + 2], l[kQmax + 2];
        double sum = h;
        const double rh = rcp(h);
        xi[0] = 0.0;
        xi[1] = 1.0;
#pragma unroll
        for (int i = 2; i <= kQmax + 1; ++i) {
          sum += C[Ctl::kHist + i - 2];
          xi[i] = i <= q + 1 ? sum * rh : 0.0;
        }
        bdf_coeffs(q, xi, l, Cerr);
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i <= kQmax + 1; ++i) {
          C[Ctl::kXi + i] = xi[i];
          C[Ctl::kL + i] = l[i];
        }
        C[Ctl::kTn] = landing ? tout : t + h;
        l1 = W.uni(l[1]);
        Cerr = W.uni(Cerr);
      }
      const double rl1 = W.uni(rcp(l1));
      const double gamma = W.uni(h * rl1);
      double gamma_bar = W.uni(C[Ctl::kGammaBar]);
      bool fresh = false;
      // (gamma_bar = 0 before the first setup, which need_setup forces)
      // (GMRES kernels form no matrix and take no setups)
      if constexpr (!KRY) {
        if (need_setup || nst >= nst_setup + 20 || fabs(gamma * rcp(gamma_bar) - 1.0) > 0.3) {
          int info;
          {
            LT a[S];
            if constexpr (LIN == kLinDq) {
              dq_matrix<S, LT, ABC, TH>(a, m, L, W, z[0], Fi, gamma, h, ewt, ns, n, inv_n);
              nfe += n + 1;
            } else if constexpr (TH) {
              newton_matrix_thermal<S, LT>(a, m, L, W, z[0], Fi, gamma, ns);
            } else {
              newton_matrix<S, LT, ABC, TL>(a, m, L, W, z[0], gamma, false);
            }
            info = gj_invert<S, LT, TL>(a, W, L, &itail);
          }
          if (!RES && P.ckpt && own) P.ckpt_setup[cell * P.ckpt_vs + W.lane] = z[0];
          nsetups++;
          nst_setup = nst;
          gamma_bar = gamma;
          C[Ctl::kGammaBar] = gamma;
          R2 = 1.0;
          need_setup = false;
          fresh = true;
          if (br.any(info != 0)) {
            // singular Newton matrix: recoverable once per step by cutting h
            nd_unpredict(z);
            need_setup = true;
            if (++nsf_step >= 2) {
              status = kSetupFailure;
              break;
            }
            nd_rescale(z, 0.25);
            h = W.uni(h * 0.25);
            C[Ctl::kEtaMax] = 1.0;
            continue;
          }
        }
      }
      const double cfac =
          KRY ? 1.0 : W.uni(gamma != gamma_bar ? 2.0 * rcp(1.0 + gamma * rcp(gamma_bar)) : 1.0);
      // GMRES tolerance, Eq. (6): c_l = 0.05 times the Newton
      // tolerance c_eps eps = 0.1 / Cerr, in the scaled 2-norm (sqrt(n) times
      // the WRMS norm)
      const double ltol = KRY ? W.uni(0.005 * rcp(Cerr) * sqrt(static_cast<double>(n))) : 0.0;

      // Newton iteration on G(e) = e - gamma f(z_0 + e) + z_1 / l_1, Eq. (4)
      bool conv = false;
      double dprev2 = 0.0;
      // stopping test of Eq. (4) with eps = 1/Cerr, on squared norms
      const double tol2 = 0.01 * W.uni(rcp(Cerr * Cerr));
      e = 0.0;
      for (int mit = 0; mit < 3; ++mit) {
        f = rhs<ABC, TH>(m, L, W, z[0] + e, Fi, ns);
        nfe++;
        nni++;
        const double Gi = e - gamma * f + z[1] * rl1;
        double delta;
        if constexpr (KRY) {
          // inexact Newton: J at the current iterate; a reduced but
          // unconverged residual is accepted on the first iteration only
          int nl = 0;
          const int lret = gmres<S, ABC, TH>(m, L, W, z[0] + e, f, Fi, ewt, gamma, -Gi,
                                             P.gmres_maxl, ltol, ns, n, inv_n, delta, nl);
          nli += nl;
          nfe += nl;
          if (lret != 0) ncfl++;
          if (lret == 2 || (lret == 1 && mit > 0)) break;
        } else {
          delta = inv_solve<S, LT, sizeof(LT) == 4 && !TH, TL>(L, W, -Gi, &itail);
          if (cfac != 1.0) delta *= cfac;
        }
        e += delta;
        const double d2 = norm2(delta, ewt);
        if (!isfinite(d2)) break;
        if (mit >= 1) {
          const double ratio2 = d2 * rcp(dprev2);
          R2 = W.uni(0.09 * R2 > ratio2 ? 0.09 * R2 : ratio2);
        }
        if ((R2 < 1.0 ? R2 : 1.0) * d2 <= tol2) {
          conv = true;
          break;
        }
        if (mit >= 1 && d2 > 4.0 * dprev2) break;
        dprev2 = d2;
      }
      if (!conv) {
        ncfn++;
        nd_unpredict(z);
        if (++ncf_step >= P.max_ncf) {
          status = kConvFailure;
          break;
        }
        if (fresh || KRY) {
          nd_rescale(z, 0.25);
          h = W.uni(h * 0.25);
          C[Ctl::kEtaMax] = 1.0;
        }
        need_setup = true;
        continue;
      }

      // local error test (Sec. 2)
      dsm2 = W.uni(Cerr * Cerr * norm2(e, ewt));
      if (dsm2 <= 1.0) break;
      netf++;
      nd_unpredict(z);
      if (++nef_step >= P.max_netf) {
        status = kErrFailure;
        break;
      }
      C[Ctl::kEtaMax] = 1.0;
      if (nef_step >= 3) {
        // restart at order 1 from the last accepted y
        const double hnew = W.uni(0.1 * h);
        q = 1;
        const double f0 = rhs<ABC, TH>(m, L, W, z[0], Fi, ns);
        nfe++;
#pragma unroll
        for (int j = 2; j <= kQmax; ++j) z[j] = 0.0;
        z[1] = hnew * f0;
        h = hnew;
        qwait = 2;
        have_eprev = false;
        rebuilt = true;
      } else {
        double eta = eta_from2(6.0, dsm2, q + 1);
        if (eta < 0.1) eta = 0.1;
        if (nef_step >= 2 && eta > 0.2) eta = 0.2;
        eta = W.uni(eta);
        nd_rescale(z, eta);
        h = W.uni(h * eta);
      }
    }
    if (status != kSuccess) break;

    // accept: correct the Nordsieck array
    t = W.uni(C[Ctl::kTn]);
    // l_j = 0 for j > q
#pragma unroll
    for (int j = 0; j <= kQmax; ++j) z[j] = fma(C[Ctl::kL + j], e, z[j]);
    nst++;
    wave_lds_sync();
#pragma unroll
    for (int k = kQmax; k >= 1; --k) C[Ctl::kHist + k] = C[Ctl::kHist + k - 1];
    C[Ctl::kHist] = h;
    qstep = q;
    if (RES ? static_cast<unsigned>(nst - rs->first) < static_cast<unsigned>(rs->n_rows)
            : P.rec != nullptr) {
      double *rp = RES ? rs->rows + static_cast<int64_t>(nst - rs->first) * P.rec_stride
                       : P.rec + (static_cast<int64_t>(cell) * P.rec_cap + (nst - 1)) * P.rec_stride;
      if (own) rp[W.lane] = z[0];
      if (W.lane == 0) {
        rp[n] = h;
        rp[n + 1] = static_cast<double>(q + (rebuilt ? 256 : 0));
      }
    }
    rebuilt = false;
    const double hstep = h;
    qwait--;
    if (qwait == 1 && q < qmax) {
      eprev = e;
      C[Ctl::kHprev] = hstep;
      have_eprev = true;
    }
    const double eta_max = W.uni(C[Ctl::kEtaMax]);
    if (t < tout) {
      if (eta_max == 1.0) {
        if (qwait < 2) qwait = 2;  // right after a failure: hold h and q
      } else {
        // without an order decision this step, h changes only if eta >= 1.5
        double eta = 0.0;
        int qnew = q;
        if (qwait == 0) {
          qwait = 2;
          const bool lower = q > 1, higher = q < qmax && have_eprev;
          double lte2m = 0.0, lte2p = 0.0;
          if (lower) {
            const double lte = factorial(q - 1) / harmonic(q - 1);
            lte2m = lte * lte * norm2(nd_get(z, q), ewt);
          }
          if (higher) {
            const double r = ipow(hstep / C[Ctl::kHprev], q + 1);
            const double c = rcp((q + 2) * harmonic(q + 1));
            lte2p = c * c * norm2(e - r * eprev, ewt);
          }
          // the three candidates' roots in one evaluation: the group's lane 0
          // takes order q, lane 1 order q - 1, lane 2 order q + 1 (each lane
          // computes the same function of its own inputs, so the values are
          // those of three separate evaluations)
          const int gl = W.lane;
          const double et = eta_from2(gl == 2 ? 10.0 : 6.0, gl == 0 ? dsm2 : gl == 1 ? lte2m : lte2p,
                                      gl == 0 ? q + 1 : gl == 1 ? q : q + 2);
          eta = W.uni(W.bcast(et, 0));
          if (lower) {
            const double eta_qm1 = W.uni(W.bcast(et, 1));
            if (eta_qm1 > eta) {
              eta = eta_qm1;
              qnew = q - 1;
            }
          }
          if (higher) {
            const double eta_qp1 = W.uni(W.bcast(et, 2));
            if (eta_qp1 > eta) {
              eta = eta_qp1;
              qnew = q + 1;
            }
          }
        } else if (36.0 * dsm2 <= hold_bound(q + 1)) {
          eta = W.uni(eta_from2(6.0, dsm2, q + 1));
        }
        if (eta >= 1.5) {
          if (eta > eta_max) eta = eta_max;
          if (qnew == q + 1) {
            // add (e / xi_{q+1}) x Lambda(x): keeps interpolation, raises the degree
            const double c = 1.0 / C[Ctl::kXi + q + 1];
#pragma unroll
            for (int j = 1; j <= kQmax; ++j) {
              if (j == q + 1) z[j] = 0.0;
              if (j <= q + 1) z[j] += c * C[Ctl::kL + j - 1] * e;
            }
          } else if (qnew == q - 1) {
            // subtract z_q x prod_{i<q} (x + xi_i)
            double c[kQmax + 2];
#pragma unroll
            for (int j = 0; j <= kQmax + 1; ++j) c[j] = 0.0;
            c[1] = 1.0;
#pragma unroll
            for (int i = 1; i <= kQmax - 1; ++i)
              if (i <= q - 1) {
                const double xi_i = C[Ctl::kXi + i];
#pragma unroll
                for (int j = i + 1; j >= 1; --j) c[j] = c[j - 1] + xi_i * c[j];
              }
            const double zq = nd_get(z, q);
#pragma unroll
            for (int j = 1; j <= kQmax; ++j) {
              if (j < q) z[j] -= c[j] * zq;
              if (j == q) z[j] = 0.0;
            }
          }
          if (qnew != q) {
            q = qnew;
            qwait = q + 1;
            have_eprev = false;
          }
          nd_rescale(z, eta);
          h = W.uni(h * eta);
        }
      }
    }
    C[Ctl::kEtaMax] = 10.0;
  }

  if constexpr (RES) return;
  if (write_y && own && br.active) P.y[cell * P.ldy + W.lane] = z[0];
  if (W.lane == 0 && br.active) {
    P.status[cell] = status;
    if (P.stats) {
      CellStats st;
      st.status = status;
      st.nst = nst;
      st.nfe = nfe;
      st.nni = nni;
      st.nsetups = nsetups;
      st.netf = netf;
      st.ncfn = ncfn;
      st.q_last = q;
      st.nli = nli;
      st.ncfl = ncfl;
      st.h_last = h;
      st.t_reached = t;
      P.stats[cell] = st;
    }
    if (keep) P.rec_n[cell] = nst < P.rec_cap ? nst : P.rec_cap;
  }
}

// ---------------------------------------------------------------------------
// discrete adjoint of the frozen step sequence
// ---------------------------------------------------------------------------
//
// With the accepted step sizes h_n, orders q_n and restart flags held fixed
// and every corrector solved exactly, the forward run is a smooth map
// (y0, lnA) -> y(t_out):  step n predicts zp = A z (Pascal), solves
// y_n - gamma f(y_n) = zp_0 - zp_1 / l_1, corrects z = zp + l (y_n - zp_0);
// between steps z is rescaled by (h_n / h_{n-1})^j and the order changed
// (interpolation-preserving maps) or, after repeated error-test failures,
// rebuilt as [y, h f(y)].  The backward sweep applies the transposes of
// these maps in reverse; the solve uses (I - gamma J(y_n))^T with J at the
// recorded state.  d f / d lnA_r = nu_r q_r.

// (J^T v)_i for lane i, and pbar_r += scale q_r(y) (nu_r . v) (reaction r
// on lane r mod 64, accumulated in LDS).  vb: a 64-entry LDS buffer.
__device__ __forceinline__ double adj_scatter(const MechDev &m, const Lds &L, double *vb,
                                              double *pb, int li, double yi, double vi,
                                              double scale, bool want_jtv) {
  wave_lds_sync();
  L.yb[li] = yi;
  vb[li] = vi;
  L.fb[li] = 0.0;
  wave_lds_sync();
  for (int r = li; r < m.R; r += kWave) {
    const int2 w = L.rx[r];
    int a[3], b[3];
    double pf = L.kk[2 * r], pr = L.kk[2 * r + 1], s = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      a[k] = slot_species(w.x, k);
      b[k] = slot_species(w.y, k);
      // empty slots read yb = 1 and vb = 0 at kEmptySlot
      pf *= L.yb[a[k]];
      s -= vb[a[k]];
      pr *= L.yb[b[k]];
      s += vb[b[k]];
    }
    pb[r] += scale * (pf + pr) * s;
    if (want_jtv) {
      // d q_r / d y_j for each slot: the side's constant times the other slots
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (a[k] != kEmptySlot) {
          double d = L.kk[2 * r];
#pragma unroll
          for (int o = 0; o < 3; ++o)
            if (o != k) d *= L.yb[a[o]];
          atomicAdd(&L.fb[a[k]], d * s);
        }
        if (b[k] != kEmptySlot && m.reversible) {
          double d = L.kk[2 * r + 1];
#pragma unroll
          for (int o = 0; o < 3; ++o)
            if (o != k) d *= L.yb[b[o]];
          atomicAdd(&L.fb[b[k]], d * s);
        }
      }
    }
  }
  wave_lds_sync();
  return L.fb[li];
}

// Recorded steps of one cell: step s (1-based) is the row p + (s - first) *
// stride (the whole record, first = 1; or a recomputed segment).
struct RecView {
  const double *p;
  int first, stride;
  __device__ const double *row(int s) const { return p + static_cast<int64_t>(s - first) * stride; }
};

// xi_i and l_j of recorded step `step` (1-based); hist from the records.
__device__ __forceinline__ void rec_coeffs(const RecView &rv, int n, double hpad, int step, int q,
                                           double (&xi)[kQmax + 2], double (&l)[kQmax + 2],
                                           double &Cerr) {
  const double hn = rv.row(step)[n];
  double sum = hn;
  xi[0] = 0.0;
  xi[1] = 1.0;
#pragma unroll
  for (int i = 2; i <= kQmax + 1; ++i) {
    const int idx = step - i + 1;  // 1-based step of h_{n-i+1}
    sum += idx >= 1 ? rv.row(idx)[n] : hpad;
    xi[i] = i <= q + 1 ? sum / hn : 0.0;
  }
  bdf_coeffs(q, xi, l, Cerr);
}

// Sweeps steps hi down to lo (1 <= lo, hi <= the cell's step count) of one
// cell through the rows rv.  init: the sweep starts at the cell's last step
// from dL/dy(t_out); else from the state an earlier call parked (P.adj: the
// lane vectors zbar_0 .. zbar_kQmax and the order-raise term; P.pbar: the
// dL/dlnA sums).  lo == 1 finishes the cell (dL/dy0 and dL/dlnA written),
// else the state is parked for the call that sweeps the steps before lo.  The
// sums run in step order either way, so a sweep in pieces equals one sweep
// over all steps bit for bit.
template <int S>
__device__ __forceinline__ void adjoint_steps(const Params &P, int64_t cell, int li, double *lds,
                                              const RecView &rv, int hi, int lo, bool init) {
  const MechDev &m = P.mech;
  const int R = m.R;
  const Lds L = carve<kTabLds>(lds, R, m.rx, nullptr);
  const Grp<1> W1(li);
  double *vb = reinterpret_cast<double *>(L.fac) + S * S;  // [64 + 8], vb[kEmptySlot] = 0
  double *pb = vb + kWave + 8;
  if (li == 0) {
    L.yb[kEmptySlot] = 1.0;
    vb[kEmptySlot] = 0.0;
  }
  const int n = P.n_sp;
  const bool own = li < n;
  const int stride = P.rec_stride;
  double *park = P.adj ? P.adj + cell * (kQmax + 2) * P.ckpt_vs : nullptr;

  const double T = P.T ? P.T[cell] : 1.0;
  wave_lds_sync();
  for (int r = li; r < R; r += kWave) {
    double lk = m.lnA[r];
    lk -= m.EaR[r] / T;
    double kf = exp(lk);
    if (P.kscale) kf *= P.kscale[cell * P.ldk + r];
    L.kk[2 * r] = kf;
    L.kk[2 * r + 1] = m.reversible ? -(kf * exp(-m.lnK[r])) : -0.0;
    const_cast<int2 *>(L.rx)[r] = reinterpret_cast<const int2 *>(m.rx)[r];
    pb[r] = init ? 0.0 : P.pbar[cell * P.ldp + r];
  }
  const double hpad = uni(P.rec_hpad[cell]);
  double zb[kQmax + 1];
  double ebx = 0.0;
  if (init) {
#pragma unroll
    for (int j = 0; j <= kQmax; ++j) zb[j] = 0.0;
    zb[0] = own ? P.ybar[cell * P.ldy + li] : 0.0;
  } else {
#pragma unroll
    for (int j = 0; j <= kQmax; ++j) zb[j] = own ? park[j * P.ckpt_vs + li] : 0.0;
    ebx = own ? park[(kQmax + 1) * P.ckpt_vs + li] : 0.0;
  }
  double y0bar = zb[0];

  for (int step = hi; step >= lo; --step) {
    const int qr = uni(static_cast<int>(rv.row(step)[n + 1]));
    const int q = qr & 255;
    const double hn = uni(rv.row(step)[n]);
    double xi[kQmax + 2], l[kQmax + 2], Cerr;
    rec_coeffs(rv, n, hpad, step, q, xi, l, Cerr);
    const double gamma = uni(hn / l[1]);
    const double yn = own ? rv.row(step)[li] : 0.0;
    // z_n = zp + l e, e = y_n - zp_0
    double eb = ebx;
#pragma unroll
    for (int j = 0; j <= kQmax; ++j)
      if (j <= q) eb = fma(l[j], zb[j], eb);
    zb[0] -= eb;
    // (I - gamma J(y_n))^T mu = eb
    {
      double a[S];
      newton_matrix<S, double>(a, m, L, W1, yn, gamma, true);
      gj_invert<S, double>(a, W1, L);
    }
    const double mu = own ? inv_solve<S, double, false>(L, W1, eb) : 0.0;
    adj_scatter(m, L, vb, pb, li, yn, mu, gamma, false);
    // a = zp_0 - zp_1 / l_1
    zb[0] += mu;
    zb[1] -= mu / l[1];
    // predictor transpose (reverse order of the Pascal updates)
#pragma unroll
    for (int k = kQmax; k >= 1; --k)
#pragma unroll
      for (int j = k; j <= kQmax; ++j)
        if (k <= q && j <= q) zb[j] += zb[j - 1];
    ebx = 0.0;
    if (step == 1) {
      // z = [y0, h_1 f(y0)]
      const double y0 = own ? P.rec_y0[cell * stride + li] : 0.0;
      const double jtv = adj_scatter(m, L, vb, pb, li, y0, zb[1], hn, true);
      y0bar = zb[0] + hn * jtv;
      break;
    }
    const int qp = uni(static_cast<int>(rv.row(step - 1)[n + 1])) & 255;
    if (qr >> 8) {
      // z was rebuilt as [y_{n-1}, h_n f(y_{n-1})] before this step
      const double yp = own ? rv.row(step - 1)[li] : 0.0;
      const double jtv = adj_scatter(m, L, vb, pb, li, yp, zb[1], hn, true);
      zb[0] += hn * jtv;
#pragma unroll
      for (int j = 1; j <= kQmax; ++j) zb[j] = 0.0;
    } else {
      const double eta = uni(hn / rv.row(step - 1)[n]);
      double fct = 1.0;
#pragma unroll
      for (int j = 1; j <= kQmax; ++j) {
        fct *= eta;
        if (j <= q) zb[j] *= fct;
      }
      if (q == qp + 1 || q == qp - 1) {
        double xip[kQmax + 2], lp[kQmax + 2], Cp;
        rec_coeffs(rv, n, hpad, step - 1, qp, xip, lp, Cp);
        if (q == qp + 1) {
          const double c = 1.0 / pick(xip, qp + 1);
#pragma unroll
          for (int j = 1; j <= kQmax; ++j)
            if (j <= qp + 1) ebx += c * lp[j - 1] * zb[j];
#pragma unroll
          for (int j = 1; j <= kQmax; ++j)
            if (j == qp + 1) zb[j] = 0.0;
        } else {
          double c[kQmax + 2];
#pragma unroll
          for (int j = 0; j <= kQmax + 1; ++j) c[j] = 0.0;
          c[1] = 1.0;
#pragma unroll
          for (int i = 1; i <= kQmax - 1; ++i)
            if (i <= qp - 1) {
#pragma unroll
              for (int j = i + 1; j >= 1; --j) c[j] = c[j - 1] + xip[i] * c[j];
            }
          double acc = 0.0;
#pragma unroll
          for (int j = 1; j <= kQmax; ++j)
            if (j < qp) acc -= c[j] * zb[j];
#pragma unroll
          for (int j = 1; j <= kQmax; ++j)
            if (j == qp) zb[j] = acc;
        }
      }
    }
  }
  if (lo == 1) {
    if (own) P.y0bar[cell * P.ldy + li] = y0bar;
  } else if (own) {
#pragma unroll
    for (int j = 0; j <= kQmax; ++j) park[j * P.ckpt_vs + li] = zb[j];
    park[(kQmax + 1) * P.ckpt_vs + li] = ebx;
  }
  wave_lds_sync();
  for (int r = li; r < R; r += kWave) P.pbar[cell * P.ldp + r] = pb[r];
}

// Checkpointed records: the segments of a cell (steps cK + 1 .. (c + 1)K,
// K = P.ckpt_every, the last one cut at the cell's step count) are swept from
// the last in passes; pass j takes segment nseg - 1 - j of every cell that
// has more than j segments.  A cell without steps has one empty segment.
__device__ __forceinline__ int adj_segments(const Params &P, int64_t cell) {
  const int N = uni(P.rec_n[cell]);
  return N > 0 ? (N + P.ckpt_every - 1) / P.ckpt_every : 1;
}

// The rows of one cell's segment (P.seg_rows rows of P.rec_stride from
// P.seg): rows 0 .. kQmax hold steps n0 - kQmax .. n0 (their step sizes; step
// n0 also its state and order, from the checkpoint), the rest steps n0 + 1 ..
__device__ __forceinline__ RecView adj_rows(const Params &P, int64_t cell, int n0) {
  return RecView{P.seg + cell * P.seg_rows * P.rec_stride, n0 - kQmax, P.rec_stride};
}

// Pass j, first half: rerun the cell's segment from its checkpoint with the
// forward step code (the same steps, bit for bit) into its rows.
template <int S, bool ABC>
__device__ __forceinline__ void rerun_segment(const Params &P, int64_t cell, const Grp<1> &W,
                                              double *lds, int j) {
  const int nseg = adj_segments(P, cell);
  const int N = uni(P.rec_n[cell]);
  if (j >= nseg || N == 0) return;
  const int K = P.ckpt_every, c = nseg - 1 - j, n0 = c * K;
  const double *ck = P.ckpt + (cell * P.ckpt_cap + c) * Ckpt::stride(P.ckpt_vs);
  double *rows = P.seg + cell * P.seg_rows * P.rec_stride;
  const int n = P.n_sp, stride = P.rec_stride;
  if (W.lane == 0) {
#pragma unroll
    for (int k = 0; k <= kQmax; ++k) rows[k * stride + n] = ck[Ckpt::kHist + kQmax - k];
    rows[kQmax * stride + n + 1] = ck[Ckpt::kQtaken];
  }
  if (W.lane < n) rows[kQmax * stride + W.lane] = ck[Ckpt::vec(0, S) + W.lane];
  const Resume rs{ck, rows, n0 - kQmax, n0 + K < N ? n0 + K : N, P.seg_rows};
  integrate_cell<S, double, kTabLds, 1, ABC, false, kLinAnalytic, false, true>(
      P, cell, W, lds, nullptr, BatchRed<false>{}, 1, &rs);
}

// Pass j, second half: sweep the rerun segment.
template <int S>
__device__ __forceinline__ void sweep_segment(const Params &P, int64_t cell, int li, double *lds,
                                              int j) {
  const int nseg = adj_segments(P, cell);
  if (j >= nseg) return;
  const int N = uni(P.rec_n[cell]);
  const int K = P.ckpt_every, c = nseg - 1 - j, n0 = c * K;
  adjoint_steps<S>(P, cell, li, lds, adj_rows(P, cell, n0), n0 + K < N ? n0 + K : N, n0 + 1, j == 0);
}

__host__ __device__ constexpr int lds_doubles_adjoint(int S, int R) {
  return lds_doubles(S, R, 8) + kWave + 8 + R;
}

}  // namespace bdfx
