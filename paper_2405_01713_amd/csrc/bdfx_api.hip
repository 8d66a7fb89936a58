// bdfx_api.hip -- host runtime behind the C ABI of include/bdfx.h.
//
// Owns the context (device, stream, plan, bound buffers) and the
// device-resident mechanism tables; builds the reaction slot words and the
// lane-major analytic-Jacobian term tables from the stoichiometry; launches
// the per-size integrator kernels (one wavefront per cell).  Nothing here allocates device memory after
// bdfx_bind() (the paper's memory-pool lesson, Sec. 4.3.1), so integrate and
// perturb can be captured into a HIP graph by the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "bdfx.h"
#include "bdf_kernels.h"

BDFX_DECLARE_SIZE(3)
BDFX_DECLARE_SIZE(4)
BDFX_DECLARE_SIZE(8)
BDFX_DECLARE_SIZE(9)
BDFX_DECLARE_SIZE(16)
BDFX_DECLARE_SIZE(21)
BDFX_DECLARE_SIZE(32)
BDFX_DECLARE_SIZE(53)
BDFX_DECLARE_SIZE(64)
BDFX_DECLARE_PAIR(53, 9)

hipError_t bdfx_launch_perturb(const bdfx::Params &P, uint64_t seed, int64_t step, double amp,
                               hipStream_t s);
hipError_t bdfx_launch_fill_u32(uint32_t *p, int n, uint32_t v, hipStream_t s);
hipError_t bdfx_launch_copy_rows(double *y, int ldy, const int32_t *list, int64_t n, int S,
                                 double *dst, bool restore, hipStream_t s);
hipError_t bdfx_launch_sum_cells(const double *pbar, int ldp, const int32_t *list, int64_t n, int R,
                                 double *out, hipStream_t s);
int bdfx_extremes_blocks(int64_t n, int S, int max_blocks);
hipError_t bdfx_launch_extremes(const double *y, int ldy, const int32_t *list, int64_t n, int S,
                                int blocks, double *part, hipStream_t s);
hipError_t bdfx_launch_typical(int n_mech, int ldt, const int32_t *S, const int32_t *nblk,
                               const int64_t *part_off, const double *part, double eta, double *atol,
                               double *typ, hipStream_t s);

static_assert(sizeof(bdfx_cell_stats) == sizeof(bdfx::CellStats), "stats layout");
static_assert(sizeof(bdfx_cell_stats) == 56, "stats size");

namespace {

thread_local std::string g_create_error;

struct SizeEntry {
  int S;
  hipError_t (*launch)(const bdfx::Params &, bool, int, int, int, int, const bdfx::LaunchCfg &,
                       hipStream_t);
  hipError_t (*occupancy)(bool, int, int, int, int, int, size_t, int *);
  // adjoint kernels (kind 0: full-record sweep; 1, 2: rerun and sweep of a
  // checkpointed pass)
  hipError_t (*adjoint)(const bdfx::Params &, int, int, bool, const bdfx::LaunchCfg &, hipStream_t);

};

#define BDFX_SIZE_ENTRY(S) \
  {S, bdfx_launch_s##S, bdfx_occupancy_s##S, bdfx_adjoint_s##S}
const SizeEntry kSizes[] = {
    BDFX_SIZE_ENTRY(3),  BDFX_SIZE_ENTRY(4),  BDFX_SIZE_ENTRY(8),
    BDFX_SIZE_ENTRY(9),  BDFX_SIZE_ENTRY(16), BDFX_SIZE_ENTRY(21),
    BDFX_SIZE_ENTRY(32), BDFX_SIZE_ENTRY(53), BDFX_SIZE_ENTRY(64),
};
#undef BDFX_SIZE_ENTRY

// Smallest compiled size that holds S species (exact sizes 3, 9, 21, 53 are
// compiled for the benchmark mechanisms; others are padded with inert
// species whose Newton-matrix rows are identity rows).
const SizeEntry *size_for(int S) {
  for (const auto &e : kSizes)
    if (e.S >= S) return &e;
  return nullptr;
}

// Compiled pairs of padded sizes for the one-launch form of two-mechanism
// batches (k_integrate_pair): larger size first.
struct PairEntry {
  int SA, SB;
  hipError_t (*launch)(const bdfx::Params &, const bdfx::Params &, bool, int, int,
                       const bdfx::LaunchCfg &, hipStream_t);
  hipError_t (*occupancy)(bool, int, int, int, size_t, int *);
};

const PairEntry kPairs[] = {
    {53, 9, bdfx_launch_pair_s53_s9, bdfx_occupancy_pair_s53_s9},
};

const PairEntry *pair_for(int SA, int SB) {
  for (const auto &e : kPairs)
    if (e.SA == SA && e.SB == SB) return &e;
  return nullptr;
}

}  // namespace

// largest per-bin sample the autotuner times (rows saved in the workspace)
constexpr int64_t kTuneCells = 16384;
// most waves one CU can hold (8 per SIMD): bounds the rate-constant slots of
// persistent grids
constexpr int64_t kMaxWavesPerCu = 32;
// blocks of the typical-value extremes pass per mechanism (partials in the workspace)
constexpr int kExtMaxBlocks = 256;

struct bdfx_mech_s {
  bdfx_ctx ctx = nullptr;
  int S = 0, R = 0;
  int n = 0;             // state entries per cell: S, plus the temperature if non-isothermal
  bool reversible = false;
  bool abc = false;      // every reaction A + B <=> C (specialised kernels)
  bool thermal = false;  // temperature as a state (heat capacities given)
  void *dmem = nullptr;
  bdfx::MechDev dev{};
  std::vector<double> w;
};

struct Bin {
  int mech;
  int64_t offset, count;
  // launch of the integrator for this bin, fixed at bind time so that
  // bdfx_integrate() only enqueues kernels (it may be captured in a graph)
  const SizeEntry *se = nullptr;
  int32_t lds_doubles = 0;
  bdfx::LaunchCfg cfg{};
  // launch shape: from the options, or chosen by bdfx_autotune()
  int32_t waves_per_simd = 0, waves_per_block = 1, queue_chunk = 1, cells_per_wave = 1;
  bool tuned = false;
  int tab = bdfx::kTabLds;  // placement of the reaction tables (bdfx::kTab*)
  int64_t tune_sample = 0;  // bdfx_autotune(): cells timed and time of the pick
  float tune_ms = 0.0f;
};

struct bdfx_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int n_cu = 0;
  int lds_max_block = 65536;  // LDS one block may allocate on the device
  // plan
  bool planned = false, bound = false, integrated = false;
  int64_t N = 0;
  std::vector<bdfx_mech> mechs;
  bdfx_options opt{};
  std::vector<double> atol;
  double *d_atol = nullptr;
  int S_max = 0, R_max = 0;
  size_t ws_need = 0;
  size_t off_queue = 0, off_bins = 0, off_rec = 0, off_recn = 0, off_rechpad = 0, off_recy0 = 0,
         off_pbar = 0, off_tune = 0, off_kk = 0, off_ext = 0, off_tatol = 0, off_ckpt = 0,
         off_ckpt_setup = 0, off_seg = 0, off_adj = 0;
  int32_t ckpt_cap = 0;    // checkpoints per cell (checkpoint_every > 0)
  int32_t ckpt_vs = 0;     // largest padded size: checkpoint vectors hold at most this many
  bool typical = false;  // per-mechanism typical-value atol in effect (bdfx_typical_atol)
  int64_t tune_cells = 0;  // rows the autotuner can save in the workspace
  int64_t kk_slots = 0;    // rate-constant slots (waves) for tables in global memory
  int rec_stride = 0;
  // bind
  char *ws = nullptr;
  double *y = nullptr;
  int ldy = 0, ldk = 0;
  const int32_t *cell_mech = nullptr;
  const double *T = nullptr, *kscale = nullptr, *F = nullptr;
  int32_t *status = nullptr;
  bdfx_cell_stats *stats = nullptr;
  std::vector<Bin> bins;
  // BDFX_SCHED_FUSED: both bins in one launch (nullptr: one launch per bin)
  const PairEntry *pair = nullptr;
  int pair_a = 0, pair_b = 1;    // bin indices of the larger and the smaller mechanism
  int pair_waves = 1;            // A-waves per block (the rest of the block's waves are B-waves)
  int32_t pair_lds_b = 0;        // LDS doubles of a bin-B wave (tables in LDS)
  bool pair_off = false;         // bdfx_autotune timed the one launch slower than two
  bdfx::LaunchCfg pair_cfg{};
  double last_t0 = 0.0, last_tout = 0.0;
};

static int fail(bdfx_ctx c, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c)
    c->err = buf;
  else
    g_create_error = buf;
  return code;
}

#define HIPCHK(c, expr)                                                                          \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) return fail(c, BDFX_EHIP, "%s: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

extern "C" {

const char *bdfx_version(void) { return "bdfx 0.1 (gfx950)"; }

const char *bdfx_last_error(bdfx_ctx ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

int bdfx_create(bdfx_ctx *out, int device, void *hip_stream) {
  if (!out) return fail(nullptr, BDFX_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(nullptr, BDFX_EHIP, "no HIP device available");
  if (device < 0 || device >= ndev) return fail(nullptr, BDFX_EINVAL, "bad device %d", device);
  auto *c = new bdfx_ctx_s();
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipSetDevice(device) != hipSuccess ||
      hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      hipDeviceGetAttribute(&c->lds_max_block, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
          hipSuccess) {
    delete c;
    return fail(nullptr, BDFX_EHIP, "cannot query device %d", device);
  }
  *out = c;
  return BDFX_OK;
}

int bdfx_set_stream(bdfx_ctx ctx, void *hip_stream) {
  if (!ctx) return BDFX_EINVAL;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return BDFX_OK;
}

int bdfx_destroy(bdfx_ctx ctx) {
  if (!ctx) return BDFX_EINVAL;
  hipSetDevice(ctx->device);
  if (ctx->d_atol) hipFree(ctx->d_atol);
  delete ctx;
  return BDFX_OK;
}

// ---------------------------------------------------------------------------
// mechanisms
// ---------------------------------------------------------------------------

int bdfx_mech_create(bdfx_ctx ctx, const bdfx_mech_desc *d, bdfx_mech *out) {
  if (!ctx || !d || !out) return fail(ctx, BDFX_EINVAL, "NULL argument");
  *out = nullptr;
  const int S = d->n_species, R = d->n_reactions;
  if (S < 1 || S > BDFX_MAX_SPECIES) return fail(ctx, BDFX_EINVAL, "n_species %d out of 1..64", S);
  if (R < 1 || R > (1 << 15)) return fail(ctx, BDFX_EINVAL, "n_reactions %d out of range", R);
  if (!d->reac || !d->prod || !d->lnA) return fail(ctx, BDFX_EINVAL, "reac/prod/lnA required");
  const bool thermal = d->cv != nullptr;
  if (thermal != (d->u0 != nullptr)) return fail(ctx, BDFX_EINVAL, "cv and u0 go together");
  if (thermal && S + 1 > BDFX_MAX_SPECIES)
    return fail(ctx, BDFX_EINVAL, "non-isothermal: n_species + 1 must be <= 64");
  if (thermal)
    for (int i = 0; i < S; ++i)
      if (!(d->cv[i] > 0.0) || !std::isfinite(d->cv[i]) || !std::isfinite(d->u0[i]))
        return fail(ctx, BDFX_EINVAL, "species %d: cv must be positive, u0 finite", i);
  for (int r = 0; r < R; ++r)
    for (int l = 0; l < BDFX_SLOTS; ++l) {
      const int a = d->reac[r * 3 + l], b = d->prod[r * 3 + l];
      if (a < -1 || a >= S || b < -1 || b >= S)
        return fail(ctx, BDFX_EINVAL, "reaction %d slot %d: species out of range", r, l);
    }

  // reaction slots, one byte per species (bdfx::kEmptySlot = empty)
  std::vector<int32_t> rx(2 * R);
  for (int r = 0; r < R; ++r) {
    uint32_t wr = 0, wp = 0;
    for (int l = 0; l < 3; ++l) {
      const int a = d->reac[r * 3 + l], b = d->prod[r * 3 + l];
      wr |= static_cast<uint32_t>(a < 0 ? bdfx::kEmptySlot : a) << (8 * l);
      wp |= static_cast<uint32_t>(b < 0 ? bdfx::kEmptySlot : b) << (8 * l);
    }
    rx[2 * r] = static_cast<int32_t>(wr);
    rx[2 * r + 1] = static_cast<int32_t>(wp);
  }
  const bool reversible = d->lnK != nullptr;
  bool abc = true;
  for (int r = 0; r < R && abc; ++r)
    abc = d->reac[r * 3] >= 0 && d->reac[r * 3 + 1] >= 0 && d->reac[r * 3 + 2] < 0 &&
          d->prod[r * 3] >= 0 && d->prod[r * 3 + 1] < 0 && d->prod[r * 3 + 2] < 0;

  std::vector<double> lnA(d->lnA, d->lnA + R), EaR(R, 0.0), lnK(R, 0.0), w(S, 1.0);
  if (d->EaR) EaR.assign(d->EaR, d->EaR + R);
  if (d->lnK) lnK.assign(d->lnK, d->lnK + R);

  // one device allocation for all tables
  size_t off = 0;
  auto reserve = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 8), 256);
    return o;
  };
  const size_t o_rx = reserve(rx.size() * 4), o_lnA = reserve(R * 8), o_EaR = reserve(R * 8),
               o_lnK = reserve(R * 8), o_w = reserve(S * 8), o_cv = reserve(thermal ? S * 8 : 0),
               o_u0 = reserve(thermal ? S * 8 : 0);
  HIPCHK(ctx, hipSetDevice(ctx->device));
  void *dmem = nullptr;
  HIPCHK(ctx, hipMalloc(&dmem, off));
  char *base = static_cast<char *>(dmem);
  auto up = [&](size_t o, const void *src, size_t bytes) {
    return bytes ? hipMemcpy(base + o, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = up(o_rx, rx.data(), rx.size() * 4);
  if (e == hipSuccess) e = up(o_lnA, lnA.data(), R * 8);
  if (e == hipSuccess) e = up(o_EaR, EaR.data(), R * 8);
  if (e == hipSuccess) e = up(o_lnK, lnK.data(), R * 8);
  if (e == hipSuccess) e = up(o_w, w.data(), S * 8);
  if (e == hipSuccess && thermal) e = up(o_cv, d->cv, S * 8);
  if (e == hipSuccess && thermal) e = up(o_u0, d->u0, S * 8);
  if (e != hipSuccess) {
    hipFree(dmem);
    return fail(ctx, BDFX_EHIP, "mechanism upload: %s", hipGetErrorString(e));
  }
  auto *m = new bdfx_mech_s();
  m->ctx = ctx;
  m->S = S;
  m->R = R;
  m->n = S + (thermal ? 1 : 0);
  m->reversible = reversible;
  m->abc = abc;
  m->thermal = thermal;
  m->dmem = dmem;
  m->w = w;
  bdfx::MechDev &dv = m->dev;
  dv.S = S;
  dv.R = R;
  dv.reversible = reversible ? 1 : 0;
  dv.rx = reinterpret_cast<const int32_t *>(base + o_rx);
  dv.lnA = reinterpret_cast<const double *>(base + o_lnA);
  dv.EaR = reinterpret_cast<const double *>(base + o_EaR);
  dv.lnK = reinterpret_cast<const double *>(base + o_lnK);
  dv.w = reinterpret_cast<const double *>(base + o_w);
  dv.cv = thermal ? reinterpret_cast<const double *>(base + o_cv) : nullptr;
  dv.u0 = thermal ? reinterpret_cast<const double *>(base + o_u0) : nullptr;
  *out = m;
  return BDFX_OK;
}

int bdfx_mech_set_weights(bdfx_mech m, const double *weights) {
  if (!m || !weights) return BDFX_EINVAL;
  m->w.assign(weights, weights + m->S);
  bdfx_ctx c = m->ctx;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipMemcpy(const_cast<double *>(m->dev.w), weights, m->S * 8, hipMemcpyHostToDevice));
  return BDFX_OK;
}

int bdfx_mech_set_lnA(bdfx_mech m, const double *d_lnA) {
  if (!m || !d_lnA) return BDFX_EINVAL;
  bdfx_ctx c = m->ctx;
  if (!c) return BDFX_EINVAL;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipMemcpyAsync(const_cast<double *>(m->dev.lnA), d_lnA, static_cast<size_t>(m->R) * 8,
                           hipMemcpyDeviceToDevice, c->stream));
  return BDFX_OK;
}

int bdfx_mech_destroy(bdfx_mech m) {
  if (!m) return BDFX_EINVAL;
  if (m->ctx) hipSetDevice(m->ctx->device);
  if (m->dmem) hipFree(m->dmem);
  delete m;
  return BDFX_OK;
}

// ---------------------------------------------------------------------------
// plan / bind
// ---------------------------------------------------------------------------

int bdfx_plan(bdfx_ctx ctx, int64_t n_cells, int32_t n_mech, const bdfx_mech *mechs,
              const bdfx_options *o, size_t *ws_bytes) {
  if (!ctx || !mechs || !o || !ws_bytes) return fail(ctx, BDFX_EINVAL, "NULL argument");
  if (n_cells < 0 || n_cells > (int64_t{1} << 31) - 1)
    return fail(ctx, BDFX_EINVAL, "n_cells %lld out of range", static_cast<long long>(n_cells));
  if (n_mech < 1 || n_mech > BDFX_MAX_MECH) return fail(ctx, BDFX_EINVAL, "n_mech out of range");
  if (!(o->rtol > 0.0)) return fail(ctx, BDFX_EINVAL, "rtol must be > 0");
  if (!o->atol || o->atol_len < 1) return fail(ctx, BDFX_EINVAL, "atol required");
  if (o->lu_precision != 0 && o->lu_precision != 64 && o->lu_precision != 32)
    return fail(ctx, BDFX_EINVAL, "lu_precision must be 64 or 32");
  if (o->scheduler != BDFX_SCHED_STATIC && o->scheduler != BDFX_SCHED_QUEUE &&
      o->scheduler != BDFX_SCHED_FUSED)
    return fail(ctx, BDFX_EINVAL, "unknown scheduler %d", o->scheduler);
  if (o->waves_per_simd != 0 && (o->waves_per_simd < 3 || o->waves_per_simd > 5))
    return fail(ctx, BDFX_EINVAL, "waves_per_simd must be 0, 3, 4 or 5");
  if (o->waves_per_block < 0 || o->waves_per_block > 16 || o->blocks_per_cu < 0 ||
      o->queue_chunk < 0 || o->cells_per_wave < 0 || o->cells_per_wave > 2)
    return fail(ctx, BDFX_EINVAL, "invalid launch shape");
  if (o->max_order < 0 || o->max_order > BDFX_MAX_ORDER)
    return fail(ctx, BDFX_EINVAL, "max_order out of 1..5");
  if (o->record_steps < 0) return fail(ctx, BDFX_EINVAL, "record_steps < 0");
  if (o->jacobian != BDFX_JAC_ANALYTIC && o->jacobian != BDFX_JAC_DQ)
    return fail(ctx, BDFX_EINVAL, "jacobian must be BDFX_JAC_ANALYTIC or BDFX_JAC_DQ");
  if (o->gmres_maxl < 0 || o->gmres_maxl > BDFX_GMRES_MAXL)
    return fail(ctx, BDFX_EINVAL, "gmres_maxl must be 0..%d", BDFX_GMRES_MAXL);
  if (o->gmres_maxl > 0 && o->jacobian != BDFX_JAC_ANALYTIC)
    return fail(ctx, BDFX_EINVAL, "jacobian selects the Newton matrix of the direct solver; "
                                  "GMRES forms none (use BDFX_JAC_ANALYTIC)");
  if (o->gmres_maxl > 0 && o->record_steps > 0)
    return fail(ctx, BDFX_EUNSUPPORTED, "step recording (adjoint) needs the direct solver");
  if (o->checkpoint_every < 0) return fail(ctx, BDFX_EINVAL, "checkpoint_every < 0");
  if (o->checkpoint_every > 0 && o->record_steps <= 0)
    return fail(ctx, BDFX_EINVAL, "checkpoint_every needs record_steps > 0");
  if (o->checkpoint_every > 0 && (o->lu_precision == 32 || o->jacobian != BDFX_JAC_ANALYTIC))
    return fail(ctx, BDFX_EUNSUPPORTED,
                "checkpointed records: FP64 Newton matrix from the analytic Jacobian");
  if (o->lockstep < 0 || o->lockstep > BDFX_MAX_LOCKSTEP)
    return fail(ctx, BDFX_EINVAL, "lockstep must be 0..%d", BDFX_MAX_LOCKSTEP);
  if (o->lockstep > 0 &&
      (o->jacobian != BDFX_JAC_ANALYTIC || o->gmres_maxl > 0 || o->record_steps > 0))
    return fail(ctx, BDFX_EUNSUPPORTED,
                "lock-step batches: direct solver, analytic Jacobian, no step recording");
  int S_max = 0, R_max = 0;
  for (int m = 0; m < n_mech; ++m) {
    if (!mechs[m] || mechs[m]->ctx != ctx) return fail(ctx, BDFX_EINVAL, "bad mechanism %d", m);
    S_max = std::max(S_max, mechs[m]->n);
    if (mechs[m]->thermal && o->record_steps > 0)
      return fail(ctx, BDFX_EUNSUPPORTED, "step recording (adjoint) needs isothermal mechanisms");
    if (mechs[m]->thermal && o->lockstep > 0)
      return fail(ctx, BDFX_EUNSUPPORTED, "lock-step batches need isothermal mechanisms");
    R_max = std::max(R_max, mechs[m]->R);
  }
  if (o->atol_len != 1 && o->atol_len < S_max)
    return fail(ctx, BDFX_EINVAL, "atol_len must be 1 or >= %d", S_max);
  for (int i = 0; i < o->atol_len; ++i)
    if (!(o->atol[i] > 0.0) || !std::isfinite(o->atol[i]))
      return fail(ctx, BDFX_EINVAL, "atol[%d] must be positive", i);

  ctx->planned = ctx->bound = ctx->integrated = false;
  ctx->N = n_cells;
  ctx->mechs.assign(mechs, mechs + n_mech);
  ctx->opt = *o;
  if (ctx->opt.max_order == 0) ctx->opt.max_order = 5;
  if (ctx->opt.max_steps <= 0) ctx->opt.max_steps = 5000;
  if (ctx->opt.max_err_test_fails <= 0) ctx->opt.max_err_test_fails = 7;
  if (ctx->opt.max_conv_fails <= 0) ctx->opt.max_conv_fails = 10;
  if (ctx->opt.lu_precision == 0) ctx->opt.lu_precision = 64;
  if (ctx->opt.queue_chunk <= 0) ctx->opt.queue_chunk = 1;
  ctx->atol.assign(o->atol, o->atol + o->atol_len);
  ctx->opt.atol = nullptr;
  ctx->S_max = S_max;
  ctx->R_max = R_max;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (ctx->d_atol) {
    hipFree(ctx->d_atol);
    ctx->d_atol = nullptr;
  }
  HIPCHK(ctx, hipMalloc(&ctx->d_atol, ctx->atol.size() * 8));
  HIPCHK(ctx, hipMemcpy(ctx->d_atol, ctx->atol.data(), ctx->atol.size() * 8,
                        hipMemcpyHostToDevice));

  // workspace layout
  size_t off = 0;
  auto reserve = [&](size_t bytes) {
    const size_t o2 = off;
    off = align_up(off + bytes, 256);
    return o2;
  };
  ctx->off_queue = reserve(64 * 4);
  ctx->off_bins = reserve(static_cast<size_t>(n_mech > 1 ? n_cells : 0) * 4);
  ctx->rec_stride = S_max + 2;
  const int64_t cap = o->record_steps;
  const int K = o->checkpoint_every;
  ctx->off_rec = reserve(K > 0 ? 0 : static_cast<size_t>(n_cells) * cap * ctx->rec_stride * 8);
  ctx->ckpt_cap = K > 0 ? static_cast<int32_t>((cap + K - 1) / K) : 0;
  ctx->ckpt_vs = 0;
  for (int m = 0; m < n_mech; ++m)
    if (const SizeEntry *se = size_for(mechs[m]->n)) ctx->ckpt_vs = std::max(ctx->ckpt_vs, se->S);
  ctx->off_ckpt = reserve(static_cast<size_t>(n_cells) * ctx->ckpt_cap *
                          bdfx::Ckpt::stride(ctx->ckpt_vs) * 8);
  ctx->off_ckpt_setup = reserve(K > 0 ? static_cast<size_t>(n_cells) * ctx->ckpt_vs * 8 : 0);
  // the checkpointed sweep: each cell's current segment rows and its parked
  // sweep state
  const size_t seg_rows = K > 0 ? static_cast<size_t>(K) + bdfx::kQmax + 1 : 0;
  ctx->off_seg = reserve(static_cast<size_t>(n_cells) * seg_rows * ctx->rec_stride * 8);
  ctx->off_adj = reserve(K > 0 ? static_cast<size_t>(n_cells) * (bdfx::kQmax + 2) * ctx->ckpt_vs * 8 : 0);
  ctx->off_recn = reserve(cap ? static_cast<size_t>(n_cells) * 4 : 0);
  ctx->off_rechpad = reserve(cap ? static_cast<size_t>(n_cells) * 8 : 0);
  ctx->off_recy0 = reserve(cap ? static_cast<size_t>(n_cells) * ctx->rec_stride * 8 : 0);
  ctx->off_pbar = reserve(cap ? static_cast<size_t>(n_cells) * R_max * 8 : 0);
  ctx->tune_cells = std::min<int64_t>(n_cells, kTuneCells);
  // (two bins' samples at once: the autotuner times the one-launch form too)
  ctx->off_tune = reserve(static_cast<size_t>(2) * ctx->tune_cells * S_max * 8);
  // persistent grids may keep each wave's rate constants in global memory
  ctx->kk_slots = o->scheduler != BDFX_SCHED_STATIC
                      ? std::min<int64_t>(static_cast<int64_t>(ctx->n_cu) * kMaxWavesPerCu, n_cells + 16)
                      : 0;
  ctx->off_kk = reserve(static_cast<size_t>(ctx->kk_slots) * 2 * R_max * 8);
  ctx->off_ext = reserve(static_cast<size_t>(n_mech) * kExtMaxBlocks * 2 * bdfx::kWave * 8);
  ctx->off_tatol = reserve(static_cast<size_t>(n_mech) * S_max * 8);
  ctx->typical = false;
  ctx->ws_need = off;
  *ws_bytes = off;
  ctx->planned = true;
  return BDFX_OK;
}

static int configure_bins(bdfx_ctx ctx);

// linear solver of the context's integrator kernels (bdfx::kLin*)
static int lin_of(bdfx_ctx ctx) {
  return ctx->opt.gmres_maxl > 0 ? bdfx::kLinGmres
         : ctx->opt.jacobian == BDFX_JAC_DQ ? bdfx::kLinDq
                                            : bdfx::kLinAnalytic;
}

// kernel selection flags of a mechanism under the context's options
static int kernel_flags(bdfx_ctx ctx, bdfx_mech m) {
  return (m->abc ? 1 : 0) | (m->thermal ? 2 : 0) | (ctx->opt.jacobian == BDFX_JAC_DQ ? 4 : 0) |
         (ctx->opt.gmres_maxl > 0 ? 8 : 0) | (ctx->opt.lockstep > 0 ? 16 : 0);
}

// whether a mechanism of this size can run two cells per wave under the
// context's options (isothermal, analytic Jacobian, direct solver)
static bool two_cells_per_wave_ok(bdfx_ctx ctx, bdfx_mech m, int S) {
  return S <= 32 && !m->thermal && ctx->opt.jacobian != BDFX_JAC_DQ && ctx->opt.gmres_maxl == 0 &&
         ctx->opt.lockstep == 0 && ctx->opt.scheduler != BDFX_SCHED_FUSED &&
         ctx->opt.checkpoint_every == 0;
}

int bdfx_bind(bdfx_ctx ctx, void *d_ws, size_t ws_bytes, double *d_y, int32_t ldy,
              const int32_t *d_cell_mech, const double *d_T, const double *d_kscale, int32_t ldk,
              const double *d_forcing, int32_t *d_status, bdfx_cell_stats *d_stats) {
  if (!ctx) return BDFX_EINVAL;
  if (!ctx->planned) return fail(ctx, BDFX_EORDER, "bdfx_plan must precede bdfx_bind");
  if (ws_bytes < ctx->ws_need)
    return fail(ctx, BDFX_EWORKSPACE, "workspace %zu < %zu bytes", ws_bytes, ctx->ws_need);
  if (ctx->ws_need && !d_ws) return fail(ctx, BDFX_EINVAL, "workspace NULL");
  if (ctx->N > 0 && (!d_y || !d_status)) return fail(ctx, BDFX_EINVAL, "y and status required");
  if (ldy < ctx->S_max) return fail(ctx, BDFX_EINVAL, "ldy %d < S_max %d", ldy, ctx->S_max);
  if (d_kscale && ldk < ctx->R_max) return fail(ctx, BDFX_EINVAL, "ldk %d < R_max", ldk);
  if (ctx->mechs.size() > 1 && !d_cell_mech && ctx->N > 0)
    return fail(ctx, BDFX_EINVAL, "cell_mech required with several mechanisms");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  ctx->ws = static_cast<char *>(d_ws);
  ctx->y = d_y;
  ctx->ldy = ldy;
  ctx->ldk = ldk;
  ctx->cell_mech = d_cell_mech;
  ctx->T = d_T;
  ctx->kscale = d_kscale;
  ctx->F = d_forcing;
  ctx->status = d_status;
  ctx->stats = d_stats;
  ctx->bins.clear();
  ctx->pair_off = false;
  const int nm = static_cast<int>(ctx->mechs.size());
  if (nm == 1) {
    ctx->bins.push_back({0, 0, ctx->N});
  } else {
    // per-mechanism cell lists (counting sort, stable), built once here
    std::vector<int32_t> cm(ctx->N);
    HIPCHK(ctx, hipMemcpy(cm.data(), d_cell_mech, ctx->N * 4, hipMemcpyDeviceToHost));
    std::vector<int64_t> cnt(nm + 1, 0);
    for (int64_t c = 0; c < ctx->N; ++c) {
      if (cm[c] < 0 || cm[c] >= nm)
        return fail(ctx, BDFX_EINVAL, "cell_mech[%lld] = %d out of range",
                    static_cast<long long>(c), cm[c]);
      cnt[cm[c] + 1]++;
    }
    for (int m = 0; m < nm; ++m) cnt[m + 1] += cnt[m];
    std::vector<int32_t> list(ctx->N);
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t c = 0; c < ctx->N; ++c) list[pos[cm[c]]++] = static_cast<int32_t>(c);
    HIPCHK(ctx, hipMemcpy(ctx->ws + ctx->off_bins, list.data(), ctx->N * 4,
                          hipMemcpyHostToDevice));
    // expensive (larger) mechanisms first
    std::vector<int> order(nm);
    for (int m = 0; m < nm; ++m) order[m] = m;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return ctx->mechs[a]->n > ctx->mechs[b]->n; });
    for (int m : order) ctx->bins.push_back({m, cnt[m], cnt[m + 1] - cnt[m]});
  }
  if (const int rc = configure_bins(ctx)) return rc;
  ctx->bound = true;
  ctx->integrated = false;
  return BDFX_OK;
}

// ---------------------------------------------------------------------------
// integrate
// ---------------------------------------------------------------------------

// Kernel, LDS size and grid of one bin from its launch shape.
static int configure_bin(bdfx_ctx ctx, Bin &b) {
  const bool fp32 = ctx->opt.lu_precision == 32;
  const bool queue = ctx->opt.scheduler != BDFX_SCHED_STATIC;
  const bdfx_mech m = ctx->mechs[b.mech];
  b.se = size_for(m->n);
  if (!b.se) return fail(ctx, BDFX_EUNSUPPORTED, "no kernel for %d state entries", m->n);
  const int cpw = b.cells_per_wave;
  if (cpw != 1 && !(cpw == 2 && two_cells_per_wave_ok(ctx, m, b.se->S)))
    return fail(ctx, BDFX_EUNSUPPORTED, "%d cells per wave with %d state entries%s", cpw, b.se->S,
                m->thermal ? " (non-isothermal)" : "");
  // lock-step: one block per batch, one wave per cell of it, tables in LDS,
  // and the batch's reduction slots after the waves' areas
  const int lock = ctx->opt.lockstep;
  if (lock > 0) {  // the one shape of the lock-step kernels, as reported by bdfx_get_tuning
    b.waves_per_block = lock;
    b.waves_per_simd = 0;
    b.queue_chunk = 1;
  }
  const int waves = lock > 0 ? lock : std::max(b.waves_per_block, 1);
  const size_t lock_bytes = lock > 0 ? (2 * bdfx::kMaxBatch + 2) * 8 : 0;
  b.cfg.block = bdfx::kWave * waves;
  const int64_t per_block = static_cast<int64_t>(waves) * cpw;
  const int64_t need = (b.count + per_block - 1) / per_block;
  // Tables in LDS unless leaving some in global memory lets more waves reside
  // (LDS-limited sizes): first the slot words, then also the rate constants
  // (persistent grids only, whose waves each own a slot).  Ties keep the
  // tables in LDS.
  int occ[3] = {0, 0, 0};
  size_t lds[3];
  int64_t grid[3] = {0, 0, 0};
  const int tail = bdfx::inv_tail(b.se->S, fp32 ? 4 : 8, m->thermal, lin_of(ctx), lock > 0, cpw);
  for (int k : {bdfx::kTabLds, bdfx::kTabRxGlobal, bdfx::kTabGlobal}) {
    const int32_t d = static_cast<int32_t>(
        align_up(bdfx::lds_doubles(b.se->S, m->R, fp32 ? 4 : 8, k, m->thermal,
                                   ctx->opt.gmres_maxl, tail),
                 2));
    lds[k] = static_cast<size_t>(waves) * cpw * d * 8 + lock_bytes;
    if (lds[k] > 65536 || (k != bdfx::kTabLds && cpw != 1) || (k == bdfx::kTabGlobal && !queue) ||
        (k != bdfx::kTabLds && lock > 0))
      continue;
    HIPCHK(ctx, b.se->occupancy(fp32, b.waves_per_simd, k, cpw, kernel_flags(ctx, m), b.cfg.block,
                                lds[k], &occ[k]));
    if (queue) {
      const int per_cu = ctx->opt.blocks_per_cu > 0 ? ctx->opt.blocks_per_cu : std::max(occ[k], 1);
      grid[k] = std::min<int64_t>(static_cast<int64_t>(per_cu) * ctx->n_cu, need);
    }
    if (k == bdfx::kTabGlobal && grid[k] * waves > ctx->kk_slots) occ[k] = 0;
  }
  int k = bdfx::kTabLds;
  if (occ[bdfx::kTabRxGlobal] > occ[k]) k = bdfx::kTabRxGlobal;
  if (occ[bdfx::kTabGlobal] > occ[k]) k = bdfx::kTabGlobal;
  b.tab = k;
  b.cfg.lds_bytes = lds[k];
  b.lds_doubles = static_cast<int32_t>((lds[k] - lock_bytes) / 8 / (waves * cpw));
  if (b.cfg.lds_bytes > 65536)
    return fail(ctx, BDFX_EUNSUPPORTED, "LDS per block %zu exceeds 64 KiB", b.cfg.lds_bytes);
  if (queue) {
    b.cfg.grid = static_cast<int>(grid[k]);
  } else {
    if (need > INT32_MAX) return fail(ctx, BDFX_EUNSUPPORTED, "too many cells for one grid");
    b.cfg.grid = static_cast<int>(need);
  }
  return BDFX_OK;
}

// The one launch of a two-mechanism batch (BDFX_SCHED_FUSED): the bins of the
// larger and the smaller mechanism become bins A and B of k_integrate_pair,
// with bin A's register budget and table placement.  A block holds wa A-waves
// and wb B-waves (wa + wb <= 4, wb >= 0, LDS within the device's per-block
// limit); the shape chosen keeps as many A-waves per CU as bin A's own launch
// has and, among those, adds the most B-waves, which then run in the register
// and LDS room A leaves (with none left, the A-waves take the B cells after
// their own, in one launch).  The grid holds as many blocks as fit the GPU.  Used when
// both mechanisms are isothermal A + B <=> C mechanisms on the direct solver
// with the analytic Jacobian, their padded sizes form a compiled pair, an A
// area holds a B cell and some shape keeps A's resident waves; otherwise
// ctx->pair stays null and the bins are launched one after the other (one
// cell per wave in either case).
static int configure_pair(bdfx_ctx ctx) {
  ctx->pair = nullptr;
  if (ctx->opt.scheduler != BDFX_SCHED_FUSED || ctx->bins.size() != 2 || ctx->pair_off)
    return BDFX_OK;
  if (ctx->opt.jacobian != BDFX_JAC_ANALYTIC || ctx->opt.gmres_maxl > 0 || ctx->opt.lockstep > 0)
    return BDFX_OK;
  int ia = 0, ib = 1;
  if (ctx->bins[0].se->S < ctx->bins[1].se->S) std::swap(ia, ib);
  const Bin &a = ctx->bins[ia], &b = ctx->bins[ib];
  const bdfx_mech ma = ctx->mechs[a.mech], mb = ctx->mechs[b.mech];
  if (a.count == 0 || b.count == 0 || !ma->abc || !mb->abc || ma->thermal || mb->thermal ||
      a.cells_per_wave != 1 || b.cells_per_wave != 1)
    return BDFX_OK;
  const PairEntry *pe = pair_for(a.se->S, b.se->S);
  if (!pe) return BDFX_OK;
  const bool fp32 = ctx->opt.lu_precision == 32;
  const int32_t lds_b = static_cast<int32_t>(align_up(
      bdfx::lds_doubles(b.se->S, mb->R, fp32 ? 4 : 8, bdfx::kTabLds, false, 0,
                        bdfx::inv_tail(b.se->S, fp32 ? 4 : 8, false, bdfx::kLinAnalytic, false, 1)),
      2));
  if (a.lds_doubles < lds_b) return BDFX_OK;
  // A-waves per CU in bin A's own launch
  int occ_a = 0;
  HIPCHK(ctx, a.se->occupancy(fp32, a.waves_per_simd, a.tab, 1, kernel_flags(ctx, ma),
                              a.cfg.block, a.cfg.lds_bytes, &occ_a));
  const int a_per_cu = occ_a * std::max(a.waves_per_block, 1);
  int best_a = 0, best_b = 0, best_wa = 0, best_wb = 0, best_occ = 0;
  // (wb = 0: blocks of larger-mechanism waves only, which take the smaller
  // mechanism's cells once their own are done)
  for (int wa = 1; wa <= 4; ++wa)
    for (int wb = 0; wa + wb <= 4; ++wb) {
      const size_t lds = (static_cast<size_t>(wa) * a.lds_doubles + wb * lds_b) * 8;
      if (lds > static_cast<size_t>(ctx->lds_max_block)) continue;
      int occ = 0;
      HIPCHK(ctx, pe->occupancy(fp32, a.waves_per_simd, a.tab, bdfx::kWave * (wa + wb), lds, &occ));
      const int na = occ * wa, nb = occ * wb;
      if (na > best_a || (na == best_a && nb > best_b)) {
        best_a = na;
        best_b = nb;
        best_wa = wa;
        best_wb = wb;
        best_occ = occ;
      }
    }
  if (best_occ < 1 || best_a < a_per_cu) return BDFX_OK;
  const size_t lds = (static_cast<size_t>(best_wa) * a.lds_doubles + best_wb * lds_b) * 8;
  int64_t grid = static_cast<int64_t>(ctx->opt.blocks_per_cu > 0 ? ctx->opt.blocks_per_cu : best_occ) *
                 ctx->n_cu;
  if (a.tab == bdfx::kTabGlobal) grid = std::min<int64_t>(grid, ctx->kk_slots / best_wa);
  grid = std::min<int64_t>(grid, (a.count + b.count + best_wa + best_wb - 1) / (best_wa + best_wb));
  if (grid < 1) return BDFX_OK;
  ctx->pair = pe;
  ctx->pair_a = ia;
  ctx->pair_b = ib;
  ctx->pair_waves = best_wa;
  ctx->pair_lds_b = lds_b;
  ctx->pair_cfg.grid = static_cast<int>(grid);
  ctx->pair_cfg.block = bdfx::kWave * (best_wa + best_wb);
  ctx->pair_cfg.lds_bytes = lds;
  return BDFX_OK;
}

// Kernel, LDS size and grid of every bin (called by bdfx_bind).
static int configure_bins(bdfx_ctx ctx) {
  for (Bin &b : ctx->bins) {
    if (!b.tuned) {
      b.waves_per_simd = ctx->opt.waves_per_simd;
      b.waves_per_block = ctx->opt.waves_per_block > 0 ? ctx->opt.waves_per_block : 1;
      b.queue_chunk = ctx->opt.queue_chunk > 0 ? ctx->opt.queue_chunk : 1;
      // two cells per wave where the mechanism fits a half-wave
      const SizeEntry *se = size_for(ctx->mechs[b.mech]->n);
      b.cells_per_wave =
          ctx->opt.cells_per_wave == 2 && se && two_cells_per_wave_ok(ctx, ctx->mechs[b.mech], se->S)
              ? 2
              : 1;
    }
    if (const int rc = configure_bin(ctx, b)) return rc;
  }
  return configure_pair(ctx);
}

static bdfx::Params make_params(bdfx_ctx ctx, const Bin &b, double t0, double tout) {
  const bdfx_mech m = ctx->mechs[b.mech];
  bdfx::Params P{};
  P.mech = m->dev;
  P.n_list = b.count;
  P.list = ctx->mechs.size() > 1 ? reinterpret_cast<const int32_t *>(ctx->ws + ctx->off_bins) +
                                       b.offset
                                 : nullptr;
  P.y = ctx->y;
  P.ldy = ctx->ldy;
  P.ldk = ctx->ldk;
  P.T = ctx->T;
  P.kscale = ctx->kscale;
  P.F = ctx->F;
  P.status = ctx->status;
  P.stats = reinterpret_cast<bdfx::CellStats *>(ctx->stats);
  P.t0 = t0;
  P.tout = tout;
  P.rtol = ctx->opt.rtol;
  if (ctx->typical) {
    P.atol = reinterpret_cast<const double *>(ctx->ws + ctx->off_tatol) +
             static_cast<int64_t>(b.mech) * ctx->S_max;
    P.atol_len = ctx->S_max;
  } else {
    P.atol = ctx->d_atol;
    P.atol_len = static_cast<int32_t>(ctx->atol.size());
  }
  P.max_order = ctx->opt.max_order;
  P.max_steps = ctx->opt.max_steps;
  P.max_netf = ctx->opt.max_err_test_fails;
  P.max_ncf = ctx->opt.max_conv_fails;
  P.n_sp = m->n;
  P.gmres_maxl = ctx->opt.gmres_maxl;
  P.queue = reinterpret_cast<uint32_t *>(ctx->ws + ctx->off_queue) + b.mech;
  P.chunk = b.queue_chunk;
  P.kk_slots = ctx->kk_slots ? reinterpret_cast<double *>(ctx->ws + ctx->off_kk) : nullptr;
  P.kk_nslots = ctx->kk_slots;
  if (ctx->opt.record_steps > 0) {
    if (ctx->opt.checkpoint_every > 0) {
      P.ckpt = reinterpret_cast<double *>(ctx->ws + ctx->off_ckpt);
      P.ckpt_setup = reinterpret_cast<double *>(ctx->ws + ctx->off_ckpt_setup);
      P.ckpt_every = ctx->opt.checkpoint_every;
      P.ckpt_cap = ctx->ckpt_cap;
      P.ckpt_vs = ctx->ckpt_vs;
    } else {
      P.rec = reinterpret_cast<double *>(ctx->ws + ctx->off_rec);
    }
    P.rec_cap = ctx->opt.record_steps;
    P.rec_stride = ctx->rec_stride;
    P.rec_n = reinterpret_cast<int32_t *>(ctx->ws + ctx->off_recn);
    P.rec_hpad = reinterpret_cast<double *>(ctx->ws + ctx->off_rechpad);
    P.rec_y0 = reinterpret_cast<double *>(ctx->ws + ctx->off_recy0);
  }
  return P;
}

int bdfx_integrate(bdfx_ctx ctx, double t0, double t_out) {
  if (!ctx) return BDFX_EINVAL;
  if (!ctx->bound) return fail(ctx, BDFX_EORDER, "bdfx_bind must precede bdfx_integrate");
  if (!(t_out > t0) || !std::isfinite(t0) || !std::isfinite(t_out))
    return fail(ctx, BDFX_EINVAL, "need finite t_out > t0");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const bool fp32 = ctx->opt.lu_precision == 32;
  const bool queue = ctx->opt.scheduler != BDFX_SCHED_STATIC;
  if (queue) HIPCHK(ctx, bdfx_launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->ws + ctx->off_queue),
                                              64, 0u, ctx->stream));
  if (ctx->pair) {
    const Bin &a = ctx->bins[ctx->pair_a], &b = ctx->bins[ctx->pair_b];
    bdfx::Params PA = make_params(ctx, a, t0, t_out), PB = make_params(ctx, b, t0, t_out);
    PA.use_queue = PB.use_queue = 1;
    PA.lds_doubles = a.lds_doubles;
    PB.lds_doubles = ctx->pair_lds_b;
    PA.pair_waves = PB.pair_waves = ctx->pair_waves;
    HIPCHK(ctx, ctx->pair->launch(PA, PB, fp32, a.waves_per_simd, a.tab, ctx->pair_cfg,
                                  ctx->stream));
    ctx->last_t0 = t0;
    ctx->last_tout = t_out;
    ctx->integrated = true;
    return BDFX_OK;
  }
  for (const Bin &b : ctx->bins) {
    if (b.count == 0 || b.cfg.grid < 1) continue;
    bdfx::Params P = make_params(ctx, b, t0, t_out);
    P.use_queue = queue ? 1 : 0;
    P.lds_doubles = b.lds_doubles;
    HIPCHK(ctx, b.se->launch(P, fp32, b.waves_per_simd, b.tab, b.cells_per_wave,
                             kernel_flags(ctx, ctx->mechs[b.mech]), b.cfg, ctx->stream));
  }
  ctx->last_t0 = t0;
  ctx->last_tout = t_out;
  ctx->integrated = true;
  return BDFX_OK;
}

int bdfx_perturb(bdfx_ctx ctx, uint64_t seed, int64_t outer_step, double amplitude) {
  if (!ctx) return BDFX_EINVAL;
  if (!ctx->bound) return fail(ctx, BDFX_EORDER, "bdfx_bind must precede bdfx_perturb");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  for (const Bin &b : ctx->bins) {
    if (b.count == 0) continue;
    bdfx::Params P = make_params(ctx, b, 0.0, 0.0);
    HIPCHK(ctx, bdfx_launch_perturb(P, seed, outer_step, amplitude, ctx->stream));
  }
  ctx->integrated = false;
  return BDFX_OK;
}

// ---------------------------------------------------------------------------
// autotuning of the launch shape
// ---------------------------------------------------------------------------

static bdfx_tuning tuning_of(const Bin &b) {
  bdfx_tuning t{};
  t.mech = b.mech;
  t.waves_per_simd = b.waves_per_simd;
  t.waves_per_block = b.waves_per_block;
  t.queue_chunk = b.queue_chunk;
  t.cells_per_wave = b.cells_per_wave;
  t.sample_cells = b.tune_sample;
  t.ms = b.tune_ms;
  t.tables = b.tab;
  return t;
}

static bdfx_tuning tuning_of(bdfx_ctx ctx, const Bin &b) {
  bdfx_tuning t = tuning_of(b);
  t.fused = ctx->pair != nullptr ? 1 : 0;
  return t;
}

}  // extern "C"

// Times, on the first ns cells of both bins (rows saved and restored around
// each run, first run a warm-up), the two bins' own launches one after the
// other and the one-launch form (ctx->pair set); both in ms.
static hipError_t time_pair(bdfx_ctx ctx, double t0, double t_out, int64_t ns, hipEvent_t e0,
                            hipEvent_t e1, float *t_seq, float *t_pair) {
  const bool fp32 = ctx->opt.lu_precision == 32;
  const Bin *bin[2] = {&ctx->bins[ctx->pair_a], &ctx->bins[ctx->pair_b]};
  Bin tb[2];
  bdfx::Params P[2];
  double *save[2];
  for (int k = 0; k < 2; ++k) {
    tb[k] = *bin[k];
    tb[k].count = std::min(ns, bin[k]->count);
    P[k] = make_params(ctx, tb[k], t0, t_out);
    P[k].use_queue = 1;
    P[k].lds_doubles = bin[k]->lds_doubles;
    P[k].chunk = bin[k]->queue_chunk;
    save[k] = reinterpret_cast<double *>(ctx->ws + ctx->off_tune) +
              static_cast<int64_t>(k) * ctx->tune_cells * ctx->S_max;
  }
  uint32_t *qctr = reinterpret_cast<uint32_t *>(ctx->ws + ctx->off_queue);
  hipError_t e = hipSuccess;
  for (int form = 0; form < 2 && e == hipSuccess; ++form) {
    float total = 0.0f;
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
      for (int k = 0; k < 2 && e == hipSuccess; ++k)
        e = bdfx_launch_copy_rows(ctx->y, ctx->ldy, P[k].list, tb[k].count,
                                  ctx->mechs[tb[k].mech]->n, save[k], false, ctx->stream);
      if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
      if (e == hipSuccess) e = bdfx_launch_fill_u32(qctr, 64, 0u, ctx->stream);
      if (form == 0) {
        for (int k = 0; k < 2 && e == hipSuccess; ++k) {
          const bdfx_mech m = ctx->mechs[tb[k].mech];
          e = tb[k].se->launch(P[k], fp32, tb[k].waves_per_simd, tb[k].tab, 1, kernel_flags(ctx, m),
                               tb[k].cfg, ctx->stream);
        }
      } else if (e == hipSuccess) {
        bdfx::Params PA = P[0], PB = P[1];
        PB.lds_doubles = ctx->pair_lds_b;
        PA.pair_waves = PB.pair_waves = ctx->pair_waves;
        e = ctx->pair->launch(PA, PB, fp32, tb[0].waves_per_simd, tb[0].tab, ctx->pair_cfg,
                              ctx->stream);
      }
      if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
      for (int k = 0; k < 2 && e == hipSuccess; ++k)
        e = bdfx_launch_copy_rows(ctx->y, ctx->ldy, P[k].list, tb[k].count,
                                  ctx->mechs[tb[k].mech]->n, save[k], true, ctx->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) total += ms;
    }
    (form == 0 ? *t_seq : *t_pair) = total / 2.0f;
  }
  return e;
}

extern "C" {

int bdfx_autotune(bdfx_ctx ctx, double t0, double t_out, int64_t sample_cells, bdfx_tuning *out) {
  if (!ctx) return BDFX_EINVAL;
  if (!ctx->bound) return fail(ctx, BDFX_EORDER, "bdfx_bind must precede bdfx_autotune");
  if (!(t_out > t0) || !std::isfinite(t0) || !std::isfinite(t_out))
    return fail(ctx, BDFX_EINVAL, "need finite t_out > t0");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (ctx->opt.lockstep > 0) {  // lock-step kernels have one launch shape: nothing to time
    for (size_t bi = 0; bi < ctx->bins.size() && out; ++bi) out[bi] = tuning_of(ctx, ctx->bins[bi]);
    return BDFX_OK;
  }
  const bool fp32 = ctx->opt.lu_precision == 32;
  const bool queue = ctx->opt.scheduler != BDFX_SCHED_STATIC;
  const int64_t ns = sample_cells > 0 ? std::min(sample_cells, ctx->tune_cells) : ctx->tune_cells;
  ctx->integrated = false;  // the timed runs overwrite the sample cells' step records
  double *save = reinterpret_cast<double *>(ctx->ws + ctx->off_tune);
  uint32_t *qctr = reinterpret_cast<uint32_t *>(ctx->ws + ctx->off_queue);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(ctx, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return fail(ctx, BDFX_EHIP, "hipEventCreate failed");
  }
  int rc = BDFX_OK;
  const int wps_c[] = {0, 3, 4, 5}, wpb_c[] = {1, 2, 4}, chunk_c[] = {1, 4}, cpw_c[] = {1, 2};
  for (size_t bi = 0; bi < ctx->bins.size() && rc == BDFX_OK; ++bi) {
    Bin &b = ctx->bins[bi];
    if (b.count == 0) continue;
    const bdfx_mech m = ctx->mechs[b.mech];
    Bin trial = b;
    trial.count = std::min(ns, b.count);  // the first cells of the bin
    bdfx::Params P = make_params(ctx, trial, t0, t_out);
    P.use_queue = queue ? 1 : 0;
    float best = 0.0f;
    bool have = false;
    Bin pick = b;
    for (int cpw : cpw_c)
    for (int wps : wps_c)
      for (int wpb : wpb_c)
        for (int chunk : chunk_c) {
          if (!queue && chunk != 1) continue;
          if (cpw == 2 && !two_cells_per_wave_ok(ctx, m, b.se->S)) continue;
          trial.cells_per_wave = cpw;
          trial.waves_per_simd = wps;
          trial.waves_per_block = wpb;
          trial.queue_chunk = chunk;
          if (configure_bin(ctx, trial) != BDFX_OK) continue;  // e.g. LDS too large
          P.lds_doubles = trial.lds_doubles;
          P.chunk = chunk;
          float total = 0.0f;
          hipError_t e = hipSuccess;
          for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {  // rep 0 warms up
            e = bdfx_launch_copy_rows(ctx->y, ctx->ldy, P.list, trial.count, m->n, save, false,
                                      ctx->stream);
            if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
            if (e == hipSuccess && queue) e = bdfx_launch_fill_u32(qctr, 64, 0u, ctx->stream);
            if (e == hipSuccess)
              e = trial.se->launch(P, fp32, wps, trial.tab, cpw, kernel_flags(ctx, m), trial.cfg,
                                   ctx->stream);
            if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
            if (e == hipSuccess)
              e = bdfx_launch_copy_rows(ctx->y, ctx->ldy, P.list, trial.count, m->n, save, true,
                                        ctx->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) total += ms;
          }
          if (e != hipSuccess) {
            rc = fail(ctx, BDFX_EHIP, "autotune trial: %s", hipGetErrorString(e));
            break;
          }
          if (!have || total < best) {
            best = total;
            have = true;
            pick = trial;
          }
        }
    if (rc != BDFX_OK || !have) break;
    b.waves_per_simd = pick.waves_per_simd;
    b.waves_per_block = pick.waves_per_block;
    b.queue_chunk = pick.queue_chunk;
    b.cells_per_wave = pick.cells_per_wave;
    b.tuned = true;
    b.tune_sample = trial.count;
    b.tune_ms = best / 2.0f;
    rc = configure_bin(ctx, b);
  }
  ctx->pair_off = false;
  if (rc == BDFX_OK) rc = configure_pair(ctx);
  if (rc == BDFX_OK && ctx->pair) {
    // the one launch against the two bins' own launches, on both samples
    float t_seq = 0.0f, t_pair = 0.0f;
    const hipError_t e = time_pair(ctx, t0, t_out, ns, e0, e1, &t_seq, &t_pair);
    if (e != hipSuccess) {
      rc = fail(ctx, BDFX_EHIP, "autotune pair trial: %s", hipGetErrorString(e));
    } else if (t_pair > t_seq) {
      ctx->pair_off = true;
      ctx->pair = nullptr;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  for (size_t bi = 0; bi < ctx->bins.size() && out && rc == BDFX_OK; ++bi)
    out[bi] = tuning_of(ctx, ctx->bins[bi]);
  if (rc == BDFX_OK) {
    const hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(ctx, BDFX_EHIP, "%s", hipGetErrorString(e));
  }
  return rc;
}

int bdfx_set_tuning(bdfx_ctx ctx, const bdfx_tuning *t, int32_t n) {
  if (!ctx || (n > 0 && !t)) return BDFX_EINVAL;
  if (!ctx->bound) return fail(ctx, BDFX_EORDER, "bdfx_bind must precede bdfx_set_tuning");
  for (int32_t k = 0; k < n; ++k) {
    if (t[k].waves_per_simd != 0 && (t[k].waves_per_simd < 3 || t[k].waves_per_simd > 5))
      return fail(ctx, BDFX_EINVAL, "waves_per_simd must be 0, 3, 4 or 5");
    if (t[k].waves_per_block < 1 || t[k].waves_per_block > 16 || t[k].queue_chunk < 1 ||
        (t[k].cells_per_wave != 1 && t[k].cells_per_wave != 2))
      return fail(ctx, BDFX_EINVAL, "invalid launch shape");
    for (Bin &b : ctx->bins)
      if (b.mech == t[k].mech) {
        b.waves_per_simd = t[k].waves_per_simd;
        b.waves_per_block = t[k].waves_per_block;
        b.queue_chunk = t[k].queue_chunk;
        b.cells_per_wave = t[k].cells_per_wave;
        b.tuned = true;
        b.tune_sample = 0;
        b.tune_ms = 0.0f;
        if (const int rc = configure_bin(ctx, b)) return rc;
      }
  }
  return configure_pair(ctx);
}

int bdfx_typical_atol(bdfx_ctx ctx, double eta, double *d_typical) {
  if (!ctx) return BDFX_EINVAL;
  if (!ctx->bound) return fail(ctx, BDFX_EORDER, "bdfx_bind must precede bdfx_typical_atol");
  if (!std::isfinite(eta) || eta < 0.0) return fail(ctx, BDFX_EINVAL, "eta must be finite, >= 0");
  if (eta == 0.0) {
    ctx->typical = false;
    return BDFX_OK;
  }
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const int n_mech = static_cast<int>(ctx->mechs.size());
  double *part = reinterpret_cast<double *>(ctx->ws + ctx->off_ext);
  int32_t S[BDFX_MAX_MECH] = {0}, nblk[BDFX_MAX_MECH] = {0};
  int64_t off[BDFX_MAX_MECH] = {0};
  for (int m = 0; m < n_mech; ++m) {
    S[m] = ctx->mechs[m]->n;
    off[m] = static_cast<int64_t>(m) * kExtMaxBlocks * 2 * bdfx::kWave;
  }
  for (const Bin &b : ctx->bins) {
    if (b.count == 0) continue;
    const int32_t *list = n_mech > 1 ? reinterpret_cast<const int32_t *>(ctx->ws + ctx->off_bins) +
                                           b.offset
                                     : nullptr;
    const int nb = bdfx_extremes_blocks(b.count, S[b.mech], kExtMaxBlocks);
    HIPCHK(ctx, bdfx_launch_extremes(ctx->y, ctx->ldy, list, b.count, S[b.mech], nb,
                                     part + off[b.mech], ctx->stream));
    nblk[b.mech] = nb;
  }
  HIPCHK(ctx, bdfx_launch_typical(n_mech, ctx->S_max, S, nblk, off, part, eta,
                                  reinterpret_cast<double *>(ctx->ws + ctx->off_tatol), d_typical,
                                  ctx->stream));
  ctx->typical = true;
  return BDFX_OK;
}

// Scratch of bdfx_typical_atol_static: the k_extremes block partials of one
// call (kExtMaxBlocks blocks x {minimum, maximum} x 64 species, 256 KiB),
// resident on every device the library runs on until the process ends.  Host
// code never passes this name to a kernel: the kernels take the device address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[kExtMaxBlocks * 2 * bdfx::kWave];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

// Device address of this device's copy of `scratch` (the device must be
// current); looked up once per device.
hipError_t scratch_on(int device, double **out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double *>(p);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}
}  // namespace

int bdfx_typical_atol_static(int device, void *hip_stream, const double *d_y, int64_t n_cells,
                             int32_t ldy, int32_t n_species, double eta, double *d_atol,
                             double *d_typical) {
  if (!d_y || !d_atol) return fail(nullptr, BDFX_EINVAL, "d_y and d_atol must not be NULL");
  if (n_cells < 1) return fail(nullptr, BDFX_EINVAL, "n_cells must be >= 1");
  if (n_species < 1 || n_species > BDFX_MAX_SPECIES)
    return fail(nullptr, BDFX_EINVAL, "n_species %d outside 1..%d (the scratch holds %d species)",
                n_species, BDFX_MAX_SPECIES, BDFX_MAX_SPECIES);
  if (ldy < n_species) return fail(nullptr, BDFX_EINVAL, "ldy %d < n_species %d", ldy, n_species);
  if (!std::isfinite(eta) || !(eta > 0.0)) return fail(nullptr, BDFX_EINVAL, "eta must be finite, > 0");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(nullptr, BDFX_EHIP, "no HIP device available");
  if (device < 0 || device >= ndev || device >= kMaxDevices)
    return fail(nullptr, BDFX_EINVAL, "bad device %d", device);
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess)
    return fail(nullptr, BDFX_EHIP, "cannot select device %d", device);
  const hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  double *part = nullptr;
  hipError_t e = scratch_on(device, &part);
  const int32_t S[1] = {n_species};
  const int32_t nblk[1] = {bdfx_extremes_blocks(n_cells, n_species, kExtMaxBlocks)};
  const int64_t off[1] = {0};
  if (e == hipSuccess) e = bdfx_launch_extremes(d_y, ldy, nullptr, n_cells, n_species, nblk[0], part, s);
  if (e == hipSuccess) e = bdfx_launch_typical(1, n_species, S, nblk, off, part, eta, d_atol, d_typical, s);
  hipSetDevice(prev);
  if (e != hipSuccess) return fail(nullptr, BDFX_EHIP, "typical values: %s", hipGetErrorString(e));
  return BDFX_OK;
}

int bdfx_get_tuning(bdfx_ctx ctx, bdfx_tuning *out, int32_t n) {
  if (!ctx || (n > 0 && !out) || n < 0) return BDFX_EINVAL;
  if (!ctx->bound) return fail(ctx, BDFX_EORDER, "bdfx_bind must precede bdfx_get_tuning");
  for (int32_t k = 0; k < n && k < static_cast<int32_t>(ctx->bins.size()); ++k)
    out[k] = tuning_of(ctx, ctx->bins[k]);
  return BDFX_OK;
}

int bdfx_stats_summary(bdfx_ctx ctx, bdfx_summary *out) {
  if (!ctx || !out) return BDFX_EINVAL;
  if (!ctx->bound) return fail(ctx, BDFX_EORDER, "nothing bound");
  if (!ctx->stats && ctx->N > 0) return fail(ctx, BDFX_EINVAL, "no stats buffer bound");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  std::vector<bdfx_cell_stats> st(ctx->N);
  if (ctx->N)
    HIPCHK(ctx, hipMemcpyAsync(st.data(), ctx->stats, ctx->N * sizeof(bdfx_cell_stats),
                               hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  std::memset(out, 0, sizeof(*out));
  out->n_cells = ctx->N;
  for (const auto &s : st) {
    if (s.status == 0)
      out->n_success++;
    else
      out->n_failed++;
    if (s.status <= 0 && s.status >= -10) out->status_count[-s.status]++;
    out->nst += s.nst;
    out->nfe += s.nfe;
    out->nni += s.nni;
    out->nsetups += s.nsetups;
    out->netf += s.netf;
    out->ncfn += s.ncfn;
    out->nli += s.nli;
    out->ncfl += s.ncfl;
    out->max_nst = std::max<int64_t>(out->max_nst, s.nst);
  }
  return BDFX_OK;
}

int bdfx_get_record_layout(bdfx_ctx ctx, bdfx_record_layout *out) {
  if (!ctx || !out) return fail(ctx, BDFX_EINVAL, "NULL argument");
  if (!ctx->bound || ctx->opt.record_steps <= 0)
    return fail(ctx, BDFX_EORDER, "no step record: bind with record_steps > 0 first");
  if (ctx->opt.checkpoint_every > 0)
    return fail(ctx, BDFX_EUNSUPPORTED, "checkpointed records hold no per-step rows");
  out->cap = ctx->opt.record_steps;
  out->stride = ctx->rec_stride;
  out->off_steps = ctx->off_rec;
  out->off_count = ctx->off_recn;
  out->off_hpad = ctx->off_rechpad;
  out->off_y0 = ctx->off_recy0;
  return BDFX_OK;
}

int bdfx_adjoint(bdfx_ctx ctx, const double *d_ybar, double *d_y0bar, double *d_lnA_bar) {
  if (!ctx) return BDFX_EINVAL;
  if (!ctx->bound) return fail(ctx, BDFX_EORDER, "bdfx_bind must precede bdfx_adjoint");
  if (ctx->opt.record_steps <= 0)
    return fail(ctx, BDFX_EORDER, "the forward run must be planned with record_steps > 0");
  if (!ctx->integrated)
    return fail(ctx, BDFX_EORDER, "bdfx_integrate must precede bdfx_adjoint (no perturb since)");
  if (!d_ybar || !d_y0bar) return fail(ctx, BDFX_EINVAL, "ybar and y0bar required");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  double *pbar = reinterpret_cast<double *>(ctx->ws + ctx->off_pbar);
  const int K = ctx->opt.checkpoint_every;
  for (const Bin &b : ctx->bins) {
    if (b.count == 0) continue;
    const bdfx_mech m = ctx->mechs[b.mech];
    const SizeEntry *se = size_for(m->S);
    bdfx::Params P = make_params(ctx, b, ctx->last_t0, ctx->last_tout);
    P.ybar = d_ybar;
    P.y0bar = d_y0bar;
    P.pbar = pbar;
    P.ldp = ctx->R_max;
    const int32_t lds_sweep = static_cast<int32_t>(align_up(bdfx::lds_doubles_adjoint(se->S, m->R), 2));
    bdfx::LaunchCfg cfg;
    cfg.block = bdfx::kWave;  // one wave per block, one block per cell
    cfg.grid = static_cast<int>(b.count);
    cfg.lds_bytes = static_cast<size_t>(lds_sweep) * 8;
    if (cfg.lds_bytes > 65536)
      return fail(ctx, BDFX_EUNSUPPORTED, "adjoint LDS per block %zu exceeds 64 KiB", cfg.lds_bytes);
    P.lds_doubles = lds_sweep;
    if (K == 0) {
      HIPCHK(ctx, se->adjoint(P, 0, 0, m->abc, cfg, ctx->stream));
    } else {
      // passes over the segments from the last: rerun, then sweep
      P.seg = reinterpret_cast<double *>(ctx->ws + ctx->off_seg);
      P.seg_rows = K + bdfx::kQmax + 1;
      P.adj = reinterpret_cast<double *>(ctx->ws + ctx->off_adj);
      bdfx::Params PR = P;
      PR.lds_doubles = static_cast<int32_t>(align_up(
          bdfx::lds_doubles(se->S, m->R, 8, bdfx::kTabLds, false, 0,
                            bdfx::inv_tail(se->S, 8, false, bdfx::kLinAnalytic, false, 1)),
          2));
      bdfx::LaunchCfg cr = cfg;
      cr.lds_bytes = static_cast<size_t>(PR.lds_doubles) * 8;
      for (int j = 0; j < ctx->ckpt_cap; ++j) {
        HIPCHK(ctx, se->adjoint(PR, 1, j, m->abc, cr, ctx->stream));
        HIPCHK(ctx, se->adjoint(P, 2, j, m->abc, cfg, ctx->stream));
      }
    }
    if (d_lnA_bar)
      HIPCHK(ctx, bdfx_launch_sum_cells(pbar, ctx->R_max, P.list, b.count, m->R,
                                        d_lnA_bar + static_cast<int64_t>(b.mech) * ctx->R_max,
                                        ctx->stream));
  }
  return BDFX_OK;
}

}  // extern "C"
