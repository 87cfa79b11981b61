// Host side of the C ABI declared in include/fire.h: contexts, landscape and
// reference-map storage, argument checks, schedule selection and the launch
// sequences of the simulation, GA, ensemble and scan entry points.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "fire.h"
#include "fire_internal.h"

using namespace firegpu;

namespace {

struct LandscapeHost {
  bool live = false;
  int W = 0, H = 0, stride = 0;
  uint8_t forest = 1;
  uint4 *rec = nullptr;
  double *cov = nullptr;  // [H*W][2] psi, slope/100, then [H*W][8] omega
  uint32_t *blocked = nullptr;
  uint8_t *burn_steps = nullptr;  // device [256], NULL = one step for every type
  // observed share of simulations that left their LDS window (moving
  // average over window runs; windows are not used while it exceeds
  // kWindowRetryMax)
  float win_frac = 0.f;
  int win_obs = 0;
  // landscape means for ordering simulations by expected fire size: share
  // of forest among burnable cells, mean psi, mean sigma of an edge, and
  // the number of burnable cells
  double mean_forest = 0.0, mean_psi = 0.0, mean_sigma = 0.0;
  int64_t burnable = 0;
};

struct TargetHost {
  bool live = false;
  int landscape_id = -1;
  uint32_t n_ref = 0;
  uint32_t *bits = nullptr;
};

}  // namespace

struct fire_ctx {
  int device = 0;
  int num_cu = 256;
  size_t max_lds = 65536;
  std::string err;
  std::vector<LandscapeHost> ls;
  std::vector<TargetHost> tg;
  LandscapeDev *d_ls = nullptr;
  int d_ls_cap = 0;
  TargetDev *d_tg = nullptr;
  int d_tg_cap = 0;
  uint32_t *d_work = nullptr;   // [0..kMaxClasses) work counters, [kErrWord] error flag
  uint32_t *d_ovf = nullptr;
  size_t ovf_words = 0;
  uint32_t *d_retry = nullptr;  // window runs: per launch, count + simulation list
  size_t retry_words = 0;
  // retry counts of window runs, written into host-mapped memory by the
  // re-run launch (read once stat_ev[i] has passed): slot i holds the count
  // of a launch on landscape stat_ls[i] of stat_n[i] simulations
  static constexpr int kStatSlots = 16;
  uint32_t *h_stat = nullptr;
  hipEvent_t stat_ev[kStatSlots] = {};
  int stat_ls[kStatSlots] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
  int stat_n[kStatSlots] = {};
  // workgroups of each simulation-kernel variant resident per CU as far as
  // registers allow ([threads 64..1024][table][turn-off times][window];
  // 0 = unknown)
  int reg_blocks[5][2][2][3] = {};  // [threads][table][dur][whole LDS, window, global bitset]
  // resident workgroups per CU of (variant, dynamic LDS bytes), as the
  // runtime computes them (allocation granularity included)
  std::map<std::pair<int, size_t>, int> occ_cache;
  uint32_t *d_tables = nullptr;
  size_t tables_words = 0;
  // staging of host descriptors for fire_run
  void *h_stage = nullptr;
  void *d_stage = nullptr;
  size_t stage_bytes = 0;
  hipEvent_t stage_done = nullptr;
  bool stage_pending = false;
  // fixed schedule (autotuner) or built-in choice
  bool sched_fixed = false;
  fire_schedule sched{};
  // per size-class schedules (autotuner): (log2 bucket of max_cells, batch
  // kind: see batch_kind) -> schedule
  struct ClassSched {
    int bucket;
    int kind;
    fire_schedule s;
  };
  std::vector<ClassSched> class_sched;
  // side streams and events for running size classes concurrently
  hipStream_t side[7] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[8] = {};
  // GA scratch
  double *d_ga = nullptr;
  size_t ga_bytes = 0;
  // per-cell ablation path: two state planes, betas, counters, host mirror
  uint8_t *d_dense = nullptr;
  size_t dense_bytes = 0;
  unsigned long long *h_dense = nullptr;
  // set once a simulation launch has been recorded into a stream capture:
  // from then on a scratch buffer that a later call outgrows is retired
  // (kept allocated until the context is destroyed) instead of freed, so
  // that captured graphs never address freed memory
  bool captured = false;
  std::vector<void *> retired;
  // this device's copy of the no-allocation scratch array (set at creation)
  uint32_t *noalloc = nullptr;
  // caller's buffer for per-simulation start/end clocks (fire_set_sim_timing)
  uint64_t *times = nullptr;
  int64_t times_cap = 0;
};

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxClasses = 8;   // concurrent persistent launches per fire_run
constexpr int kErrWord = 16;     // error flag word in d_work
constexpr int kWorkWords = 32;

int cells_bucket(int64_t cells) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < cells) ++b;
  return b;
}

fire_status fail(fire_ctx *c, fire_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

#define HIP_OR_FAIL(ctx, expr)                                             \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess)                                                  \
      return fail((ctx), e_ == hipErrorOutOfMemory ? FIRE_E_OOM            \
                                                   : FIRE_E_DEVICE,        \
                  "%s: %s", #expr, hipGetErrorString(e_));                \
  } while (0)

hipError_t ensure(void **p, size_t *have, size_t want) {
  if (*have >= want && *p) return hipSuccess;
  if (*p) {
    hipError_t e = hipFree(*p);
    *p = nullptr;
    *have = 0;
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipMalloc(p, want);
  if (e == hipSuccess) *have = want;
  return e;
}

bool stream_capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return cs != hipStreamCaptureStatusNone;
}

// Grow a context scratch buffer to `want` bytes. Never during a stream
// capture (the graph would keep the address of a buffer a later call could
// replace): the caller gets FIRE_E_UNSUPPORTED and should run the same call
// once eagerly first. Once anything has been captured, the old buffer is
// retired rather than freed.
fire_status grow(fire_ctx *c, void **p, size_t *have, size_t want, hipStream_t st,
                 const char *what) {
  if (*have >= want && *p) return FIRE_OK;
  if (stream_capturing(st))
    return fail(c, FIRE_E_UNSUPPORTED,
                "%s would grow from %zu to %zu bytes during stream capture; run the same call "
                "once without capture first", what, *have, want);
  HIP_OR_FAIL(c, hipDeviceSynchronize());
  if (*p && c->captured) {
    c->retired.push_back(*p);
    *p = nullptr;
    *have = 0;
  }
  HIP_OR_FAIL(c, ensure(p, have, want));
  return FIRE_OK;
}

fire_status sync_tables(fire_ctx *c) {
  // mirror the landscape and target tables on the device
  int nl = (int)c->ls.size(), nt = (int)c->tg.size();
  std::vector<LandscapeDev> hl(nl > 0 ? nl : 1);
  for (int i = 0; i < nl; ++i) {
    const LandscapeHost &L = c->ls[i];
    LandscapeDev d{};
    d.W = L.W; d.H = L.H; d.stride = L.stride; d.valid = L.live ? 1 : 0;
    d.rec = L.rec; d.ps = L.cov;
    d.omega = L.cov ? L.cov + 2 * (int64_t)L.W * L.H : nullptr;
    d.blocked = L.blocked;
    d.burn_steps = L.burn_steps;
    d.forest_class = L.forest;
    hl[i] = d;
  }
  std::vector<TargetDev> ht(nt > 0 ? nt : 1);
  for (int i = 0; i < nt; ++i) {
    const TargetHost &T = c->tg[i];
    TargetDev d{};
    d.landscape_id = T.landscape_id; d.valid = T.live ? 1 : 0;
    d.n_ref = T.n_ref; d.bits = T.bits;
    ht[i] = d;
  }
  if (nl > c->d_ls_cap || !c->d_ls) {
    int cap = nl < 16 ? 16 : nl * 2;
    if (c->d_ls && c->captured) c->retired.push_back(c->d_ls);
    else if (c->d_ls) HIP_OR_FAIL(c, hipFree(c->d_ls));
    c->d_ls = nullptr;
    HIP_OR_FAIL(c, hipMalloc(&c->d_ls, sizeof(LandscapeDev) * cap));
    c->d_ls_cap = cap;
  }
  if (nt > c->d_tg_cap || !c->d_tg) {
    int cap = nt < 16 ? 16 : nt * 2;
    if (c->d_tg && c->captured) c->retired.push_back(c->d_tg);
    else if (c->d_tg) HIP_OR_FAIL(c, hipFree(c->d_tg));
    c->d_tg = nullptr;
    HIP_OR_FAIL(c, hipMalloc(&c->d_tg, sizeof(TargetDev) * cap));
    c->d_tg_cap = cap;
  }
  HIP_OR_FAIL(c, hipDeviceSynchronize());
  if (nl > 0)
    HIP_OR_FAIL(c, hipMemcpy(c->d_ls, hl.data(), sizeof(LandscapeDev) * nl,
                             hipMemcpyHostToDevice));
  if (nt > 0)
    HIP_OR_FAIL(c, hipMemcpy(c->d_tg, ht.data(), sizeof(TargetDev) * nt,
                             hipMemcpyHostToDevice));
  return FIRE_OK;
}

bool valid_window(int w) { return w == -1 || w == 0 || (w >= 64 && w <= 4096 && w % 32 == 0); }

bool valid_threads(int t) {
  return t == 64 || t == 128 || t == 256 || t == 512 || t == 1024;
}

// LDS of one simulation workgroup: bitset, two frontier queues, control
// words and, with turn-off times, a remaining-life byte per queue entry.
size_t lds_bytes_for(int bitset_words, int queue_cap, bool dur = false) {
  size_t b = sizeof(uint32_t) * ((size_t)bitset_words + 2 * (size_t)queue_cap + 16);
  if (dur) b += (2 * (size_t)queue_cap + 3) / 4 * 4;
  return b;
}

// Largest queue_cap whose LDS fits `bytes`.
int queue_cap_for(size_t bytes, int bitset_words, bool dur) {
  const size_t fixed = sizeof(uint32_t) * ((size_t)bitset_words + 16) + (dur ? 3 : 0);
  if (bytes <= fixed) return 0;
  return (int)((bytes - fixed) / (dur ? 10 : 8));
}

constexpr int kMaxPerCu = 16;  // built-in workgroups per compute unit, at most
constexpr int64_t kTableBudget = (int64_t)2 << 30;  // bytes of threshold tables per run
// bytes of global-memory burn bitsets per launch (caps the resident
// simulations of a lattice whose bitset does not fit LDS)
constexpr int64_t kGlobalBitsBudget = (int64_t)1 << 30;
// LDS per workgroup left unused by the built-in queue sizing: with every
// byte of an equal share taken, gfx950 kept one workgroup fewer resident
// than the runtime's occupancy figure (measured: 5 x 32.4 KiB ran 4 per CU)
constexpr size_t kLdsMargin = 1024;

int threads_index(int t) { return t == 64 ? 0 : t == 128 ? 1 : t == 256 ? 2 : t == 512 ? 3 : 4; }

// Workgroups of a simulation-kernel variant resident per CU as far as its
// registers allow (queried once per variant; LDS is accounted separately),
// negated for a variant whose registers spill to scratch.
int reg_blocks(fire_ctx *c, int threads, bool table, bool dur, bool win, bool gb = false) {
  int &v = c->reg_blocks[threads_index(threads)][table ? 1 : 0][dur ? 1 : 0][win ? 1 : gb ? 2 : 0];
  if (v == 0) {
    v = sim_occupancy(threads, table, dur, win, 0, gb);
    if (v <= 0) v = 1;
    // a variant that spills registers to scratch is not a built-in choice
    if (sim_scratch_bytes(threads, table, dur, win, gb) > 0) v = -v;
  }
  return v;
}

// Workgroups of a variant resident per CU with `lds` bytes of dynamic LDS.
int resident(fire_ctx *c, int threads, bool table, bool dur, bool win, size_t lds,
             bool gb = false) {
  const int key = threads_index(threads) * 16 + (gb ? 8 : 0) + (table ? 4 : 0) + (dur ? 2 : 0) +
                  (win ? 1 : 0);
  auto it = c->occ_cache.find({key, lds});
  if (it != c->occ_cache.end()) return it->second;
  int v = sim_occupancy(threads, table, dur, win, lds, gb);
  if (v < 0) v = 0;
  c->occ_cache[{key, lds}] = v;
  return v;
}

// Built-in schedule for landscapes of up to max_cells cells. A simulation
// runs in one workgroup, so what bounds a batch is how many simulations are
// resident at once: for each workgroup size the LDS queues take what the
// bitset leaves of an equal share of the compute unit's LDS, the resident
// count is the smaller of that share count and the kernel's register
// occupancy, and the size that keeps the most simulations of the batch
// resident wins (ties: the larger workgroup, whose lanes cover larger
// fronts in one pass).
fire_schedule default_schedule(fire_ctx *c, int64_t max_cells,
                               int bitset_words, int32_t n_params, bool dur = false,
                               int64_t n_sims = (int64_t)1 << 30, bool win = false,
                               bool gb = false) {
  fire_schedule best{};
  int64_t best_conc = -1;
  // a table per parameter vector pays off once each serves a few
  // simulations (the per-trial Eq. 1 evaluation costs several times a
  // 4-byte table read), while the tables fit the budget
  const bool table = n_params <= 8 || (n_sims >= 8 * (int64_t)n_params &&
                                       (int64_t)n_params * max_cells * 32 <= kTableBudget);
  for (int threads : {1024, 512, 256, 128}) {
    int per_cu = 0;
    for (int k = kMaxPerCu; k >= 1; --k) {
      const size_t slot = c->max_lds / k;
      if (slot >= lds_bytes_for(bitset_words, 256, dur)) {
        per_cu = k;
        break;
      }
    }
    if (per_cu == 0) per_cu = 1;
    // the resident workgroups (no more than the batch fills) share the LDS;
    // queues take what is left (less a margin the hardware needs)
    const int64_t need = std::max<int64_t>(1, (n_sims + c->num_cu - 1) / c->num_cu);
    const int rb = reg_blocks(c, threads, table, dur, win, gb);
    if (rb < 0 && threads > 128) continue;  // spills; 128 threads is the fallback
    const int res = (int)std::min<int64_t>(std::min(per_cu, rb < 0 ? -rb : rb), need);
    int qcap = queue_cap_for(c->max_lds / res - kLdsMargin, bitset_words, dur);
    if (qcap > 16384) qcap = 16384;
    while (qcap > 64 &&
           resident(c, threads, table, dur, win, lds_bytes_for(bitset_words, qcap, dur), gb) < res)
      qcap -= 64;
    if (qcap < 64) qcap = 64;
    const int64_t conc = std::min<int64_t>((int64_t)res * c->num_cu, n_sims);
    if (conc > best_conc) {
      best_conc = conc;
      best.threads = threads;
      best.queue_cap = qcap;
      best.table_mode = table ? 1 : 0;
      best.wg_per_cu = res;
    }
  }
  best.window = 0;
  best.wave = 0;
  return best;
}

struct RunPlan {
  fire_schedule s;
  bool wave;  // first launch: one simulation per wavefront (simw_kernel)
  bool dur;  // some landscape of the launch has turn-off times
  // whole-lattice launches whose bitset does not fit LDS keep it in global
  // memory (gb: the first launch, gb2: the re-run launch of a window plan)
  bool gb = false, gb2 = false;
  int bitset_words;
  int64_t max_cells;
  size_t lds;
  int grid;
  // Window runs: the first launch gives each simulation an LDS window of
  // `win` cells a side around its ignition; the simulations whose fire
  // reaches the window edge run again in a second launch over the whole
  // lattice, with the plan below.
  int win;
  fire_schedule s2;
  int bitset_words2;
  size_t lds2;
  int grid2;
};

// Built-in windows only while no window run on the landscape has had to
// repeat a simulation: the repeats run after the window launch, so even a
// few of them cost a whole simulation's latency.
constexpr float kWindowRetryMax = 0.0f;
constexpr int kMinAutoQueue = 1024;      // LDS queue entries a built-in window should leave
// Built-in windows only for batches of replicates (at most this many
// parameter vectors): with many different vectors (a GA population, Monte
// Carlo draws) some fires outgrow any window and their repeats, which start
// only after the window launch ends, cost more than the residency gains.
constexpr int kWindowMaxParams = 8;
// LDS queue entries of a built-in wavefront-per-simulation plan (fires whose
// front exceeds it are run again by the workgroup kernel)
constexpr int kWaveQueue = 512;

// LDS, queue and residency of one launch shape; false if it cannot fit.
bool shape_launch(fire_ctx *c, fire_schedule &s, int bitset_words, bool dur, bool win,
                  int32_t n_sims, size_t *lds_out, int *grid_out, bool gb = false) {
  if (dur && lds_bytes_for(bitset_words, s.queue_cap, true) > c->max_lds) {
    // a schedule tuned without life bytes: shrink the LDS queues to fit
    // (results do not depend on the queue capacity)
    const int q = queue_cap_for(c->max_lds, bitset_words, true);
    if (q >= 64) s.queue_cap = q;
  }
  const size_t lds = lds_bytes_for(bitset_words, s.queue_cap, dur);
  if (lds > c->max_lds) return false;
  // workgroups that fit at once (registers, LDS and its granularity)
  const int fit = resident(c, s.threads, s.table_mode != 0, dur, win, lds, gb);
  int per_cu = s.wg_per_cu < fit ? s.wg_per_cu : fit;
  if (per_cu < 1) per_cu = 1;
  int64_t grid = (int64_t)per_cu * c->num_cu;
  if (grid > n_sims) grid = n_sims;
  if (grid < 1) grid = 1;
  *lds_out = lds;
  *grid_out = (int)grid;
  return true;
}

// Kind of batch for the class schedules: 0 at most kWindowMaxParams
// parameter vectors (replicate batches), 1 more vectors with at least 8
// simulations each (GA populations), 2 other batches (one or a few
// simulations per vector: Monte Carlo draws, random-parameter batches).
int batch_kind(int32_t n_params, int32_t n_sims) {
  if (n_params <= kWindowMaxParams) return 0;
  return (int64_t)n_sims >= 8 * (int64_t)n_params ? 1 : 2;
}

// Launch plan for simulations on landscapes of at most max_h rows of
// max_stride bitset words (bitset_words = the largest H * stride) and
// max_cells cells.
fire_status plan_run(fire_ctx *c, int bitset_words, int64_t max_cells, int max_h,
                     int max_stride, int32_t n_params, int32_t n_sims, bool table_allowed,
                     RunPlan *out, bool dur = false, float win_frac = 0.f) {
  fire_schedule s = default_schedule(c, max_cells, bitset_words, n_params, dur, n_sims);
  s.window = -1;  // built-in: decide below
  s.wave = -1;
  if (c->sched_fixed) {
    s = c->sched;
  } else {
    // class schedules are timed on one-step burns; runs with turn-off
    // times keep the built-in choice
    const int b = cells_bucket(max_cells);
    const int kind = batch_kind(n_params, n_sims);
    if (!dur)
      for (const auto &e : c->class_sched)
        if (e.bucket == b && e.kind == kind) s = e.s;
  }
  if (!table_allowed) s.table_mode = 0;
  fire_schedule full = s;
  size_t lds = 0;
  int grid = 0;
  bool gb = false;
  if (!shape_launch(c, full, bitset_words, dur, false, n_sims, &lds, &grid)) {
    // the whole-lattice bitset does not fit LDS: each workgroup keeps its
    // simulation's bitset in global memory and the LDS holds the queues
    gb = true;
    if (!c->sched_fixed) {
      const int tm = full.table_mode;
      full = default_schedule(c, max_cells, 0, n_params, dur, n_sims, false, true);
      full.table_mode = tm;
    }
    if (!shape_launch(c, full, 0, dur, false, n_sims, &lds, &grid, true))
      return fail(c, FIRE_E_UNSUPPORTED,
                  "LDS needed (%zu B: 2x%d queue entries) exceeds the device limit of %zu B",
                  lds_bytes_for(0, full.queue_cap, dur), full.queue_cap, c->max_lds);
    const int64_t cap = std::max<int64_t>(1, kGlobalBitsBudget / (4 * (int64_t)bitset_words));
    if (grid > cap) grid = (int)cap;
  }
  full.window = 0;
  full.wave = 0;
  out->s = full;
  out->wave = false;
  out->dur = dur;
  out->gb = gb;
  out->gb2 = false;
  out->bitset_words = bitset_words;
  out->max_cells = max_cells;
  out->lds = lds;
  out->grid = grid;
  out->win = 0;
  // window: asked for by the schedule, or (built-in) the largest one that
  // keeps as many simulations of the batch resident as any window can, when
  // that is more than whole-lattice bitsets allow and recent window runs on
  // these landscapes rarely had to be repeated
  auto window_words = [&](int side) {
    return std::min(side, max_h) * std::min(side / 32, max_stride);
  };
  auto shape_for = [&](int side, fire_schedule &ws, size_t *wl, int *wg) -> bool {
    const int wbw = window_words(side);
    ws = s.window < 0 ? default_schedule(c, max_cells, wbw, n_params, dur, n_sims, true) : s;
    // no window runs with 1024-thread workgroups: such a run, with a window
    // every fire outgrew, stopped responding on the GPU and the cause is not
    // found; those schedules run over the whole lattice
    if (ws.threads > 512) return false;
    ws.table_mode = full.table_mode;
    return shape_launch(c, ws, wbw, dur, true, n_sims, wl, wg);
  };
  // wavefront-per-simulation plan: only when the schedule asks for it. On
  // the 512x512 calibration batch it took 0.565 ms against 0.42 ms for the
  // workgroup kernel (fronts of a few hundred cells need several 64-lane
  // passes per step), so built-in plans use the workgroup kernel
  const bool want_wave = !dur && s.wave == 1;
  if (want_wave) {
    const int qcap = s.wave == 1 ? s.queue_cap : kWaveQueue;
    auto wave_shape = [&](int side, size_t *wl, int *wg) -> bool {
      const int wbw = side > 0 ? std::min(side, max_h) * std::min(side / 32, max_stride)
                               : bitset_words;
      const size_t lds = simw_lds_bytes(wbw, qcap);
      if (lds > c->max_lds || simw_scratch_bytes(full.table_mode != 0, side > 0) > 0)
        return false;
      const int occ = simw_occupancy(full.table_mode != 0, side > 0, lds);
      if (occ < 1) return false;
      *wl = lds;
      *wg = (int)std::min<int64_t>((int64_t)occ * c->num_cu, n_sims);
      return true;
    };
    int wside = -1;
    size_t wl = 0;
    int wg = 0;
    if (s.wave == 1 && s.window >= 0) {
      wside = s.window;
      if (!wave_shape(wside, &wl, &wg))
        return fail(c, FIRE_E_UNSUPPORTED, "wave schedule (window %d, queue_cap %d) does not fit",
                    s.window, qcap);
    } else {
      // the whole lattice if every simulation of the batch is then
      // resident, else the largest window that makes them resident (or,
      // failing that, keeps the most resident)
      int best_wg = -1;
      size_t l0;
      int g0;
      if (wave_shape(0, &l0, &g0)) {
        wside = 0; wl = l0; wg = g0; best_wg = g0;
      }
      const int top = std::max(max_h, 32 * max_stride);
      for (int side = (top / 32) * 32; side >= 64 && best_wg < std::min(n_sims, c->num_cu * kMaxPerCu);
           side -= 32) {
        if (std::min(side, max_h) * std::min(side / 32, max_stride) >= bitset_words) continue;
        if (wave_shape(side, &l0, &g0) && g0 > best_wg) {
          wside = side; wl = l0; wg = g0; best_wg = g0;
          if (g0 >= n_sims) break;
        }
      }
    }
    if (wside >= 0) {
      fire_schedule ws = full;
      ws.threads = 64;
      ws.queue_cap = qcap;
      ws.wg_per_cu = 1;
      ws.window = wside;
      ws.wave = 1;
      out->gb = false;
      out->gb2 = gb;
      out->s2 = full;
      out->bitset_words2 = bitset_words;
      out->lds2 = lds;
      out->grid2 = std::min(grid, c->num_cu);
      out->s = ws;
      out->wave = true;
      out->bitset_words = wside > 0 ? std::min(wside, max_h) * std::min(wside / 32, max_stride)
                                    : bitset_words;
      out->lds = wl;
      out->grid = wg;
      out->win = wside;
      return FIRE_OK;
    }
  }
  int win = 0;
  if (s.window > 0) {
    win = s.window;
  } else if (s.window < 0 && win_frac <= kWindowRetryMax && n_params <= kWindowMaxParams) {
    // most resident simulations first; among those, the largest window
    // whose LDS queues keep kMinAutoQueue entries (fronts then stay in LDS),
    // else the one with the longest queues
    const int top = std::max(max_h, 32 * max_stride);
    // a window has to beat whole-lattice bitsets in LDS; global-memory
    // bitsets (L2 atomics every step) lose to any window that fits
    int best_conc = gb ? 0 : grid;
    int best_q = 0;
    for (int side = 64; side < top; side += 32) {
      fire_schedule ws;
      size_t wl;
      int wg;
      if (window_words(side) >= bitset_words || !shape_for(side, ws, &wl, &wg)) continue;
      const int q = std::min(ws.queue_cap, kMinAutoQueue);
      if (wg > best_conc || (wg == best_conc && win > 0 && q >= best_q)) {
        best_conc = wg;
        best_q = q;
        win = side;
      }
    }
  }
  if (win <= 0 || window_words(win) >= bitset_words) return FIRE_OK;
  fire_schedule ws;
  size_t wlds = 0;
  int wgrid = 0;
  if (!shape_for(win, ws, &wlds, &wgrid)) return FIRE_OK;
  // window runs only with kernel variants that keep their registers (the
  // spilling variants are slow enough that residency gains nothing)
  if (sim_scratch_bytes(ws.threads, ws.table_mode != 0, dur, true) > 0) return FIRE_OK;
  ws.window = win;
  ws.wave = 0;
  out->gb = false;
  out->gb2 = gb;
  out->s2 = full;
  out->bitset_words2 = bitset_words;
  out->lds2 = lds;
  // the re-run launch usually finds nothing to do: one workgroup per CU
  // keeps its cost small
  out->grid2 = std::min(grid, c->num_cu);
  out->s = ws;
  out->bitset_words = window_words(win);
  out->lds = wlds;
  out->grid = wgrid;
  out->win = win;
  return FIRE_OK;
}

// Spill words of a launch: 2 * ovf_cap entries per workgroup, then (with
// turn-off times) as many remaining-life bytes; a window plan's two
// launches run one after the other and share the area.
int64_t spill_words_one(int64_t max_cells, int queue_cap, int grid, bool dur) {
  int64_t ovf_cap = max_cells - queue_cap;
  if (ovf_cap < 1) ovf_cap = 1;
  const int64_t entries = (int64_t)grid * 2 * ovf_cap;
  return entries + (dur ? (entries + 3) / 4 : 0);
}

int64_t spill_entry_words(const RunPlan &p) {
  // the wavefront kernel keeps its queues in LDS only
  int64_t w = p.wave ? 0 : spill_words_one(p.max_cells, p.s.queue_cap, p.grid, p.dur);
  if (p.win > 0 || p.wave)
    w = std::max(w, spill_words_one(p.max_cells, p.s2.queue_cap, p.grid2, p.dur));
  return w;
}

// Global-memory burn bitsets of the plan's launches (one per workgroup of a
// launch whose whole-lattice bitset does not fit LDS), after the spill
// entries; the two launches of a window plan run one after the other and
// share the area.
int64_t global_bits_words(const RunPlan &p) {
  int64_t w = p.gb ? (int64_t)p.grid * p.bitset_words : 0;
  if (p.gb2) w = std::max(w, (int64_t)p.grid2 * p.bitset_words2);
  return w;
}

int64_t spill_words(const RunPlan &p) { return spill_entry_words(p) + global_bits_words(p); }

// Retry lists of window runs: `words` words (waits for the device when it grows).
fire_status ensure_retry(fire_ctx *c, int64_t words, hipStream_t st) {
  size_t have = c->retry_words * sizeof(uint32_t);
  fire_status r = grow(c, (void **)&c->d_retry, &have, (size_t)words * sizeof(uint32_t), st,
                       "the retry list");
  c->retry_words = have / sizeof(uint32_t);
  return r;
}

// Make the spill area hold `words` entries (waits for the device when it grows).
fire_status ensure_spill(fire_ctx *c, int64_t words, hipStream_t st) {
  size_t have = c->ovf_words * sizeof(uint32_t);
  fire_status r = grow(c, (void **)&c->d_ovf, &have, (size_t)words * sizeof(uint32_t), st,
                       "the frontier spill area");
  c->ovf_words = have / sizeof(uint32_t);
  return r;
}

// Fold finished retry-count copies into the landscapes' re-run shares.
void harvest_stats(fire_ctx *c) {
  for (int i = 0; i < fire_ctx::kStatSlots; ++i) {
    const int l = c->stat_ls[i];
    if (l < 0 || hipEventQuery(c->stat_ev[i]) != hipSuccess) continue;
    (void)hipGetLastError();
    if (l < (int)c->ls.size() && c->ls[l].live && c->stat_n[i] > 0) {
      LandscapeHost &L = c->ls[l];
      const float f = (float)c->h_stat[i] / (float)c->stat_n[i];
      L.win_frac = L.win_obs ? 0.5f * L.win_frac + 0.5f * f : f;
      ++L.win_obs;
    }
    c->stat_ls[i] = -1;
  }
}

// A free statistics slot for a window launch's retry count (not under
// stream capture; -1 when every slot is still in flight). The re-run launch
// writes the count into the slot's host-mapped word and an event recorded
// after it tells when the word is final.
int stat_slot(fire_ctx *c, hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
    (void)hipGetLastError();
    return -1;
  }
  harvest_stats(c);
  for (int i = 0; i < fire_ctx::kStatSlots; ++i)
    if (c->stat_ls[i] < 0) return i;
  return -1;
}

// One persistent launch over n_sims descriptors (or over `order`, a list of
// n_sims indices into sims_dev), with its own work counter and spill area;
// a window plan adds the second launch over the simulations listed in
// `retry` (device, 1 + n_sims words).
SimArgs sim_args(fire_ctx *c, const double *betas_dev, int32_t n_params,
                 const fire_sim *sims_dev, const uint32_t *order, int32_t n_sims,
                 uint64_t seed, const uint32_t *tables, int64_t table_stride, int32_t table_ls,
                 fire_result *out, uint32_t *out_maps, int64_t map_words, int64_t max_cells,
                 int queue_cap, int grid, bool dur, int bitset_words, uint32_t *work,
                 uint32_t *spill) {
  int64_t ovf_cap = max_cells - queue_cap;
  if (ovf_cap < 1) ovf_cap = 1;
  SimArgs a{};
  a.ls = c->d_ls; a.n_ls = (int32_t)c->ls.size();
  a.tg = c->d_tg; a.n_tg = (int32_t)c->tg.size();
  a.betas = betas_dev; a.n_params = n_params;
  a.sims = sims_dev; a.order = order; a.n_sims = n_sims;
  a.key0 = (uint32_t)seed; a.key1 = (uint32_t)(seed >> 32);
  a.tables = tables; a.table_stride = table_stride; a.table_ls = table_ls;
  a.out = out; a.maps = out_maps; a.map_words = map_words;
  a.work = work; a.error_flag = c->d_work + kErrWord;
  a.ovf = spill; a.ovf_cap = ovf_cap;
  a.ovf_life = dur ? reinterpret_cast<uint8_t *>(spill + (int64_t)grid * 2 * ovf_cap) : nullptr;
  a.queue_cap = queue_cap; a.bitset_words = bitset_words;
  a.win = 0; a.retry = nullptr; a.n_dev = nullptr; a.stat_out = nullptr;
  a.times = c->times; a.times_cap = c->times ? c->times_cap : 0;
  return a;
}

fire_status launch_run(fire_ctx *c, const RunPlan &p, const double *betas_dev,
                       int32_t n_params, const fire_sim *sims_dev,
                       const uint32_t *order, int32_t n_sims, uint64_t seed,
                       const uint32_t *tables, int64_t table_stride,
                       int32_t table_ls, fire_result *out, uint32_t *out_maps,
                       int64_t map_words, int counter, uint32_t *spill, uint32_t *retry,
                       hipStream_t st, int stat_lid = -1, uint32_t *work_base = nullptr) {
  // work counters: the context's (or, for the no-allocation entry point,
  // words of its scratch)
  uint32_t *const wb = work_base ? work_base : c->d_work;
  SimArgs a = sim_args(c, betas_dev, n_params, sims_dev, order, n_sims, seed, tables,
                       table_stride, table_ls, out, out_maps, map_words, p.max_cells,
                       p.s.queue_cap, p.grid, p.dur, p.bitset_words, wb + counter, spill);
  const bool two = p.win > 0 || p.wave;  // a second, whole-lattice launch for repeats
  if (two && !retry) return fail(c, FIRE_E_INVALID, "window plan without a retry list");
  uint32_t *const work2 = two ? wb + counter + kMaxClasses : nullptr;
  // the launches' work counters and the retry count, in one launch
  HIP_OR_FAIL(c, launch_zero_words(a.work, work2, two ? retry : nullptr, st));
  uint32_t *const gbits = spill + spill_entry_words(p);
  a.gbits = p.gb ? gbits : nullptr;
  if (two) {
    a.win = p.win;
    a.retry = retry;
  }
  if (p.wave)
    HIP_OR_FAIL(c, launch_simw(a, tables != nullptr, p.grid, p.lds, st));
  else
    HIP_OR_FAIL(c, launch_sim(a, p.s.threads, tables != nullptr, p.dur, p.grid, p.lds, st));
  if (two) {
    SimArgs b = sim_args(c, betas_dev, n_params, sims_dev, retry + 1, n_sims, seed, tables,
                         table_stride, table_ls, out, out_maps, map_words, p.max_cells,
                         p.s2.queue_cap, p.grid2, p.dur, p.bitset_words2, work2, spill);
    b.n_dev = retry;
    b.gbits = p.gb2 ? gbits : nullptr;
    const int slot = stat_lid >= 0 ? stat_slot(c, st) : -1;
    if (slot >= 0) b.stat_out = c->h_stat + slot;
    HIP_OR_FAIL(c, launch_sim(b, p.s2.threads, tables != nullptr, p.dur, p.grid2, p.lds2, st));
    if (slot >= 0) {
      if (hipEventRecord(c->stat_ev[slot], st) == hipSuccess) {
        c->stat_ls[slot] = stat_lid;
        c->stat_n[slot] = n_sims;
      } else {
        (void)hipGetLastError();
      }
    }
  }
  return FIRE_OK;
}

bool finite_all(const float *p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

const char *fire_version(void) { return "1.0.0 gfx950"; }

fire_status fire_ctx_create(int device, fire_ctx **out) {
  if (!out) return FIRE_E_INVALID;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
    return FIRE_E_INVALID;
  fire_ctx *c = new (std::nothrow) fire_ctx();
  if (!c) return FIRE_E_OOM;
  c->device = device;
  hipDeviceProp_t prop;
  if (hipSetDevice(device) != hipSuccess ||
      hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete c;
    return FIRE_E_DEVICE;
  }
  c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                            device) == hipSuccess && lds > 0)
    c->max_lds = (size_t)lds;
  else
    c->max_lds = prop.sharedMemPerBlock;
  // raising the dynamic-LDS ceiling is advisory on this platform
  if (set_sim_lds_limit(c->max_lds) != hipSuccess) (void)hipGetLastError();
  // the no-allocation entry point's scratch on this device (device current)
  if (noalloc_scratch(&c->noalloc) != hipSuccess) {
    delete c;
    return FIRE_E_DEVICE;
  }
  bool ev_ok = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; i < kMaxClasses && ev_ok; ++i)
    ev_ok = hipEventCreateWithFlags(&c->join_ev[i], hipEventDisableTiming) == hipSuccess;
  for (int i = 0; i < fire_ctx::kStatSlots && ev_ok; ++i)
    ev_ok = hipEventCreateWithFlags(&c->stat_ev[i], hipEventDisableTiming) == hipSuccess;
  if (!ev_ok || hipMalloc(&c->d_work, kWorkWords * sizeof(uint32_t)) != hipSuccess ||
      hipMemset(c->d_work, 0, kWorkWords * sizeof(uint32_t)) != hipSuccess ||
      hipEventCreateWithFlags(&c->stage_done, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc((void **)&c->h_stat, sizeof(uint32_t) * fire_ctx::kStatSlots) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    fire_ctx_destroy(c);
    return FIRE_E_DEVICE;
  }
  *out = c;
  return FIRE_OK;
}

void fire_ctx_destroy(fire_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (auto &L : c->ls) {
    if (L.rec) (void)hipFree(L.rec);
    if (L.cov) (void)hipFree(L.cov);
    if (L.blocked) (void)hipFree(L.blocked);
    if (L.burn_steps) (void)hipFree(L.burn_steps);
  }
  for (auto &T : c->tg)
    if (T.bits) (void)hipFree(T.bits);
  if (c->d_ls) (void)hipFree(c->d_ls);
  if (c->d_tg) (void)hipFree(c->d_tg);
  if (c->d_work) (void)hipFree(c->d_work);
  if (c->d_ovf) (void)hipFree(c->d_ovf);
  if (c->d_retry) (void)hipFree(c->d_retry);
  if (c->h_stat) (void)hipHostFree(c->h_stat);
  for (int i = 0; i < fire_ctx::kStatSlots; ++i)
    if (c->stat_ev[i]) (void)hipEventDestroy(c->stat_ev[i]);
  if (c->d_tables) (void)hipFree(c->d_tables);
  for (void *p : c->retired) (void)hipFree(p);
  if (c->d_stage) (void)hipFree(c->d_stage);
  if (c->h_stage) (void)hipHostFree(c->h_stage);
  if (c->d_ga) (void)hipFree(c->d_ga);
  if (c->d_dense) (void)hipFree(c->d_dense);
  if (c->h_dense) (void)hipHostFree(c->h_dense);
  if (c->stage_done) (void)hipEventDestroy(c->stage_done);
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  for (int i = 0; i < kMaxClasses; ++i)
    if (c->join_ev[i]) (void)hipEventDestroy(c->join_ev[i]);
  for (int i = 0; i < kMaxClasses - 1; ++i)
    if (c->side[i]) (void)hipStreamDestroy(c->side[i]);
  delete c;
}

const char *fire_last_error(const fire_ctx *c) {
  return c ? c->err.c_str() : "null context";
}

fire_status fire_set_sim_timing(fire_ctx *c, uint64_t *times_dev, int64_t capacity) {
  if (!c) return FIRE_E_INVALID;
  if (times_dev && capacity < 1)
    return fail(c, FIRE_E_INVALID, "timing buffer capacity %lld", (long long)capacity);
  if (times_dev && ((uintptr_t)times_dev) % 8 != 0)
    return fail(c, FIRE_E_INVALID, "timing buffer must be 8-byte aligned");
  c->times = times_dev;
  c->times_cap = times_dev ? capacity : 0;
  return FIRE_OK;
}

fire_status fire_sync(fire_ctx *c, void *stream) {
  if (!c) return FIRE_E_INVALID;
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, hipStreamSynchronize((hipStream_t)stream));
  uint32_t flag = 0;
  HIP_OR_FAIL(c, hipMemcpy(&flag, c->d_work + kErrWord, sizeof flag, hipMemcpyDeviceToHost));
  if (flag) {
    uint32_t zero = 0;
    HIP_OR_FAIL(c, hipMemcpy(c->d_work + kErrWord, &zero, sizeof zero, hipMemcpyHostToDevice));
    return fail(c, FIRE_E_INVALID,
                "a simulation descriptor was rejected on the device "
                "(bad id, ignition outside the lattice, map or table mismatch)");
  }
  return FIRE_OK;
}

fire_status fire_landscape_load(fire_ctx *c, const fire_landscape_desc *d,
                                int32_t *out_id) {
  if (!c) return FIRE_E_INVALID;
  if (!d || !out_id) return fail(c, FIRE_E_INVALID, "null argument");
  if (d->width < 1 || d->height < 1 || d->width > kMaxDim || d->height > kMaxDim)
    return fail(c, FIRE_E_INVALID, "lattice %dx%d outside [1, %d]", d->width,
                d->height, kMaxDim);
  if (!d->veg || !d->elev_m || !d->slope_deg || !d->aspect_deg || !d->wind_to_deg)
    return fail(c, FIRE_E_INVALID, "null landscape layer");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  const int W = d->width, H = d->height, stride = (W + 31) / 32;
  const int64_t n = (int64_t)W * H;
  // host copies for validation (and staging when the input is on the host)
  std::vector<uint8_t> veg(n);
  std::vector<float> layers[4];
  const float *src[4] = {d->elev_m, d->slope_deg, d->aspect_deg, d->wind_to_deg};
  hipMemcpyKind kind = d->on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
  HIP_OR_FAIL(c, hipMemcpy(veg.data(), d->veg, n, kind));
  for (int k = 0; k < 4; ++k) {
    layers[k].resize(n);
    HIP_OR_FAIL(c, hipMemcpy(layers[k].data(), src[k], n * sizeof(float), kind));
    if (!finite_all(layers[k].data(), n))
      return fail(c, FIRE_E_INVALID, "non-finite value in landscape layer %d", k);
  }
  LandscapeHost L;
  L.W = W; L.H = H; L.stride = stride;
  L.forest = d->forest_class ? d->forest_class : 1;
  {
    // about half of a cell's edges lead uphill, where sigma is slope/100
    int64_t nb = 0, nf = 0;
    double sp = 0.0, ss = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      if (veg[i] == 0) continue;
      ++nb;
      nf += veg[i] == L.forest;
      if (layers[1][i] > 5.0f) sp += std::cos(((double)layers[2][i] - 315.0) * kPi / 180.0);
      ss += 0.5 * (double)layers[1][i] / 100.0;
    }
    L.burnable = nb;
    if (nb > 0) {
      L.mean_forest = (double)nf / (double)nb;
      L.mean_psi = sp / (double)nb;
      L.mean_sigma = ss / (double)nb;
    }
  }
  uint8_t *d_veg = nullptr;
  float *d_f = nullptr;
  hipError_t e = hipMalloc(&L.rec, sizeof(uint4) * n);
  if (e == hipSuccess) e = hipMalloc(&L.cov, sizeof(double) * 10 * n);
  if (e == hipSuccess) e = hipMalloc(&L.blocked, sizeof(uint32_t) * H * stride);
  if (e == hipSuccess) e = hipMalloc(&d_veg, n);
  if (e == hipSuccess) e = hipMalloc(&d_f, sizeof(float) * 4 * n);
  if (e == hipSuccess) e = hipMemcpy(d_veg, veg.data(), n, hipMemcpyHostToDevice);
  for (int k = 0; k < 4 && e == hipSuccess; ++k)
    e = hipMemcpy(d_f + k * n, layers[k].data(), n * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = launch_preprocess(d_veg, d_f, d_f + n, d_f + 2 * n, d_f + 3 * n, W, H,
                          stride, L.rec, L.cov, L.cov + 2 * n, L.blocked, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (d_veg) (void)hipFree(d_veg);
  if (d_f) (void)hipFree(d_f);
  if (e != hipSuccess) {
    if (L.rec) (void)hipFree(L.rec);
    if (L.cov) (void)hipFree(L.cov);
    if (L.blocked) (void)hipFree(L.blocked);
    if (L.burn_steps) (void)hipFree(L.burn_steps);
    return fail(c, e == hipErrorOutOfMemory ? FIRE_E_OOM : FIRE_E_DEVICE,
                "landscape upload: %s", hipGetErrorString(e));
  }
  L.live = true;
  int id = -1;
  for (size_t i = 0; i < c->ls.size(); ++i)
    if (!c->ls[i].live) { id = (int)i; break; }
  if (id < 0) { id = (int)c->ls.size(); c->ls.push_back(L); }
  else c->ls[id] = L;
  fire_status st = sync_tables(c);
  if (st != FIRE_OK) return st;
  *out_id = id;
  return FIRE_OK;
}

fire_status fire_landscape_free(fire_ctx *c, int32_t id) {
  if (!c) return FIRE_E_INVALID;
  if (id < 0 || id >= (int)c->ls.size() || !c->ls[id].live)
    return fail(c, FIRE_E_INVALID, "unknown landscape id %d", id);
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, hipDeviceSynchronize());
  LandscapeHost &L = c->ls[id];
  (void)hipFree(L.rec); (void)hipFree(L.cov); (void)hipFree(L.blocked);
  if (L.burn_steps) (void)hipFree(L.burn_steps);
  L = LandscapeHost();
  for (auto &T : c->tg)
    if (T.live && T.landscape_id == id) {
      (void)hipFree(T.bits);
      T = TargetHost();
    }
  return sync_tables(c);
}

fire_status fire_landscape_set_burn_steps(fire_ctx *c, int32_t id, const uint8_t *steps) {
  if (!c) return FIRE_E_INVALID;
  if (id < 0 || id >= (int)c->ls.size() || !c->ls[id].live)
    return fail(c, FIRE_E_INVALID, "unknown landscape id %d", id);
  bool all_one = true;
  if (steps)
    for (int v = 1; v < 256; ++v) {
      if (steps[v] == 0) return fail(c, FIRE_E_INVALID, "turn-off time 0 for vegetation %d", v);
      all_one = all_one && steps[v] == 1;
    }
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, hipDeviceSynchronize());
  LandscapeHost &L = c->ls[id];
  L.win_frac = 0.f;  // fire sizes change with the turn-off times
  L.win_obs = 0;
  const int64_t n = (int64_t)L.W * L.H;
  if (!steps || all_one) {
    if (L.burn_steps) HIP_OR_FAIL(c, hipFree(L.burn_steps));
    L.burn_steps = nullptr;
    HIP_OR_FAIL(c, launch_set_life(L.rec, n, nullptr, nullptr));
    HIP_OR_FAIL(c, hipDeviceSynchronize());
    return sync_tables(c);
  }
  if (!L.burn_steps) HIP_OR_FAIL(c, hipMalloc(&L.burn_steps, 256));
  uint8_t h[256];
  std::memcpy(h, steps, 256);
  h[0] = 1;
  HIP_OR_FAIL(c, hipMemcpy(L.burn_steps, h, 256, hipMemcpyHostToDevice));
  // each record word also carries its cell's turn-off time
  HIP_OR_FAIL(c, launch_set_life(L.rec, n, L.burn_steps, nullptr));
  HIP_OR_FAIL(c, hipDeviceSynchronize());
  return sync_tables(c);
}

fire_status fire_target_load(fire_ctx *c, int32_t lid, const uint32_t *bits,
                             int32_t *out_id) {
  if (!c) return FIRE_E_INVALID;
  if (!bits || !out_id) return fail(c, FIRE_E_INVALID, "null argument");
  if (lid < 0 || lid >= (int)c->ls.size() || !c->ls[lid].live)
    return fail(c, FIRE_E_INVALID, "unknown landscape id %d", lid);
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  const LandscapeHost &L = c->ls[lid];
  const int64_t nw = (int64_t)L.H * L.stride;
  std::vector<uint32_t> b(bits, bits + nw);
  const uint32_t tail = (L.W % 32) ? ((1u << (L.W % 32)) - 1u) : 0xFFFFFFFFu;
  uint64_t count = 0;
  for (int y = 0; y < L.H; ++y) {
    b[(int64_t)y * L.stride + L.stride - 1] &= tail;  // clear padding bits
    for (int w = 0; w < L.stride; ++w) count += __builtin_popcount(b[(int64_t)y * L.stride + w]);
  }
  if (count == 0) return fail(c, FIRE_E_INVALID, "empty reference map (Eq. 2 divides by |A|)");
  TargetHost T;
  T.landscape_id = lid;
  T.n_ref = (uint32_t)count;
  HIP_OR_FAIL(c, hipMalloc(&T.bits, sizeof(uint32_t) * nw));
  hipError_t e = hipMemcpy(T.bits, b.data(), sizeof(uint32_t) * nw, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(T.bits);
    return fail(c, FIRE_E_DEVICE, "target upload: %s", hipGetErrorString(e));
  }
  T.live = true;
  int id = -1;
  for (size_t i = 0; i < c->tg.size(); ++i)
    if (!c->tg[i].live) { id = (int)i; break; }
  if (id < 0) { id = (int)c->tg.size(); c->tg.push_back(T); }
  else c->tg[id] = T;
  fire_status st = sync_tables(c);
  if (st != FIRE_OK) return st;
  *out_id = id;
  return FIRE_OK;
}

fire_status fire_target_free(fire_ctx *c, int32_t id) {
  if (!c) return FIRE_E_INVALID;
  if (id < 0 || id >= (int)c->tg.size() || !c->tg[id].live)
    return fail(c, FIRE_E_INVALID, "unknown target id %d", id);
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, hipDeviceSynchronize());
  (void)hipFree(c->tg[id].bits);
  c->tg[id] = TargetHost();
  return sync_tables(c);
}

fire_status fire_thresholds(fire_ctx *c, int32_t lid, const double beta[5],
                            uint32_t *out_T, void *stream) {
  if (!c) return FIRE_E_INVALID;
  if (!beta || !out_T) return fail(c, FIRE_E_INVALID, "null argument");
  if (lid < 0 || lid >= (int)c->ls.size() || !c->ls[lid].live)
    return fail(c, FIRE_E_INVALID, "unknown landscape id %d", lid);
  for (int i = 0; i < 5; ++i)
    if (!std::isfinite(beta[i])) return fail(c, FIRE_E_INVALID, "non-finite beta");
  if (((uintptr_t)out_T) % 16 != 0)
    return fail(c, FIRE_E_INVALID, "out_T must be 16-byte aligned");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  // parameters staged through the context's small device buffer
  size_t have = c->ga_bytes;
  HIP_OR_FAIL(c, hipStreamSynchronize(st));
  HIP_OR_FAIL(c, ensure((void **)&c->d_ga, &have, 4096));
  c->ga_bytes = have;
  HIP_OR_FAIL(c, hipMemcpy(c->d_ga, beta, 5 * sizeof(double), hipMemcpyHostToDevice));
  const LandscapeHost &L = c->ls[lid];
  HIP_OR_FAIL(c, launch_thresholds(c->d_ls + lid, L.W, L.H, c->d_ga, L.forest, out_T, st));
  return FIRE_OK;
}

fire_status fire_thresholds_dev(fire_ctx *c, int32_t lid, const double *betas_dev,
                                int32_t n_params, uint32_t *out_T, void *stream) {
  if (!c) return FIRE_E_INVALID;
  if (!betas_dev || !out_T || n_params < 1)
    return fail(c, FIRE_E_INVALID, "null argument or n_params < 1");
  if (lid < 0 || lid >= (int)c->ls.size() || !c->ls[lid].live)
    return fail(c, FIRE_E_INVALID, "unknown landscape id %d", lid);
  if (((uintptr_t)out_T) % 16 != 0)
    return fail(c, FIRE_E_INVALID, "out_T must be 16-byte aligned");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  const LandscapeHost &L = c->ls[lid];
  HIP_OR_FAIL(c, launch_thresholds_multi(c->d_ls + lid, L.W, L.H, betas_dev, n_params, L.forest,
                                         out_T, (int64_t)L.W * L.H * 8, (hipStream_t)stream));
  return FIRE_OK;
}

static fire_status check_sims_host(fire_ctx *c, const fire_sim *sims, int32_t n,
                                   int32_t n_params, int *bitset_words,
                                   int64_t *max_cells, int *one_ls,
                                   int64_t map_words, bool maps) {
  int bw = 0;
  int64_t mc = 1;
  int ls_seen = -2;
  for (int32_t i = 0; i < n; ++i) {
    const fire_sim &s = sims[i];
    if (s.landscape_id < 0 || s.landscape_id >= (int)c->ls.size() ||
        !c->ls[s.landscape_id].live)
      return fail(c, FIRE_E_INVALID, "sim %d: unknown landscape id %d", i, s.landscape_id);
    const LandscapeHost &L = c->ls[s.landscape_id];
    if (s.target_id != -1) {
      if (s.target_id < 0 || s.target_id >= (int)c->tg.size() || !c->tg[s.target_id].live)
        return fail(c, FIRE_E_INVALID, "sim %d: unknown target id %d", i, s.target_id);
      if (c->tg[s.target_id].landscape_id != s.landscape_id)
        return fail(c, FIRE_E_INVALID, "sim %d: target %d belongs to another landscape", i,
                    s.target_id);
    }
    if (s.ign_x < 0 || s.ign_x >= L.W || s.ign_y < 0 || s.ign_y >= L.H)
      return fail(c, FIRE_E_INVALID, "sim %d: ignition (%d, %d) outside the %dx%d lattice", i,
                  s.ign_x, s.ign_y, L.W, L.H);
    if (s.param_index >= (uint32_t)n_params)
      return fail(c, FIRE_E_INVALID, "sim %d: param_index %u >= n_params %d", i,
                  s.param_index, n_params);
    const int words = L.H * L.stride;
    if (maps && words > map_words)
      return fail(c, FIRE_E_INVALID, "sim %d: map needs %d words > map_words %lld", i, words,
                  (long long)map_words);
    if (words > bw) bw = words;
    if ((int64_t)L.W * L.H > mc) mc = (int64_t)L.W * L.H;
    if (ls_seen == -2) ls_seen = s.landscape_id;
    else if (ls_seen != s.landscape_id) ls_seen = -1;
  }
  *bitset_words = bw;
  *max_cells = mc;
  *one_ls = ls_seen;
  return FIRE_OK;
}

// Table-mode thresholds: one table per parameter vector into context
// scratch, computed on the stream right before the simulations.
// Room for n_params threshold tables of landscape lid (waits for the device
// when it grows).
static fire_status ensure_tables(fire_ctx *c, int lid, int32_t n_params, hipStream_t st) {
  const LandscapeHost &L = c->ls[lid];
  const int64_t per = (int64_t)L.W * L.H * 8;
  const size_t need = sizeof(uint32_t) * (size_t)per * n_params;
  size_t have = c->tables_words * sizeof(uint32_t);
  fire_status r = grow(c, (void **)&c->d_tables, &have, need, st, "the threshold tables");
  c->tables_words = have / sizeof(uint32_t);
  return r;
}

// Table-mode thresholds: one table per parameter vector into context
// scratch, computed on the stream right before the simulations.
static fire_status build_tables(fire_ctx *c, int lid, const double *betas_dev,
                                int32_t n_params, hipStream_t st,
                                const uint32_t **tables, int64_t *stride) {
  fire_status es = ensure_tables(c, lid, n_params, st);
  if (es != FIRE_OK) return es;
  const LandscapeHost &L = c->ls[lid];
  const int64_t per = (int64_t)L.W * L.H * 8;
  HIP_OR_FAIL(c, launch_thresholds_multi(c->d_ls + lid, L.W, L.H, betas_dev, n_params, L.forest,
                                         c->d_tables, per, st));
  *tables = c->d_tables;
  *stride = per;
  return FIRE_OK;
}

// Expected fire size of a simulation on landscape L under parameters b, the
// key of the longest-expected-first order: burnable cells x the Eq. 1
// probability averaged over the forest and the other burnable cells, each
// at the landscape's mean aspect and slope terms (the wind term averages out
// over the eight directions).
static double expected_size(const LandscapeHost &L, const double *b) {
  const double x = b[0] + b[2] * L.mean_psi + b[4] * L.mean_sigma;
  const double p = L.mean_forest / (1.0 + std::exp(-(x + b[1]))) +
                   (1.0 - L.mean_forest) / (1.0 + std::exp(-x));
  return (double)L.burnable * p;
}

fire_status fire_order_sims(fire_ctx *c, const double *betas, int32_t n_params,
                            const fire_sim *sims, int32_t n_sims, int32_t *out_order) {
  if (!c) return FIRE_E_INVALID;
  if (n_sims < 0 || n_params < 1 || !betas || (n_sims > 0 && (!sims || !out_order)))
    return fail(c, FIRE_E_INVALID, "bad sizes or null pointers");
  for (int64_t i = 0; i < (int64_t)n_params * 5; ++i)
    if (!std::isfinite(betas[i])) return fail(c, FIRE_E_INVALID, "non-finite beta %lld", (long long)i);
  if (n_sims == 0) return FIRE_OK;
  int bw = 0, one_ls = -1;
  int64_t mc = 1;
  fire_status st0 = check_sims_host(c, sims, n_sims, n_params, &bw, &mc, &one_ls, 0, false);
  if (st0 != FIRE_OK) return st0;
  std::vector<std::pair<double, int32_t>> key(n_sims);
  for (int32_t i = 0; i < n_sims; ++i)
    key[i] = {-expected_size(c->ls[sims[i].landscape_id], betas + 5 * (size_t)sims[i].param_index),
              i};
  std::stable_sort(key.begin(), key.end(),
                   [](const std::pair<double, int32_t> &u, const std::pair<double, int32_t> &v) {
                     return u.first < v.first;
                   });
  for (int32_t i = 0; i < n_sims; ++i) out_order[i] = key[i].second;
  return FIRE_OK;
}

fire_status fire_run(fire_ctx *c, const double *betas, int32_t n_params,
                     const fire_sim *sims, int32_t n_sims, uint64_t seed,
                     const uint32_t *override_T, fire_result *out,
                     uint32_t *out_maps, int64_t map_words, void *stream) {
  if (!c) return FIRE_E_INVALID;
  if (n_sims < 0 || n_params < 1 || !betas || (n_sims > 0 && (!sims || !out)))
    return fail(c, FIRE_E_INVALID, "bad sizes or null pointers");
  for (int64_t i = 0; i < (int64_t)n_params * 5; ++i)
    if (!std::isfinite(betas[i])) return fail(c, FIRE_E_INVALID, "non-finite beta %lld", (long long)i);
  if (n_sims == 0) return FIRE_OK;
  int bw = 0, one_ls = -1;
  int64_t mc = 1;
  fire_status st0 = check_sims_host(c, sims, n_sims, n_params, &bw, &mc, &one_ls, map_words,
                                    out_maps != nullptr);
  if (st0 != FIRE_OK) return st0;
  if (override_T && one_ls < 0)
    return fail(c, FIRE_E_INVALID, "thresholds_override needs every sim on one landscape");
  if (override_T && ((uintptr_t)override_T) % 16 != 0)
    return fail(c, FIRE_E_INVALID, "thresholds_override must be 16-byte aligned");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  if (stream_capturing(st))
    return fail(c, FIRE_E_UNSUPPORTED,
                "fire_run stages host descriptors through pinned memory, which a captured "
                "graph would read at replay time; use fire_run_dev under stream capture");

  // With several parameter vectors the simulations start in decreasing
  // order of expected fire size (longest processing time first), so that
  // the longest fires do not start last and set the launch's tail
  // (expected_size; averaging the logistic per vegetation class, not taking
  // it at the mean covariates, keeps fires that spread through forest alone
  // ranked with the large fires). Such a batch on several landscapes runs as
  // one launch (size classes would run one after another: each persistent
  // launch fills the GPU). Results do not depend on the order.
  const bool lpt = n_params > 1;
  // Size classes: simulations grouped by landscape (by size when there are
  // more landscapes than concurrent launches), each class run by its own
  // persistent launch with LDS sized for that class.
  std::vector<int> cls_of_ls(c->ls.size(), -1);
  std::vector<int64_t> cls_cells;
  std::vector<int> cls_words, cls_h, cls_stride;
  std::vector<char> cls_dur;
  std::vector<int> ls_ids;
  for (int32_t i = 0; i < n_sims; ++i) {
    const int l = sims[i].landscape_id;
    if (cls_of_ls[l] < 0) { cls_of_ls[l] = -2; ls_ids.push_back(l); }
  }
  const bool per_ls = (int)ls_ids.size() <= kMaxClasses && !(lpt && ls_ids.size() > 1);
  if (per_ls) {
    for (int l : ls_ids) {
      cls_of_ls[l] = (int)cls_cells.size();
      cls_cells.push_back((int64_t)c->ls[l].W * c->ls[l].H);
      cls_words.push_back(c->ls[l].H * c->ls[l].stride);
      cls_h.push_back(c->ls[l].H);
      cls_stride.push_back(c->ls[l].stride);
      cls_dur.push_back(c->ls[l].burn_steps != nullptr);
    }
  } else {
    bool any = false;
    int mh = 1, ms = 1;
    for (int l : ls_ids) {
      cls_of_ls[l] = 0;
      any = any || c->ls[l].burn_steps != nullptr;
      mh = std::max(mh, c->ls[l].H);
      ms = std::max(ms, c->ls[l].stride);
    }
    cls_cells.push_back(mc);
    cls_words.push_back(bw);
    cls_h.push_back(mh);
    cls_stride.push_back(ms);
    cls_dur.push_back(any);
  }
  const int n_cls = (int)cls_cells.size();
  std::vector<std::vector<uint32_t>> members(n_cls);
  for (int32_t i = 0; i < n_sims; ++i)
    members[cls_of_ls[sims[i].landscape_id]].push_back((uint32_t)i);
  if (lpt) {
    std::vector<std::pair<double, uint32_t>> key;
    for (auto &m : members) {
      key.resize(m.size());
      for (size_t j = 0; j < m.size(); ++j) {
        const fire_sim &sd = sims[m[j]];
        key[j] = {-expected_size(c->ls[sd.landscape_id], betas + 5 * (size_t)sd.param_index),
                  m[j]};
      }
      std::stable_sort(key.begin(), key.end(),
                       [](const std::pair<double, uint32_t> &u,
                          const std::pair<double, uint32_t> &v) { return u.first < v.first; });
      for (size_t j = 0; j < m.size(); ++j) m[j] = key[j].second;
    }
  }
  std::vector<RunPlan> plans(n_cls);
  int64_t spill_total = 0;
  harvest_stats(c);
  std::vector<float> cls_frac(n_cls, 0.f);
  std::vector<int> cls_lid(n_cls, -1);
  for (int l : ls_ids) {
    const int k = cls_of_ls[l];
    cls_frac[k] = std::max(cls_frac[k], c->ls[l].win_frac);
    cls_lid[k] = per_ls ? l : -1;
  }
  for (int k = 0; k < n_cls; ++k) {
    fire_status ps = plan_run(c, cls_words[k], cls_cells[k], cls_h[k], cls_stride[k], n_params,
                              (int32_t)members[k].size(), one_ls >= 0, &plans[k],
                              cls_dur[k] != 0, cls_frac[k]);
    if (ps != FIRE_OK) return ps;
    spill_total += spill_words(plans[k]);
  }
  fire_status ss = ensure_spill(c, spill_total, st);
  if (ss != FIRE_OK) return ss;
  // retry lists: class k at retry_start[k], 1 + |class| words
  std::vector<int64_t> retry_start(n_cls, 0);
  int64_t retry_total = 0;
  for (int k = 0; k < n_cls; ++k) {
    retry_start[k] = retry_total;
    retry_total += 1 + (int64_t)members[k].size();
  }
  fire_status rs = ensure_retry(c, retry_total, st);
  if (rs != FIRE_OK) return rs;

  // stage descriptors, parameters and class member lists
  const size_t bbytes = sizeof(double) * 5 * (size_t)n_params;
  const size_t boff = (sizeof(fire_sim) * (size_t)n_sims + 255) / 256 * 256;
  const size_t ooff = (boff + bbytes + 255) / 256 * 256;
  const size_t need = ooff + sizeof(uint32_t) * (size_t)n_sims;
  if (c->stage_pending) {
    HIP_OR_FAIL(c, hipEventSynchronize(c->stage_done));
    c->stage_pending = false;
  }
  if (need > c->stage_bytes) {
    HIP_OR_FAIL(c, hipDeviceSynchronize());
    if (c->h_stage) HIP_OR_FAIL(c, hipHostFree(c->h_stage));
    if (c->d_stage) HIP_OR_FAIL(c, hipFree(c->d_stage));
    c->h_stage = c->d_stage = nullptr;
    c->stage_bytes = 0;
    size_t sz = need * 2;
    HIP_OR_FAIL(c, hipHostMalloc(&c->h_stage, sz, hipHostMallocDefault));
    HIP_OR_FAIL(c, hipMalloc(&c->d_stage, sz));
    c->stage_bytes = sz;
  }
  memcpy(c->h_stage, sims, sizeof(fire_sim) * (size_t)n_sims);
  memcpy((char *)c->h_stage + boff, betas, bbytes);
  {
    uint32_t *o = (uint32_t *)((char *)c->h_stage + ooff);
    for (int k = 0; k < n_cls; ++k)
      for (uint32_t v : members[k]) *o++ = v;
  }
  HIP_OR_FAIL(c, hipMemcpyAsync(c->d_stage, c->h_stage, need, hipMemcpyHostToDevice, st));
  HIP_OR_FAIL(c, hipEventRecord(c->stage_done, st));
  c->stage_pending = true;
  const fire_sim *d_sims = (const fire_sim *)c->d_stage;
  const double *d_betas = (const double *)((char *)c->d_stage + boff);
  const uint32_t *d_order = (const uint32_t *)((char *)c->d_stage + ooff);

  const uint32_t *tables = override_T;
  int64_t tstride = 0;
  if (override_T) {
    tstride = mc * 8;
  } else if (n_cls == 1 && one_ls >= 0 && plans[0].s.table_mode) {
    fire_status tsx = build_tables(c, one_ls, d_betas, n_params, st, &tables, &tstride);
    if (tsx != FIRE_OK) return tsx;
  }
  if (n_cls == 1)
    return launch_run(c, plans[0], d_betas, n_params, d_sims, lpt ? d_order : nullptr, n_sims,
                      seed, tables,
                      tstride, tables ? one_ls : -1, out, out_maps, map_words, 0, c->d_ovf,
                      c->d_retry, st, cls_lid[0]);

  // fork the classes onto side streams, join back to the caller's stream
  for (int k = 0; k < n_cls - 1; ++k)
    if (!c->side[k])
      HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->side[k], hipStreamNonBlocking));
  HIP_OR_FAIL(c, hipEventRecord(c->fork_ev, st));
  int64_t spill_off = 0, order_off = 0;
  // largest class first, on the caller's stream
  std::vector<int> by_size(n_cls);
  for (int k = 0; k < n_cls; ++k) by_size[k] = k;
  std::sort(by_size.begin(), by_size.end(),
            [&](int x, int y) { return cls_cells[x] > cls_cells[y]; });
  std::vector<int64_t> order_start(n_cls, 0);
  for (int k = 1; k < n_cls; ++k) order_start[k] = order_start[k - 1] + (int64_t)members[k - 1].size();
  for (int r = 0; r < n_cls; ++r) {
    const int k = by_size[r];
    hipStream_t ks = r == 0 ? st : c->side[r - 1];
    if (r > 0) HIP_OR_FAIL(c, hipStreamWaitEvent(ks, c->fork_ev, 0));
    order_off = order_start[k];
    fire_status ls_ = launch_run(c, plans[k], d_betas, n_params, d_sims, d_order + order_off,
                                 (int32_t)members[k].size(), seed, nullptr, 0, -1, out,
                                 out_maps, map_words, k, c->d_ovf + spill_off,
                                 c->d_retry + retry_start[k], ks, cls_lid[k]);
    if (ls_ != FIRE_OK) return ls_;
    spill_off += spill_words(plans[k]);
    if (r > 0) {
      HIP_OR_FAIL(c, hipEventRecord(c->join_ev[r], ks));
      HIP_OR_FAIL(c, hipStreamWaitEvent(st, c->join_ev[r], 0));
    }
  }
  return FIRE_OK;
}

static fire_status run_dev_impl(fire_ctx *c, const double *betas_dev, int32_t n_params,
                                const fire_sim *sims_dev, int32_t n_sims, uint64_t seed,
                                const uint32_t *override_T, fire_result *out,
                                uint32_t *out_maps, int64_t map_words, void *stream,
                                bool noalloc) {
  if (!c) return FIRE_E_INVALID;
  if (n_sims < 0 || n_params < 1 || !betas_dev || (n_sims > 0 && (!sims_dev || !out)))
    return fail(c, FIRE_E_INVALID, "bad sizes or null pointers");
  if (n_sims == 0) return FIRE_OK;
  // sized for every loaded landscape (the descriptors stay on the device)
  int bw = 0, nlive = 0, lid = -1, mh = 1, ms = 1;
  int64_t mc = 1;
  bool any_dur = false;
  float frac = 0.f;
  // under capture: no event queries, no buffer growth; every buffer the
  // graph records stays allocated for the context's lifetime
  const bool capturing = stream_capturing((hipStream_t)stream);
  if (capturing) c->captured = true;
  else harvest_stats(c);
  for (size_t i = 0; i < c->ls.size(); ++i) {
    const LandscapeHost &L = c->ls[i];
    if (!L.live) continue;
    ++nlive;
    lid = (int)i;
    any_dur = any_dur || L.burn_steps != nullptr;
    mh = std::max(mh, L.H);
    ms = std::max(ms, L.stride);
    frac = std::max(frac, L.win_frac);
    if (L.H * L.stride > bw) bw = L.H * L.stride;
    if ((int64_t)L.W * L.H > mc) mc = (int64_t)L.W * L.H;
  }
  if (nlive == 0) return fail(c, FIRE_E_INVALID, "no landscape loaded");
  if (override_T && nlive != 1)
    return fail(c, FIRE_E_INVALID, "thresholds_override needs exactly one loaded landscape");
  if (override_T && ((uintptr_t)override_T) % 16 != 0)
    return fail(c, FIRE_E_INVALID, "thresholds_override must be 16-byte aligned");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  RunPlan plan;
  // without allocation, thresholds come from the caller's tables or are
  // evaluated per trial (no context tables)
  fire_status ps = plan_run(c, bw, mc, mh, ms, n_params, n_sims,
                            nlive == 1 && (!noalloc || override_T != nullptr), &plan, any_dur,
                            frac);
  if (ps != FIRE_OK) return ps;
  uint32_t *spill = c->d_ovf, *retry = c->d_retry, *work = nullptr;
  if (noalloc && (plan.gb || plan.gb2))
    return fail(c, FIRE_E_INVALID,
                "the no-allocation entry point keeps burn bitsets in LDS; a lattice of %d "
                "bitset words needs them in global memory", bw);
  if (noalloc) {
    // scratch words: [0, 32) work counters, [64, 65 + n_sims) re-run list,
    // then the spill area of the launches, whose grids shrink to fit it
    const int64_t cap = (int64_t)kNoAllocScratchWords;
    const int64_t spill_off = (65 + (int64_t)n_sims + 63) / 64 * 64;
    const int64_t avail = cap - spill_off;
    auto per_wg = [&](int qcap) {
      const int64_t ovf = std::max<int64_t>(1, plan.max_cells - qcap);
      return 2 * ovf + (plan.dur ? (2 * ovf + 3) / 4 : 0);
    };
    const int64_t need1 = plan.wave ? 0 : per_wg(plan.s.queue_cap);
    const int64_t need2 = (plan.win > 0 || plan.wave) ? per_wg(plan.s2.queue_cap) : 0;
    if (avail < std::max(need1, need2))
      return fail(c, FIRE_E_INVALID,
                  "the no-allocation scratch holds %lld words; %d simulations on landscapes of "
                  "up to %lld cells need at least %lld",
                  (long long)cap, n_sims, (long long)plan.max_cells,
                  (long long)(spill_off + std::max(need1, need2)));
    if (need1 > 0) plan.grid = (int)std::min<int64_t>(plan.grid, avail / need1);
    if (need2 > 0) plan.grid2 = (int)std::min<int64_t>(plan.grid2, avail / need2);
    work = c->noalloc;
    retry = c->noalloc + 64;
    spill = c->noalloc + spill_off;
  } else {
    fire_status ss = ensure_spill(c, spill_words(plan), st);
    if (ss != FIRE_OK) return ss;
    fire_status rs = ensure_retry(c, 1 + (int64_t)n_sims, st);
    if (rs != FIRE_OK) return rs;
    spill = c->d_ovf;  // (re)allocated above
    retry = c->d_retry;
  }
  const uint32_t *tables = override_T;
  int64_t tstride = 0;
  if (override_T) {
    tstride = mc * 8;
  } else if (plan.s.table_mode) {
    if (noalloc) return fail(c, FIRE_E_INVALID, "internal: a table plan without tables");
    fire_status tsx = build_tables(c, lid, betas_dev, n_params, st, &tables, &tstride);
    if (tsx != FIRE_OK) return tsx;
  }
  return launch_run(c, plan, betas_dev, n_params, sims_dev, nullptr, n_sims, seed, tables,
                    tstride, tables ? lid : -1, out, out_maps, map_words, 0, spill, retry, st,
                    nlive == 1 ? lid : -1, work);
}

fire_status fire_run_dev(fire_ctx *c, const double *betas_dev, int32_t n_params,
                         const fire_sim *sims_dev, int32_t n_sims, uint64_t seed,
                         const uint32_t *override_T, fire_result *out,
                         uint32_t *out_maps, int64_t map_words, void *stream) {
  return run_dev_impl(c, betas_dev, n_params, sims_dev, n_sims, seed, override_T, out, out_maps,
                      map_words, stream, false);
}

fire_status fire_run_dev_noalloc(fire_ctx *c, const double *betas_dev, int32_t n_params,
                                 const fire_sim *sims_dev, int32_t n_sims, uint64_t seed,
                                 const uint32_t *override_T, fire_result *out,
                                 uint32_t *out_maps, int64_t map_words, void *stream) {
  if (c && !c->noalloc) return fail(c, FIRE_E_DEVICE, "no scratch on this device");
  return run_dev_impl(c, betas_dev, n_params, sims_dev, n_sims, seed, override_T, out, out_maps,
                      map_words, stream, true);
}

fire_status fire_run_dense(fire_ctx *c, const double *betas, int32_t n_params,
                           const fire_sim *sims, int32_t n_sims, uint64_t seed, fire_result *out,
                           uint32_t *out_maps, int64_t map_words, void *stream) {
  if (!c) return FIRE_E_INVALID;
  if (n_sims < 0 || n_params < 1 || !betas || (n_sims > 0 && (!sims || !out)))
    return fail(c, FIRE_E_INVALID, "bad sizes or null pointers");
  for (int64_t i = 0; i < (int64_t)n_params * 5; ++i)
    if (!std::isfinite(betas[i])) return fail(c, FIRE_E_INVALID, "non-finite beta %lld", (long long)i);
  if (n_sims == 0) return FIRE_OK;
  int bw = 0, one_ls = -1;
  int64_t mc = 1;
  fire_status st0 = check_sims_host(c, sims, n_sims, n_params, &bw, &mc, &one_ls, map_words,
                                    out_maps != nullptr);
  if (st0 != FIRE_OK) return st0;
  for (int32_t i = 0; i < n_sims; ++i)
    if (c->ls[sims[i].landscape_id].burn_steps)
      return fail(c, FIRE_E_UNSUPPORTED, "sim %d: the per-cell path has one-step burns only", i);
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  // scratch: state planes [2][mc] | betas [n_params*5] | counters [2]
  const size_t o_beta = (2 * (size_t)mc + 255) / 256 * 256;
  const size_t o_cnt = (o_beta + sizeof(double) * 5 * (size_t)n_params + 255) / 256 * 256;
  const size_t need = o_cnt + 2 * sizeof(unsigned long long);
  if (need > c->dense_bytes || !c->d_dense) {
    HIP_OR_FAIL(c, hipDeviceSynchronize());
    size_t have = c->dense_bytes;
    HIP_OR_FAIL(c, ensure((void **)&c->d_dense, &have, need));
    c->dense_bytes = have;
  }
  if (!c->h_dense)
    HIP_OR_FAIL(c, hipHostMalloc((void **)&c->h_dense, sizeof(unsigned long long)));
  uint8_t *plane[2] = {c->d_dense, c->d_dense + mc};
  double *d_beta = (double *)(c->d_dense + o_beta);
  unsigned long long *d_cnt = (unsigned long long *)(c->d_dense + o_cnt);
  HIP_OR_FAIL(c, hipMemcpyAsync(d_beta, betas, sizeof(double) * 5 * n_params,
                                hipMemcpyHostToDevice, st));
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  // one simulation after another, one launch per step, the host reading the
  // number of cells ignited after every step (the paper's execution style)
  for (int32_t i = 0; i < n_sims; ++i) {
    const fire_sim &sd = sims[i];
    const LandscapeHost &L = c->ls[sd.landscape_id];
    LandscapeDev D{};
    D.W = L.W; D.H = L.H; D.stride = L.stride; D.valid = 1;
    D.rec = L.rec; D.ps = L.cov;
    D.omega = L.cov ? L.cov + 2 * (int64_t)L.W * L.H : nullptr;
    D.blocked = L.blocked; D.burn_steps = nullptr;
    D.forest_class = L.forest;
    const double *beta = d_beta + 5 * (size_t)sd.param_index;
    HIP_OR_FAIL(c, launch_dense_init(plane[0], D, sd.ign_x, sd.ign_y, d_cnt, st));
    HIP_OR_FAIL(c, hipMemcpyAsync(c->h_dense, d_cnt, sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(c, hipStreamSynchronize(st));
    unsigned long long burning = *c->h_dense;
    uint32_t step = 0;
    int cur = 0;
    while (burning > 0 && step < sd.max_steps) {
      HIP_OR_FAIL(c, launch_fill_u32(reinterpret_cast<uint32_t *>(d_cnt), 0u, 2, st));
      HIP_OR_FAIL(c, launch_dense_step(plane[cur], plane[cur ^ 1], D, beta, sd.sim_index, step,
                                       k0, k1, d_cnt, st));
      HIP_OR_FAIL(c, hipMemcpyAsync(c->h_dense, d_cnt, sizeof(unsigned long long),
                                    hipMemcpyDeviceToHost, st));
      HIP_OR_FAIL(c, hipStreamSynchronize(st));
      burning = *c->h_dense;
      cur ^= 1;
      ++step;
    }
    const bool has_t = sd.target_id >= 0;
    const TargetHost *T = has_t ? &c->tg[sd.target_id] : nullptr;
    HIP_OR_FAIL(c, launch_dense_result(plane[cur], D, has_t ? T->bits : nullptr,
                                       has_t ? T->n_ref : 0u, has_t, step, d_cnt, out + i,
                                       out_maps ? out_maps + (int64_t)i * map_words : nullptr,
                                       st));
  }
  return FIRE_OK;
}

fire_status fire_set_class_schedule(fire_ctx *c, int64_t max_cells, int32_t kind,
                                    const fire_schedule *s) {
  if (!c) return FIRE_E_INVALID;
  if (max_cells < 1) return fail(c, FIRE_E_INVALID, "max_cells < 1");
  if (kind < 0 || kind > 2) return fail(c, FIRE_E_INVALID, "batch kind must be 0, 1 or 2");
  const int b = cells_bucket(max_cells);
  if (s) {
    if (!valid_threads(s->threads))
      return fail(c, FIRE_E_INVALID, "threads must be 64, 128, 256, 512 or 1024");
    if (s->queue_cap < 64 || s->wg_per_cu < 1 || s->wg_per_cu > 32 ||
        (s->table_mode != 0 && s->table_mode != 1) || !valid_window(s->window) ||
        s->wave < -1 || s->wave > 1)
      return fail(c, FIRE_E_INVALID, "schedule field out of range");
  }
  for (size_t i = 0; i < c->class_sched.size(); ++i)
    if (c->class_sched[i].bucket == b && c->class_sched[i].kind == kind) {
      if (s) c->class_sched[i].s = *s;
      else c->class_sched.erase(c->class_sched.begin() + i);
      return FIRE_OK;
    }
  if (s) c->class_sched.push_back({b, kind, *s});
  return FIRE_OK;
}

fire_status fire_set_schedule(fire_ctx *c, const fire_schedule *s) {
  if (!c) return FIRE_E_INVALID;
  if (!s) {
    c->sched_fixed = false;
    return FIRE_OK;
  }
  if (!valid_threads(s->threads) || s->queue_cap < 64 || s->wg_per_cu < 1 ||
      s->wg_per_cu > 32 || (s->table_mode != 0 && s->table_mode != 1) ||
      !valid_window(s->window) || s->wave < -1 || s->wave > 1)
    return fail(c, FIRE_E_INVALID, "schedule field out of range");
  if (s->wave == 1 && simw_lds_bytes(0, s->queue_cap) > c->max_lds)
    return fail(c, FIRE_E_INVALID, "queue_cap %d does not fit LDS", s->queue_cap);
  if (lds_bytes_for(0, s->queue_cap) > c->max_lds)
    return fail(c, FIRE_E_INVALID, "queue_cap %d does not fit LDS", s->queue_cap);
  c->sched = *s;
  c->sched_fixed = true;
  return FIRE_OK;
}

fire_status fire_get_schedule(fire_ctx *c, int64_t max_cells, int32_t n_params,
                              int32_t n_sims, fire_schedule *out) {
  if (!c) return FIRE_E_INVALID;
  if (!out || max_cells < 1 || n_sims < 1) return fail(c, FIRE_E_INVALID, "bad arguments");
  if (c->sched_fixed) {
    *out = c->sched;
    return FIRE_OK;
  }
  // the plan of n_sims simulations on a square lattice of max_cells cells
  // (window re-run statistics: the worst of the loaded landscapes)
  const int side = (int)std::ceil(std::sqrt((double)max_cells));
  const int stride = (side + 31) / 32;
  harvest_stats(c);
  float frac = 0.f;
  for (const auto &L : c->ls)
    if (L.live) frac = std::max(frac, L.win_frac);
  RunPlan plan;
  fire_status ps = plan_run(c, side * stride, max_cells, side, stride, n_params, n_sims, true,
                            &plan, false, frac);
  if (ps != FIRE_OK) return ps;
  *out = plan.s;
  out->window = plan.win;
  out->wave = plan.wave ? 1 : 0;
  return FIRE_OK;
}

fire_status fire_ga_step(fire_ctx *c, double *pop, const double *fit, double *mean_fit,
                         int32_t P, int32_t G, int32_t R, const fire_ga_cfg *cfg,
                         uint32_t gen, uint64_t ga_seed, void *stream) {
  if (!c) return FIRE_E_INVALID;
  if (!pop || !fit || !cfg) return fail(c, FIRE_E_INVALID, "null argument");
  if (P < 1 || P > 1024 || G < 2 || G > 16 || R < 1 || cfg->elite < 0 || cfg->elite > P ||
      cfg->generations < 1 || !(cfg->lo <= cfg->hi) || ga_step_lds(P, G) > c->max_lds)
    return fail(c, FIRE_E_INVALID, "GA sizes or configuration out of range");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, launch_ga_step(pop, fit, mean_fit, P, G, R, cfg->elite, cfg->pm0,
                                uniform_box(cfg->lo, cfg->hi, cfg->mut_h), gen, nullptr,
                                cfg->generations,
                                (uint32_t)ga_seed, (uint32_t)(ga_seed >> 32),
                                (hipStream_t)stream));
  return FIRE_OK;
}

fire_status fire_ga_offspring(fire_ctx *c, const double *pop, const double *fit, int32_t P,
                              int32_t G, int32_t R, const fire_ga_cfg *cfg, uint32_t gen,
                              uint64_t ga_seed, uint64_t seed_step, int32_t n_sets,
                              double *out_sets, void *stream) {
  if (!c) return FIRE_E_INVALID;
  if (!pop || !fit || !cfg || !out_sets) return fail(c, FIRE_E_INVALID, "null argument");
  if (P < 1 || P > 1024 || G < 2 || G > 16 || R < 1 || cfg->elite < 0 || cfg->elite > P ||
      cfg->generations < 1 || !(cfg->lo <= cfg->hi) || ga_step_lds(P, G) > c->max_lds ||
      n_sets < 1 || n_sets > 1024)
    return fail(c, FIRE_E_INVALID, "GA sizes, configuration or set count out of range");
  const uintptr_t a0 = (uintptr_t)pop, a1 = a0 + sizeof(double) * (size_t)P * G;
  const uintptr_t b0 = (uintptr_t)out_sets, b1 = b0 + sizeof(double) * (size_t)n_sets * P * G;
  if (a0 < b1 && b0 < a1) return fail(c, FIRE_E_INVALID, "out_sets overlaps pop");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, launch_ga_offspring(pop, fit, P, G, R, cfg->elite, cfg->pm0,
                                     uniform_box(cfg->lo, cfg->hi, cfg->mut_h), gen,
                                     cfg->generations, ga_seed, seed_step, n_sets, out_sets,
                                     (hipStream_t)stream));
  return FIRE_OK;
}

fire_status fire_ga_step_genes(fire_ctx *c, double *pop, const double *fit, double *mean_fit,
                               int32_t P, int32_t G, int32_t R, int32_t elite, double pm0,
                               const double *lo, const double *hi, const double *h,
                               uint32_t generations, uint32_t gen, uint64_t ga_seed,
                               void *stream) {
  if (!c) return FIRE_E_INVALID;
  if (!pop || !fit || !lo || !hi || !h) return fail(c, FIRE_E_INVALID, "null argument");
  if (P < 1 || P > 1024 || G < 2 || G > kMaxGenes || R < 1 || elite < 0 || elite > P ||
      generations < 1 || ga_step_lds(P, G) > c->max_lds)
    return fail(c, FIRE_E_INVALID, "GA sizes out of range");
  GeneBox box;
  for (int j = 0; j < kMaxGenes; ++j) {
    const int k = j < G ? j : G - 1;
    if (!(lo[k] <= hi[k]) || !std::isfinite(h[k]))
      return fail(c, FIRE_E_INVALID, "gene %d: bad box or mutation width", k);
    box.lo[j] = lo[k];
    box.hi[j] = hi[k];
    box.h[j] = h[k];
  }
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, launch_ga_step(pop, fit, mean_fit, P, G, R, elite, pm0, box, gen, nullptr,
                                generations, (uint32_t)ga_seed, (uint32_t)(ga_seed >> 32),
                                (hipStream_t)stream));
  return FIRE_OK;
}

fire_status fire_ga_sims_from_pop(fire_ctx *c, const double *pop, int32_t P, int32_t G, int32_t R,
                                  int32_t lid, int32_t tid, uint32_t gen, fire_sim *out_sims,
                                  double *out_betas, void *stream) {
  if (!c) return FIRE_E_INVALID;
  if (!pop || !out_sims || !out_betas) return fail(c, FIRE_E_INVALID, "null argument");
  if (P < 1 || R < 1 || G < 7 || G > kMaxGenes || (int64_t)P * R > (1 << 24))
    return fail(c, FIRE_E_INVALID, "sizes out of range (G must hold beta[5], x, y)");
  if (lid < 0 || lid >= (int)c->ls.size() || !c->ls[lid].live)
    return fail(c, FIRE_E_INVALID, "unknown landscape id %d", lid);
  if (tid != -1 && (tid < 0 || tid >= (int)c->tg.size() || !c->tg[tid].live ||
                    c->tg[tid].landscape_id != lid))
    return fail(c, FIRE_E_INVALID, "unknown target id %d for landscape %d", tid, lid);
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  const LandscapeHost &L = c->ls[lid];
  HIP_OR_FAIL(c, launch_sims_from_pop(pop, P, G, R, lid, tid, L.W, L.H, gen, nullptr, out_sims, out_betas,
                                      (hipStream_t)stream));
  return FIRE_OK;
}

// One GA calibration as a captured generation replayed `generations` times:
// prepare (sim indices, population history, work counter) -> [descriptors and
// betas from the ignition genes] -> persistent simulation -> fitness gather ->
// GA step. With ign_genes the individuals are (beta[5], x, y) and every
// generation's ignitions come from genes 5 and 6; otherwise all simulations
// start at (ign_x, ign_y).
static fire_status ga_run_graph(fire_ctx *c, int32_t lid, int32_t tid, int32_t ign_x,
                                int32_t ign_y, bool ign_genes, const double *pop0, int P, int G,
                                int R, int elite, double pm0, const GeneBox &box,
                                uint32_t generations, uint64_t sim_seed, uint64_t ga_seed,
                                double *hist_pop, double *hist_fit, void *stream) {
  if (P < 1 || P > 1024 || R < 1 || (int64_t)P * R > (1 << 24) || elite < 0 || elite > P ||
      generations < 1 || ga_step_lds(P, G) > c->max_lds)
    return fail(c, FIRE_E_INVALID, "GA sizes or configuration out of range");
  if (lid < 0 || lid >= (int)c->ls.size() || !c->ls[lid].live)
    return fail(c, FIRE_E_INVALID, "unknown landscape id %d", lid);
  if (tid < 0 || tid >= (int)c->tg.size() || !c->tg[tid].live || c->tg[tid].landscape_id != lid)
    return fail(c, FIRE_E_INVALID, "unknown target id %d for landscape %d", tid, lid);
  const LandscapeHost &L = c->ls[lid];
  if (!ign_genes && (ign_x < 0 || ign_x >= L.W || ign_y < 0 || ign_y >= L.H))
    return fail(c, FIRE_E_INVALID, "ignition outside the lattice");
  for (int i = 0; i < P * G; ++i)
    if (!std::isfinite(pop0[i])) return fail(c, FIRE_E_INVALID, "non-finite initial population");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  hipStream_t user = (hipStream_t)stream;
  const int n = P * R;
  // scratch: pop [P*G] | fit [n] | results [n] | sims [n] | betas [P*5] | gen counter
  const size_t o_pop = 0;
  const size_t o_fit = o_pop + sizeof(double) * P * G;
  const size_t o_res = (o_fit + sizeof(double) * n + 255) / 256 * 256;
  const size_t o_sims = (o_res + sizeof(fire_result) * n + 255) / 256 * 256;
  const size_t o_beta = (o_sims + sizeof(fire_sim) * n + 255) / 256 * 256;
  const size_t o_gen = (o_beta + sizeof(double) * P * 5 + 255) / 256 * 256;
  const size_t need = o_gen + 256;
  HIP_OR_FAIL(c, hipDeviceSynchronize());
  size_t have = c->ga_bytes;
  HIP_OR_FAIL(c, ensure((void **)&c->d_ga, &have, need));
  c->ga_bytes = have;
  char *base = (char *)c->d_ga;
  double *d_pop = (double *)(base + o_pop);
  double *d_fit = (double *)(base + o_fit);
  fire_result *d_res = (fire_result *)(base + o_res);
  fire_sim *d_sims = (fire_sim *)(base + o_sims);
  double *d_beta = (double *)(base + o_beta);
  uint32_t *d_gen = (uint32_t *)(base + o_gen);
  std::vector<fire_sim> hs(n);
  for (int i = 0; i < P; ++i)
    for (int r = 0; r < R; ++r) {
      fire_sim s{};
      s.landscape_id = lid; s.target_id = tid; s.ign_x = ign_x; s.ign_y = ign_y;
      s.param_index = (uint32_t)i; s.sim_index = 0; s.max_steps = 0xFFFFFFFFu;
      hs[i * R + r] = s;
    }
  HIP_OR_FAIL(c, hipMemcpy(d_sims, hs.data(), sizeof(fire_sim) * n, hipMemcpyHostToDevice));
  HIP_OR_FAIL(c, hipMemcpy(d_pop, pop0, sizeof(double) * P * G, hipMemcpyHostToDevice));
  HIP_OR_FAIL(c, launch_fill_u32(d_gen, 0u, 1, user));
  // plan the simulation launch for this landscape only (on-the-fly thresholds,
  // since the parameters change every generation)
  RunPlan plan;
  harvest_stats(c);
  fire_status ps = plan_run(c, L.H * L.stride, (int64_t)L.W * L.H, L.H, L.stride, P, n, true,
                            &plan, L.burn_steps != nullptr, L.win_frac);
  if (ps != FIRE_OK) return ps;
  // table mode: every generation first writes one threshold table per
  // individual (inside the captured graph)
  const bool tables = plan.s.table_mode != 0;
  const int64_t per = (int64_t)L.W * L.H * 8;
  if (tables) {
    fire_status ts = ensure_tables(c, lid, P, user);
    if (ts != FIRE_OK) return ts;
  }
  fire_status ss = ensure_spill(c, spill_words(plan), user);
  if (ss != FIRE_OK) return ss;
  fire_status rs = ensure_retry(c, 1 + (int64_t)n, user);
  if (rs != FIRE_OK) return rs;

  // capture one generation
  hipStream_t cap = nullptr;
  HIP_OR_FAIL(c, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) e = launch_ga_prepare(d_gen, d_sims, P, R, c->d_work, d_pop, G, hist_pop, cap);
  if (e == hipSuccess && ign_genes)
    e = launch_sims_from_pop(d_pop, P, G, R, lid, tid, L.W, L.H, 0u, d_gen, d_sims, d_beta, cap);
  const double *betas = ign_genes ? d_beta : d_pop;
  if (e == hipSuccess && tables)
    e = launch_thresholds_multi(c->d_ls + lid, L.W, L.H, betas, P, L.forest, c->d_tables, per,
                                cap);
  if (e == hipSuccess &&
      launch_run(c, plan, betas, P, d_sims, nullptr, n, sim_seed, tables ? c->d_tables : nullptr,
                 tables ? per : 0, tables ? lid : -1, d_res, nullptr, 0, 0, c->d_ovf, c->d_retry,
                 cap) != FIRE_OK)
    e = hipErrorLaunchFailure;
  if (e == hipSuccess) e = launch_ga_gather(d_gen, d_res, P, R, d_fit, hist_fit, cap);
  if (e == hipSuccess)
    e = launch_ga_step(d_pop, d_fit, nullptr, P, G, R, elite, pm0, box, 0u, d_gen, generations,
                       (uint32_t)ga_seed, (uint32_t)(ga_seed >> 32), cap);
  hipError_t e2 = hipStreamEndCapture(cap, &graph);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cap);
    return fail(c, FIRE_E_UNSUPPORTED, "GA graph capture failed: %s", hipGetErrorString(e));
  }
  for (uint32_t g = 0; g < generations && e == hipSuccess; ++g)
    e = hipGraphLaunch(exec, user);
  hipError_t e3 = hipStreamSynchronize(user);
  (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cap);
  if (e == hipSuccess) e = e3;
  if (e != hipSuccess) return fail(c, FIRE_E_DEVICE, "GA graph launch: %s", hipGetErrorString(e));
  return FIRE_OK;
}

fire_status fire_ga_run(fire_ctx *c, int32_t lid, int32_t tid, int32_t ign_x, int32_t ign_y,
                        const double *pop0, int32_t P, int32_t R, const fire_ga_cfg *cfg,
                        uint64_t sim_seed, uint64_t ga_seed, double *hist_pop,
                        double *hist_fit, void *stream) {
  if (!c) return FIRE_E_INVALID;
  if (!pop0 || !cfg || !hist_pop || !hist_fit) return fail(c, FIRE_E_INVALID, "null argument");
  if (!(cfg->lo <= cfg->hi) || !std::isfinite(cfg->mut_h))
    return fail(c, FIRE_E_INVALID, "GA sizes or configuration out of range");
  return ga_run_graph(c, lid, tid, ign_x, ign_y, false, pop0, P, 5, R, cfg->elite, cfg->pm0,
                      uniform_box(cfg->lo, cfg->hi, cfg->mut_h), cfg->generations, sim_seed,
                      ga_seed, hist_pop, hist_fit, stream);
}

fire_status fire_ga_run_ignition(fire_ctx *c, int32_t lid, int32_t tid, const double *pop0,
                                 int32_t P, int32_t R, int32_t elite, double pm0,
                                 uint32_t generations, const double *lo, const double *hi,
                                 const double *h, uint64_t sim_seed, uint64_t ga_seed,
                                 double *hist_pop, double *hist_fit, void *stream) {
  if (!c) return FIRE_E_INVALID;
  if (!pop0 || !lo || !hi || !h || !hist_pop || !hist_fit)
    return fail(c, FIRE_E_INVALID, "null argument");
  const int G = 7;
  GeneBox box;
  for (int j = 0; j < kMaxGenes; ++j) {
    const int k = j < G ? j : G - 1;
    if (!(lo[k] <= hi[k]) || !std::isfinite(h[k]))
      return fail(c, FIRE_E_INVALID, "gene %d: bad box or mutation width", k);
    box.lo[j] = lo[k];
    box.hi[j] = hi[k];
    box.h[j] = h[k];
  }
  return ga_run_graph(c, lid, tid, 0, 0, true, pop0, P, G, R, elite, pm0, box, generations,
                      sim_seed, ga_seed, hist_pop, hist_fit, stream);
}

fire_status fire_ensemble(fire_ctx *c, const double *params, const double *deltas, int32_t N,
                          int32_t G, int32_t R, double cutoff, int32_t *out_best,
                          int32_t *out_n, double *out_mean, double *out_sd, void *stream) {
  if (!c) return FIRE_E_INVALID;
  if (!params || !deltas || !out_best || !out_n || !out_mean || !out_sd)
    return fail(c, FIRE_E_INVALID, "null argument");
  if (N < 1 || G < 1 || R < 1 || (int64_t)N * R > (1LL << 30))
    return fail(c, FIRE_E_INVALID, "ensemble sizes out of range");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, launch_ensemble(params, deltas, N, G, R, cutoff, out_best, out_n, out_mean,
                                 out_sd, (hipStream_t)stream));
  return FIRE_OK;
}

fire_status fire_scan_reduce(fire_ctx *c, const double *deltas, int32_t n_cand, int32_t R,
                             double cutoff, double tau, double *out_mean, double *out_sd,
                             double *out_accept, double *out_post, void *stream) {
  if (!c) return FIRE_E_INVALID;
  if (!deltas || !out_mean || !out_sd || !out_accept || !out_post)
    return fail(c, FIRE_E_INVALID, "null argument");
  if (n_cand < 1 || R < 1 || !(tau > 0.0))
    return fail(c, FIRE_E_INVALID, "scan sizes out of range or tau <= 0");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, launch_scan_reduce(deltas, n_cand, R, cutoff, tau, out_mean, out_sd,
                                    out_accept, out_post, (hipStream_t)stream));
  return FIRE_OK;
}

}  // extern "C"
