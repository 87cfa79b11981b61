// HIP kernels (gfx950) of the stochastic CA fire model of Denham & Laneri,
// arXiv 1701.03549: landscape preprocessing, Eq. 1 thresholds, the batched
// simulation kernel with the Eq. 2 fitness fused in, and the device-side
// operators of the parameter search (Appendix B genetic algorithm,
// accepted-ensemble statistics, ignition-scan reduction).
//
// Built with -ffp-contract=off: every binary64 + - * / below is a single
// correctly rounded operation, so the only floating-point differences from
// another IEEE implementation come from cos and from the logistic function's
// own exp and reciprocal (logistic_quantised), each within a few units in
// the last place.

#include <hip/hip_runtime.h>

#include <climits>
#include <map>
#include <mutex>
#include <type_traits>
#include <math.h>
#include <stdint.h>

#include "fire_internal.h"

namespace firegpu {
namespace {

// ---------------------------------------------------------------------------
// Geometry: direction d from source to target, compass angle 45*d degrees.
__device__ __constant__ int kDx[8] = {0, 1, 1, 1, 0, -1, -1, -1};
__device__ __constant__ int kDy[8] = {-1, -1, 0, 1, 1, 1, 0, -1};

constexpr double kDegToRad = 3.14159265358979323846 / 180.0;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11), the counter-based generator the
// paper's CUDA-implementation section uses: ten rounds of two 32x32->64
// multiplies and xors, key advanced by the Weyl increments between rounds.
struct Words4 {
  uint32_t v[4];
};

__device__ __forceinline__ Words4 philox10(uint32_t c0, uint32_t c1,
                                           uint32_t c2, uint32_t c3,
                                           uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p2 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo2 = (uint32_t)p2, hi2 = (uint32_t)(p2 >> 32);
    c0 = hi2 ^ c1 ^ k0;
    c1 = lo2;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Words4 w;
  w.v[0] = c0; w.v[1] = c1; w.v[2] = c2; w.v[3] = c3;
  return w;
}

// ---------------------------------------------------------------------------
// Eq. 1 for the directed edge into target t in direction d, quantised to a
// 32-bit threshold. All covariates belong to the target: I_f from its
// vegetation, psi from its slope and aspect, omega from its wind direction
// against the edge's compass angle, sigma from its slope when it lies
// strictly higher than the source (bit d of its up mask). psi and slope/100
// (ps[2t], ps[2t+1]) and the eight omegas (omega[8t + d]) do not depend on
// beta and are computed once per landscape.
__device__ __forceinline__ uint32_t quantise(double p) {
  // branch-free: p >= 1, NaN and values that round to 2^32 - 1 or above
  // saturate, p <= 0 gives 0
  const double scaled = rint(p * 4294967296.0);
  const double clamped = scaled > 0.0 ? (scaled < 4294967295.0 ? scaled : 0.0) : 0.0;
  const uint32_t t = (uint32_t)clamped;
  const bool sat = !(p < 1.0) || scaled >= 4294967295.0;
  return sat ? kSaturated : t;
}

__device__ __forceinline__ double omega_of(float wind_deg, int d) {
  return cos(((double)wind_deg - 45.0 * (double)d) * kDegToRad);
}

// Eq. 1's probability 1 / (1 + e^(-x)), quantised. e^(-x) by Cody and
// Waite's two-constant reduction, -x = n ln2 + r with |r| <= ln2 / 2 (the
// upper part of ln 2 has 32 significant bits, so n times it is exact), and
// the Taylor series of e^r to degree 12, whose truncation error is below
// 2e-16 relative; the reciprocal of 1 + e^(-x) by the hardware estimate and
// two Newton steps. The probability then lies within a few units in the
// last place of the correctly rounded one, which moves a quantised
// threshold by one unit for about one x in 10^7. Beyond |x| = 40 the
// quantised value is 0 or saturated already, so x is clamped there; a NaN
// saturates.
__device__ __forceinline__ uint32_t logistic_quantised(double x) {
  constexpr double kLog2e = 1.4426950408889634074;
  constexpr double kLn2Hi = 6.93147180369123816490e-01;
  constexpr double kLn2Lo = 1.90821492927058770002e-10;
  const bool nan = x != x;
  x = fmin(fmax(x, -40.0), 40.0);
  const double n = rint(-x * kLog2e);
  double r = fma(-n, kLn2Hi, -x);
  r = fma(-n, kLn2Lo, r);
  double e = 1.0 / 479001600.0;  // 1/12!
  e = fma(e, r, 1.0 / 39916800.0);
  e = fma(e, r, 1.0 / 3628800.0);
  e = fma(e, r, 1.0 / 362880.0);
  e = fma(e, r, 1.0 / 40320.0);
  e = fma(e, r, 1.0 / 5040.0);
  e = fma(e, r, 1.0 / 720.0);
  e = fma(e, r, 1.0 / 120.0);
  e = fma(e, r, 1.0 / 24.0);
  e = fma(e, r, 1.0 / 6.0);
  e = fma(e, r, 0.5);
  e = fma(e, r, 1.0);
  e = fma(e, r, 1.0);
  const double d = 1.0 + __builtin_amdgcn_ldexp(e, (int)n);
  double q = __builtin_amdgcn_rcp(d);
  q = fma(q, fma(-d, q, 1.0), q);
  q = fma(q, fma(-d, q, 1.0), q);
  // q lies in (0, 1 + 2^-52]: rint(q 2^32) is in [0, 2^32], and a value
  // at or above 2^32 - 1 saturates (as quantise does)
  const double scaled = rint(q * 4294967296.0);
  const uint32_t t = (uint32_t)fmin(scaled, 4294967295.0);
  return nan || scaled >= 4294967295.0 ? kSaturated : t;
}

__device__ __forceinline__ uint32_t logistic_threshold(const double *beta, double i_f, double psi,
                                                       double omega, double sigma) {
  double x = beta[0];
  x = x + beta[1] * i_f;
  x = x + beta[2] * psi;
  x = x + beta[3] * omega;
  x = x + beta[4] * sigma;
  return logistic_quantised(x);
}

// The threshold from the landscape's precomputed covariates (F: pointer type
// of the binary64 arrays).
template <typename F>
__device__ __forceinline__ uint32_t edge_threshold(const double *beta, uint32_t vu_t, F ps, F omega,
                                                   int64_t t, int d, uint32_t forest) {
  const uint32_t veg = vu_t & 0xFFu;
  if (veg == 0) return 0u;
  const bool up = ((vu_t >> (8 + d)) & 1u) != 0;
  return logistic_threshold(beta, veg == forest ? 1.0 : 0.0, ps[2 * t], omega[8 * t + d],
                            up ? ps[2 * t + 1] : 0.0);
}

// ---------------------------------------------------------------------------
// Landscape preprocessing: per-cell 16-byte record, aspect covariate and the
// packed non-burnable map (padding bits past W count as non-burnable).
__global__ void preprocess_kernel(const uint8_t *veg, const float *elev,
                                  const float *slope, const float *aspect,
                                  const float *wind, int W, int H, int stride,
                                  uint4 *rec, double *ps, double *omega,
                                  uint32_t *blocked) {
  const int64_t n = (int64_t)W * H;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(c % W), y = (int)(c / W);
    uint32_t up = 0;
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      const int sx = x - kDx[d], sy = y - kDy[d];  // source of edge d into c
      if (sx >= 0 && sx < W && sy >= 0 && sy < H &&
          elev[c] > elev[(int64_t)sy * W + sx])
        up |= 1u << d;
    }
    const float sl = slope[c];
    rec[c] = make_uint4(__float_as_uint(sl), __float_as_uint(aspect[c]),
                        __float_as_uint(wind[c]), (uint32_t)veg[c] | (up << 8));
    ps[2 * c] = (double)sl > 5.0 ? cos(((double)aspect[c] - 315.0) * kDegToRad) : 0.0;
    ps[2 * c + 1] = (double)sl / 100.0;
#pragma unroll
    for (int d = 0; d < 8; ++d) omega[8 * c + d] = omega_of(wind[c], d);
  }
  const int64_t nw = (int64_t)H * stride;
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < nw;
       w += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(w / stride), x0 = (int)(w % stride) * 32;
    uint32_t m = 0;
    for (int b = 0; b < 32; ++b) {
      const int x = x0 + b;
      if (x >= W || veg[(int64_t)y * W + x] == 0) m |= 1u << b;
    }
    blocked[w] = m;
  }
}

// One thread per source cell writes its 8 thresholds (two 16-byte stores)
// for each of up to kBetaPerThread parameter vectors: the covariates of the
// 8 edges (omega evaluated here, not read) are computed once and serve all
// of them, one vector per loop iteration.
constexpr int kBetaPerThread = 16;

__global__ void thresholds_kernel(const LandscapeDev *lsd, int W, int H,
                                  const double *__restrict__ beta_dev, int n_beta, uint32_t forest,
                                  uint32_t *__restrict__ out_base, int64_t out_stride) {
  // parameter vectors b0 .. b0 + nb - 1; vector b's table at out_base + b * out_stride
  const LandscapeDev L = *lsd;
  const int b0 = blockIdx.y * kBetaPerThread;
  const int nb = min(kBetaPerThread, n_beta - b0);
  const int64_t n = (int64_t)W * H;
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(s % W), y = (int)(s / W);
    // the beta-independent covariates of the 8 edges (zero for an edge
    // whose target is outside or not burnable: its threshold is 0)
    double cp[8], co[8], cs[8];
    uint32_t ok = 0, fm = 0;  // edge d: bit d set when it can burn / its target is forest
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      const int tx = x + kDx[d], ty = y + kDy[d];
      cp[d] = co[d] = cs[d] = 0.0;
      if (tx < 0 || tx >= W || ty < 0 || ty >= H) continue;
      const int64_t t = (int64_t)ty * W + tx;
      const uint4 rec = L.rec[t];
      const uint32_t veg = rec.w & 0xFFu;
      if (veg == 0) continue;
      ok |= 1u << d;
      fm |= veg == forest ? 1u << d : 0u;
      cp[d] = L.ps[2 * t];
      cs[d] = ((rec.w >> (8 + d)) & 1u) ? L.ps[2 * t + 1] : 0.0;
      co[d] = omega_of(__uint_as_float(rec.z), d);
    }
    // one table at a time: the 8 evaluations of a vector are independent
    // and branch-free (an edge that cannot burn is evaluated on zero
    // covariates and its result discarded)
#pragma unroll 1
    for (int b = 0; b < nb; ++b) {
      const double *bp = beta_dev + 5 * (int64_t)(b0 + b);
      double beta[5];
#pragma unroll
      for (int i = 0; i < 5; ++i) beta[i] = bp[i];
      uint4 *o = reinterpret_cast<uint4 *>(out_base + (int64_t)(b0 + b) * out_stride + s * 8);
      uint32_t t[8];
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        const uint32_t v =
            logistic_threshold(beta, ((fm >> d) & 1u) ? 1.0 : 0.0, cp[d], co[d], cs[d]);
        t[d] = ((ok >> d) & 1u) ? v : 0u;
      }
      o[0] = make_uint4(t[0], t[1], t[2], t[3]);
      o[1] = make_uint4(t[4], t[5], t[6], t[7]);
    }
  }
}

// Bits 16..23 of every record word: the turn-off time of the cell's
// vegetation (steps[veg]), or 0 when steps is NULL.
__global__ void set_life_kernel(uint4 *rec, int64_t n, const uint8_t *steps) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t w = rec[c].w & 0xFFFFu;
    rec[c].w = w | ((steps ? (uint32_t)steps[w & 0xFFu] : 0u) << 16);
  }
}

// Zero up to three counters in one launch (NULL entries are skipped).
__global__ void zero_words_kernel(uint32_t *p0, uint32_t *p1, uint32_t *p2) {
  if (threadIdx.x == 0) {
    if (p0) *p0 = 0u;
    if (p1) *p1 = 0u;
    if (p2) *p2 = 0u;
  }
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------
// Batched simulation kernel.
//
// A persistent grid; each workgroup repeatedly takes the next simulation
// from an atomic counter and runs it alone:
//   * the burn state is a bitset in LDS (row stride ceil(W/32) words) that
//     starts as the landscape's non-burnable map, so "unburnt and burnable"
//     is a single zero bit; the ignition bit is then set;
//   * the cells that ignited at the previous step form the frontier queue,
//     entries x | y << 12 (the top byte is scratch), held in LDS up to
//     queue_cap entries and in a per-workgroup global spill area beyond;
//   * work is spread one lane per (frontier cell, group of four directions):
//     the four edges of a group take their coins from the four words of one
//     Philox call, which is most of the arithmetic of a step, so each call
//     is made once; a lane reads its four thresholds with one 16-byte load;
//   * each step runs in two phases separated by barriers. Phase 1 only
//     reads the bitset, so eligibility is judged against the burn state at
//     the start of the step; it draws the coins of the eligible edges (small
//     fronts keep the 4-bit outcome in registers, larger ones merge the two
//     nibbles of a cell into its entry's top byte). Phase 2 sets the bits of
//     the successful targets with atomic ORs; the lane whose OR flipped a bit
//     owns that new cell and appends it to the next frontier (bit-sliced
//     ballot prefix of the per-lane counts, one LDS atomic per wave).
// Every coin is a pure function of (sim_index, step, source cell, direction)
// and ignition is an OR, so the burnt set, step count, trial count and
// fitness do not depend on thread order or on the schedule.
//
// With DUR (landscapes with a turn-off time per vegetation type) every
// frontier entry also carries the number of steps its cell stays active, in
// a byte array beside the queue (LDS up to queue_cap, then the spill area):
// a new cell starts with its vegetation's turn-off time, and after the
// step's new cells are appended each entry with more than one step left is
// appended again with one step less. The next frontier is thus every cell
// that is still burning.
// ---------------------------------------------------------------------------

typedef const __attribute__((address_space(1))) uint32_t gmem_cu32;
typedef __attribute__((address_space(1))) uint32_t gmem_u32;
typedef const __attribute__((address_space(1))) double gmem_cf64;
typedef __attribute__((address_space(1))) uint8_t gmem_u8;
typedef const __attribute__((address_space(1))) uint8_t gmem_cu8;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) u32x4 gmem_cu32x4;

// Four consecutive 32-bit words from a 16-byte aligned global address.
__device__ __forceinline__ u32x4 load_x4(gmem_cu32 *q) { return *(gmem_cu32x4 *)q; }

__device__ __forceinline__ uint4 load_rec(const uint4 *base, int64_t t) {
  gmem_cu32 *q = (gmem_cu32 *)(base + t);
  return make_uint4(q[0], q[1], q[2], q[3]);
}

// The vegetation | up-mask word of record t.
__device__ __forceinline__ uint32_t rec_word(const uint4 *base, int64_t t) {
  return ((gmem_cu32 *)(base + t))[3];
}

// Offsets of direction d, packed 2 bits per direction (value + 1).
__device__ __forceinline__ int dir_dx(int d) { return ((425 >> (2 * d)) & 3) - 1; }
__device__ __forceinline__ int dir_dy(int d) { return ((6800 >> (2 * d)) & 3) - 1; }

__device__ __forceinline__ uint32_t lane_prefix(uint64_t ballot) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(ballot >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)ballot, 0u));
}

// kLen0 + k % 3: frontier length of step k; kAbort0 + k % 3: step k is not
// to run (a burning cell reached a window edge during step k - 1). Three
// slots: a slot is written only after the first barrier of the step before
// the one that reads it, and reset at the top of the step before that.
enum CtlSlot { kSim = 0, kLen0 = 1, kTrials = 4, kNew = 5, kInter = 6, kAbort0 = 7,
               kCtlWords = 16 };

// register-resident rounds of the small-front step (fronts of up to
// kRegRounds * BLOCK / 2 cells held in the LDS queue)
constexpr int kRegRounds = 2;

// GB (global bitset, never with WIN): the burn bitset of the workgroup's
// simulation is its own a.bitset_words words of a.gbits in global memory
// instead of LDS, for lattices whose bitset does not fit LDS. Its words are
// read, written and ORed with agent-scope atomics, which are performed at
// L2: the waves of the workgroup then never read a stale vector-L1 copy of
// a word another wave has ORed, nor one left from the workgroup's previous
// simulation, and the barriers order the phases as they do for LDS.
template <int BLOCK, bool TABLE, bool DUR, bool WIN, bool GB = false>
__global__ __launch_bounds__(BLOCK) void sim_kernel(SimArgs a) {
  static_assert(!(GB && WIN), "a global bitset covers the whole lattice");
  extern __shared__ uint32_t lds[];
  const int bw = a.bitset_words;
  const uint32_t cap = (uint32_t)a.queue_cap;
  uint32_t *const bits = GB ? a.gbits + (int64_t)blockIdx.x * bw : lds;
  const int lbw = GB ? 0 : bw;  // bitset words in LDS
  auto bload = [&](int w) -> uint32_t {
    if constexpr (GB) return __hip_atomic_load(&bits[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return bits[w];
  };
  auto bstore = [&](int w, uint32_t v) {
    if constexpr (GB) __hip_atomic_store(&bits[w], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else bits[w] = v;
  };
  auto bor = [&](int w, uint32_t v) -> uint32_t {
    if constexpr (GB)
      return __hip_atomic_fetch_or(&bits[w], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return atomicOr(&bits[w], v);
  };
  uint32_t *const ctl = lds + lbw + 2 * cap;
  gmem_u32 *const spill_base = (gmem_u32 *)(a.ovf + (int64_t)blockIdx.x * 2 * a.ovf_cap);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // remaining active steps of the queue entries (DUR only)
  uint8_t *const life_lds = reinterpret_cast<uint8_t *>(ctl + kCtlWords);
  gmem_u8 *const life_spill =
      DUR ? (gmem_u8 *)(a.ovf_life + (int64_t)blockIdx.x * 2 * a.ovf_cap) : nullptr;
  auto l_load = [&](uint32_t q, uint32_t i) -> uint32_t {
    if (i < cap) return life_lds[q * cap + i];
    return life_spill[(int64_t)q * a.ovf_cap + (i - cap)];
  };
  auto l_store = [&](uint32_t q, uint32_t i, uint32_t v) {
    if (i < cap) life_lds[q * cap + i] = (uint8_t)v;
    else life_spill[(int64_t)q * a.ovf_cap + (i - cap)] = (uint8_t)v;
  };

  // frontier queue q (0 or 1), entry i
  auto q_load = [&](uint32_t q, uint32_t i) -> uint32_t {
    if (i < cap) return lds[lbw + q * cap + i];
    return spill_base[(int64_t)q * a.ovf_cap + (i - cap)];
  };
  auto q_store = [&](uint32_t q, uint32_t i, uint32_t v) {
    if (i < cap) lds[lbw + q * cap + i] = v;
    else spill_base[(int64_t)q * a.ovf_cap + (i - cap)] = v;
  };

  // the count of simulations this launch runs, for the host's statistics
  if (a.stat_out != nullptr && a.n_dev != nullptr && blockIdx.x == 0 && tid == 0)
    *a.stat_out = *a.n_dev;

  for (;;) {
    if (tid == 0) {
      const uint32_t k = atomicAdd(a.work, 1u);
      const uint32_t n = a.n_dev ? *a.n_dev : (uint32_t)a.n_sims;
      const uint32_t took = k < n ? (a.order ? a.order[k] : k) : 0xFFFFFFFFu;
      ctl[kSim] = took;
      if (a.times != nullptr && (int64_t)took < a.times_cap)
        a.times[2 * (int64_t)took] = wall_clock64();
    }
    __syncthreads();
    const uint32_t sim = ctl[kSim];
    if (sim == 0xFFFFFFFFu) break;
    const fire_sim sd = a.sims[sim];

    // -- descriptor checks (uniform over the workgroup) --------------------
    bool ok = sd.landscape_id >= 0 && sd.landscape_id < a.n_ls &&
              sd.param_index < (uint32_t)a.n_params;
    LandscapeDev L{};
    if (ok) {
      L = a.ls[sd.landscape_id];
      ok = L.valid && sd.ign_x >= 0 && sd.ign_x < L.W && sd.ign_y >= 0 &&
           sd.ign_y < L.H &&
           (WIN ? min(a.win, L.H) * min(a.win >> 5, L.stride) : L.H * L.stride) <=
               a.bitset_words &&
           (a.maps == nullptr || (int64_t)L.H * L.stride <= a.map_words) &&
           (a.tables == nullptr || a.table_ls == sd.landscape_id);
    }
    TargetDev tg{};
    const bool has_target = sd.target_id >= 0;
    if (ok && has_target) {
      ok = sd.target_id < a.n_tg;
      if (ok) {
        tg = a.tg[sd.target_id];
        ok = tg.valid && tg.landscape_id == sd.landscape_id;
      }
    } else if (ok) {
      ok = sd.target_id == -1;
    }
    if (!ok) {
      if (tid == 0) {
        fire_result r;
        r.burnt = 0; r.steps = 0xFFFFFFFFu; r.trials = 0;
        r.fitness = __builtin_nan("");
        a.out[sim] = r;
        if (a.times != nullptr && (int64_t)sim < a.times_cap)
          a.times[2 * (int64_t)sim + 1] = wall_clock64();
        atomicOr(a.error_flag, 1u);
      }
      __syncthreads();
      continue;
    }

    const int W = L.W, H = L.H, stride = L.stride;
    const int words = H * stride;
    const int ix = sd.ign_x, iy = sd.ign_y;
    gmem_cu32 *const blocked = (gmem_cu32 *)L.blocked;
    const bool burnable = ((blocked[iy * stride + (ix >> 5)] >> (ix & 31)) & 1u) == 0;
    if (!burnable) {
      // a non-burnable ignition burns nothing
      if (tid == 0) {
        fire_result r;
        r.burnt = 0; r.steps = 0; r.trials = 0;
        r.fitness = has_target ? 1.0 : __builtin_nan("");
        a.out[sim] = r;
        if (a.times != nullptr && (int64_t)sim < a.times_cap)
          a.times[2 * (int64_t)sim + 1] = wall_clock64();
      }
      if (a.maps != nullptr) {
        uint32_t *m = a.maps + (int64_t)sim * a.map_words;
        for (int w = tid; w < words; w += BLOCK) m[w] = 0u;
      }
      __syncthreads();
      continue;
    }

    // -- window: the LDS bitset covers rows [wy0, wy0 + wh) and words
    //    [wx0w, wx0w + ws) of each row, placed around the ignition (the whole
    //    lattice without a window). A burning cell within one cell of a
    //    window edge that is not a lattice edge aborts the run before its
    //    neighbours are read (its edges are not tried), and the run is then
    //    repeated without a window; every neighbour that is read lies in the
    //    window.
    const int ws = WIN ? min(a.win >> 5, stride) : stride;
    const int wh = WIN ? min(a.win, H) : H;
    const int wx0w = WIN ? min(max((ix >> 5) - ws / 2, 0), stride - ws) : 0;
    const int wy0 = WIN ? min(max(iy - wh / 2, 0), H - wh) : 0;
    // cells whose edges may be tried: one cell inside every window edge
    // that lies inside the lattice (x in [x_lo, x_lo + x_span], same for y;
    // coordinates are below 4096, so the spans of an uncut axis cover all)
    const int x_lo = wx0w > 0 ? 32 * wx0w + 1 : 0;
    const uint32_t x_span = (uint32_t)((wx0w + ws < stride ? 32 * (wx0w + ws) - 2 : 8191) - x_lo);
    const int y_lo = wy0 > 0 ? wy0 + 1 : 0;
    const uint32_t y_span = (uint32_t)((wy0 + wh < H ? wy0 + wh - 2 : 8191) - y_lo);
    auto near_edge = [&](int x, int y) -> bool {
      return WIN && ((uint32_t)(x - x_lo) > x_span || (uint32_t)(y - y_lo) > y_span);
    };
    // LDS word of cell (x, y) inside the window
    const int w_off = wy0 * ws + wx0w;
    auto bw_of = [&](int x, int y) -> int { return y * ws + (x >> 5) - w_off; };
    // global word of window word w
    auto gw_of = [&](int w) -> int { return (wy0 + w / ws) * stride + wx0w + w % ws; };
    const int wwords = wh * ws;

    // -- init: bitset = non-burnable map, ignition burnt -------------------
    for (int w = tid; w < wwords; w += BLOCK) bstore(w, blocked[gw_of(w)]);
    if (tid == 0) {
      ctl[kLen0 + 0] = 1; ctl[kLen0 + 1] = 0; ctl[kLen0 + 2] = 0;
      ctl[kTrials] = 0; ctl[kNew] = 0; ctl[kInter] = 0;
      ctl[kAbort0 + 0] = 0u; ctl[kAbort0 + 1] = 0u; ctl[kAbort0 + 2] = 0u;
    }
    __syncthreads();
    // active steps of a cell that ignites (bits 16..23 of its record word
    // hold its vegetation's turn-off time when the landscape has them)
    const bool has_life = DUR && L.burn_steps != nullptr;
    auto life_of = [&](int x, int y) -> uint32_t {
      if (!has_life) return 1u;
      return (rec_word(L.rec, (int64_t)y * W + x) >> 16) & 0xFFu;
    };
    if (tid == 0) {
      bor(bw_of(ix, iy), 1u << (ix & 31));
      q_store(0, 0, (uint32_t)ix | ((uint32_t)iy << 12));
      if (DUR) l_store(0, 0, life_of(ix, iy));
    }
    double beta[5];
    if (!TABLE) {
      const double *bp = a.betas + (int64_t)sd.param_index * 5;
#pragma unroll
      for (int i = 0; i < 5; ++i) beta[i] = bp[i];
    }
    gmem_cu32 *const table =
        TABLE ? (gmem_cu32 *)(a.tables + (int64_t)sd.param_index * a.table_stride) : nullptr;
    __syncthreads();

    uint32_t cq = 0, step = 0;
    uint32_t my_trials = 0, my_new = 0;
    const uint32_t max_steps = sd.max_steps;
    const uint32_t sim_index = sd.sim_index;
    // frontier length of step k lives in ctl[kLen0 + k % 3]
    int slot = 0;
    bool aborted = false;
    // a new cell enters the queue with life 0 (not yet known); the first
    // unit of its entry looks it up in phase 1 of the next step, where the
    // read overlaps the unit's other reads, and it is needed only after
    // that phase
    auto resolve_life = [&](uint32_t e, uint32_t i) {
      if (DUR && l_load(cq, i) == 0u)
        l_store(cq, i, life_of((int)(e & 0xFFFu), (int)((e >> 12) & 0xFFFu)));
    };

    // The four edges of group g, k = 0..3, point to (0, -s), (s, -s),
    // (s, 0), (s, s) with s = +1 for g = 0 (N, NE, E, SE) and s = -1 for
    // g = 1 (S, SW, W, NW). Their LDS words and bits around a source at
    // (x, y) with word `base` and bit xb: a column step crosses a word
    // boundary only at bit 0 or 31.
    struct GroupGeom {
      int wk[4], bk[4];  // LDS word and bit of each target
      int tk[4];         // lattice offset (cells) of each target
      int s;
    };
    auto group_geom = [&](int xb, int base, uint32_t g) -> GroupGeom {
      GroupGeom q;
      q.s = g ? -1 : 1;
      const int sws = g ? -ws : ws;
      const int xs = xb + q.s;  // -1 .. 32
      const int wo = xs >> 5;   // -1, 0 or 1
      const int bs = xs & 31;
      q.wk[0] = base - sws;      q.bk[0] = xb;
      q.wk[1] = base - sws + wo; q.bk[1] = bs;
      q.wk[2] = base + wo;       q.bk[2] = bs;
      q.wk[3] = base + sws + wo; q.bk[3] = bs;
      const int sW = g ? -W : W;
      q.tk[0] = -sW;
      q.tk[1] = q.s - sW;
      q.tk[2] = q.s;
      q.tk[3] = q.s + sW;
      return q;
    };

    // Phase 1 for one unit: frontier entry e and direction group g (edges
    // d = 4g .. 4g+3, whose coins are the four words of one Philox call
    // (sim_index, step, source, g)). An edge is tried when its target is
    // inside, burnable and unburnt at the start of the step. Returns the
    // 4-bit mask of tried edges whose coin succeeds; n_tried counts the
    // tried edges.
    // `overlap` (per-trial thresholds only): evaluate the four edges'
    // Eq. 1 together, eligible or not, which shortens the step on small
    // fronts; large fronts evaluate only the eligible edges, one at a time.
    auto unit_outcome = [&](auto overlap, uint32_t e, uint32_t g,
                            uint32_t &n_tried) -> uint32_t {
      const int x = (int)(e & 0xFFFu), y = (int)((e >> 12) & 0xFFFu);
      const uint32_t s_lin = (uint32_t)(y * W + x);
      // a source at a window edge: read none of its neighbours; bit 4 of
      // the result asks phase 2 to end the run
      const bool edge = near_edge(x, y);
      uint32_t thr[4] = {0u, 0u, 0u, 0u};
      if (TABLE) {
        // the 8 thresholds of a source are 32 contiguous bytes; group g is
        // the 16-byte half g (tables are 16-byte aligned)
        const u32x4 t4 = load_x4(table + (int64_t)s_lin * 8 + 4 * g);
        thr[0] = t4.x; thr[1] = t4.y; thr[2] = t4.z; thr[3] = t4.w;
      }
      // neighbour words from the source's: one row is ws words, and a
      // column step crosses a word boundary only at bit 0 or 31. An edge
      // whose target is outside (or whose source is at a window edge) reads
      // the source's own bit, which is set: the four reads are unconditional
      // and issue back to back.
      const int base = bw_of(x, y), xb = x & 31;
      const GroupGeom q = group_geom(xb, base, g);
      const bool r1 = (unsigned)(y - q.s) < (unsigned)H && !edge;  // row -s
      const bool r2 = (unsigned)(y + q.s) < (unsigned)H && !edge;  // row +s
      const bool c1 = (unsigned)(x + q.s) < (unsigned)W;           // column +s
      const bool in[4] = {r1, r1 && c1, c1 && !edge, r2 && c1};
      uint32_t elig = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int w = in[k] ? q.wk[k] : base;
        const int b = in[k] ? q.bk[k] : xb;
        elig |= ((bload(w) >> b) & 1u) == 0 ? (1u << k) : 0u;
      }
      n_tried = __popc(elig);
      // not gated on elig: the rounds then overlap the bitset and table reads
      const Words4 r = philox10(sim_index, step, s_lin, g, a.key0, a.key1);
      uint32_t hit = 0;
      if (TABLE) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (((elig >> k) & 1u) && (thr[k] == kSaturated || r.v[k] < thr[k])) hit |= 1u << k;
      } else if (decltype(overlap)::value) {
        // the four Eq. 1 evaluations are independent: evaluated together
        // (ineligible edges read their source's own record) they overlap
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int d = 4 * (int)g + k;
          const bool el = (elig >> k) & 1u;
          const int64_t tl = el ? (int64_t)s_lin + q.tk[k] : (int64_t)s_lin;
          const uint32_t t = edge_threshold(beta, rec_word(L.rec, tl), (gmem_cf64 *)L.ps,
                                            (gmem_cf64 *)L.omega, tl, d, L.forest_class);
          if (el && (t == kSaturated || r.v[k] < t)) hit |= 1u << k;
        }
      } else {
        // the covariates of all four targets are read first (an ineligible
        // edge reads its source's own), then Eq. 1 is evaluated for the
        // eligible edges only
        uint32_t vu[4];
        double psi[4], slope[4], om[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int d = 4 * (int)g + k;
          const bool el = (elig >> k) & 1u;
          const int64_t tl = el ? (int64_t)s_lin + q.tk[k] : (int64_t)s_lin;
          vu[k] = rec_word(L.rec, tl);
          psi[k] = ((gmem_cf64 *)L.ps)[2 * tl];
          slope[k] = ((gmem_cf64 *)L.ps)[2 * tl + 1];
          om[k] = ((gmem_cf64 *)L.omega)[8 * tl + d];
        }
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {
          if (!((elig >> k) & 1u)) continue;
          const int d = 4 * (int)g + k;
          const uint32_t v = k == 0 ? vu[0] : k == 1 ? vu[1] : k == 2 ? vu[2] : vu[3];
          const uint32_t veg = v & 0xFFu;
          uint32_t t = 0u;
          if (veg != 0) {
            const double ps_k = k == 0 ? psi[0] : k == 1 ? psi[1] : k == 2 ? psi[2] : psi[3];
            const double sl_k = k == 0 ? slope[0] : k == 1 ? slope[1] : k == 2 ? slope[2] : slope[3];
            const double om_k = k == 0 ? om[0] : k == 1 ? om[1] : k == 2 ? om[2] : om[3];
            t = logistic_threshold(beta, veg == L.forest_class ? 1.0 : 0.0, ps_k, om_k,
                                   ((v >> (8 + d)) & 1u) ? sl_k : 0.0);
          }
          const uint32_t coin = k == 0 ? r.v[0] : k == 1 ? r.v[1] : k == 2 ? r.v[2] : r.v[3];
          if (t == kSaturated || coin < t) hit |= 1u << k;
        }
      }
      return hit | (WIN && edge ? 16u : 0u);
    };

    // Phase 2 for one unit: set the bits of the hit targets; returns the
    // mask of targets whose bit this lane flipped (cells it now owns).
    auto unit_ignite = [&](uint32_t e, uint32_t g, uint32_t hit) -> uint32_t {
      uint32_t fresh = 0;
      const int x = (int)(e & 0xFFFu), y = (int)((e >> 12) & 0xFFFu);
      // branch-free: an edge that did not hit ORs 0 into its source's own
      // word, so the four atomics issue back to back
      const int base = bw_of(x, y), xb = x & 31;
      const GroupGeom q = group_geom(xb, base, g);
      uint32_t old[4], bitv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool h = (hit >> k) & 1u;
        const int w = h ? q.wk[k] : base;
        bitv[k] = h ? 1u << q.bk[k] : 0u;
        old[k] = bor(w, bitv[k]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (bitv[k] && (old[k] & bitv[k]) == 0) fresh |= 1u << k;
      return fresh;
    };

    // Append each lane's fresh cells to the next frontier: a wave-wide
    // exclusive prefix of the per-lane counts (0..4) from three bit-sliced
    // ballots, one LDS atomic per wave. `direct`: the queue slot is known to
    // lie in LDS.
    auto append = [&](uint32_t e, uint32_t g, uint32_t fresh, int nslot, bool direct) {
      const uint32_t cnt = __popc(fresh);
      const uint64_t b0 = __ballot(cnt & 1u), b1 = __ballot(cnt & 2u), b2 = __ballot(cnt & 4u);
      const uint32_t total = (uint32_t)(__popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2));
      if (total == 0) return;
      uint32_t wbase = 0;
      if (lane == 0) wbase = atomicAdd(&ctl[kLen0 + nslot], total);
      wbase = __builtin_amdgcn_readfirstlane(wbase);
      if (!fresh) return;
      uint32_t idx = wbase + lane_prefix(b0) + 2 * lane_prefix(b1) + 4 * lane_prefix(b2);
      const int x = (int)(e & 0xFFFu), y = (int)((e >> 12) & 0xFFFu);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (!((fresh >> k) & 1u)) continue;
        // edge k of group g: (0, -s), (s, -s), (s, 0), (s, s)
        const int sg = g ? -1 : 1;
        const int tx = x + (k == 0 ? 0 : sg), ty = y + (k == 2 ? 0 : (k == 3 ? sg : -sg));
        const uint32_t v = (uint32_t)tx | ((uint32_t)ty << 12);
        if (direct) {
          lds[lbw + (cq ^ 1u) * cap + idx] = v;
          if (DUR) life_lds[(cq ^ 1u) * cap + idx] = 0u;
        } else {
          q_store(cq ^ 1u, idx, v);
          if (DUR) l_store(cq ^ 1u, idx, 0u);
        }
        ++idx;
        ++my_new;
      }
    };

    for (;; ++step) {
      // the frontier length and this lane's first entry are read together
      const uint32_t n_cur = ctl[kLen0 + slot];
      const uint32_t e_first = lds[lbw + cq * cap + min((uint32_t)tid >> 1, cap - 1)];
      aborted = WIN && ctl[kAbort0 + slot] != 0u;
      if (n_cur == 0 || step >= max_steps || aborted) break;
      const int nslot = slot == 2 ? 0 : slot + 1;
      if (tid == 0) {
        ctl[kLen0 + nslot] = 0;
        if (WIN) ctl[kAbort0 + nslot] = 0;
      }
      const uint32_t n_units = 2 * n_cur;

      if (n_units <= (uint32_t)(kRegRounds * BLOCK) && n_cur <= cap) {
        // -- small front: outcomes stay in registers between the phases and
        //    the current queue is in LDS; new cells go straight to LDS when
        //    they cannot outgrow it (8 per entry), else through q_store --
        const bool direct = 8 * n_cur <= cap;
        uint32_t hit[kRegRounds], ent[kRegRounds];
#pragma unroll
        for (int rr = 0; rr < kRegRounds; ++rr) {
          hit[rr] = 0;
          ent[rr] = 0;
          const uint32_t j = (uint32_t)(tid + rr * BLOCK);
          if (rr * BLOCK < (int)n_units && j < n_units) {
            const uint32_t e = rr == 0 ? e_first : lds[lbw + cq * cap + (j >> 1)];
            ent[rr] = e;
            if ((j & 1u) == 0) resolve_life(e, j >> 1);
            uint32_t nt;
            hit[rr] = unit_outcome(std::true_type{}, e, j & 1u, nt);
            my_trials += nt;
          }
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < kRegRounds; ++rr) {
          if (rr * BLOCK >= (int)n_units) break;
          const uint32_t g = (uint32_t)tid & 1u;
          if (WIN && (hit[rr] & 16u)) ctl[kAbort0 + nslot] = 1u;
          const uint32_t h4 = hit[rr] & 15u;
          const uint32_t fresh = h4 ? unit_ignite(ent[rr], g, h4) : 0u;
          append(ent[rr], g, fresh, nslot, direct);
        }
      } else {
        // -- general front: the two units of an entry merge their outcome
        //    nibbles into the entry's top byte; queues spill to global
        //    memory past queue_cap ----------------------------------------
        for (uint32_t j = tid; j < n_units; j += BLOCK) {
          const uint32_t e = q_load(cq, j >> 1);
          if ((j & 1u) == 0) resolve_life(e, j >> 1);
          uint32_t nt;
          const uint32_t m = unit_outcome(std::false_type{}, e, j & 1u, nt) & 15u;
          my_trials += nt;
          const uint32_t other = (uint32_t)__shfl_xor((int)m, 1);
          const uint32_t m8 = (j & 1u) ? 0u : (m | (other << 4));
          if (m8 != 0) q_store(cq, j >> 1, e | (m8 << 24));
        }
        __syncthreads();
        for (uint32_t base = 0; base < n_units; base += BLOCK) {
          const uint32_t j = base + (uint32_t)tid;
          const uint32_t g = j & 1u;
          uint32_t e = 0, fresh = 0;
          if (j < n_units) {
            e = q_load(cq, j >> 1);
            if (WIN && near_edge((int)(e & 0xFFFu), (int)((e >> 12) & 0xFFFu)))
              ctl[kAbort0 + nslot] = 1u;
            const uint32_t hit = (e >> (24 + 4 * g)) & 0xFu;
            if (hit) fresh = unit_ignite(e, g, hit);
          }
          append(e, g, fresh, nslot, false);
        }
      }
      if (DUR) {
        // cells still burning after this step follow the new ones
        __syncthreads();
        for (uint32_t base = 0; base < n_cur; base += BLOCK) {
          const uint32_t i = base + (uint32_t)tid;
          uint32_t lf = 0, e = 0;
          if (i < n_cur) {
            lf = l_load(cq, i);
            if (lf > 1u) e = q_load(cq, i) & 0xFFFFFFu;
          }
          const bool keep = lf > 1u;
          const uint64_t bal = __ballot(keep);
          if (bal != 0) {
            uint32_t wbase = 0;
            if (lane == 0) wbase = atomicAdd(&ctl[kLen0 + nslot], (uint32_t)__popcll(bal));
            wbase = __builtin_amdgcn_readfirstlane(wbase);
            if (keep) {
              const uint32_t idx = wbase + lane_prefix(bal);
              q_store(cq ^ 1u, idx, e);
              l_store(cq ^ 1u, idx, lf - 1u);
            }
          }
        }
      }
      __syncthreads();
      slot = nslot;
      cq ^= 1u;
    }

    if (aborted) {
      // the fire reached the window edge: queue the simulation for a run
      // without a window (every lane left the loop at the same step)
      __syncthreads();
      if (tid == 0) a.retry[1 + atomicAdd(a.retry, 1u)] = sim;
      continue;
    }

    // -- result: counts, Eq. 2 over the rows the fire reached, map ---------
    if (my_trials) atomicAdd(&ctl[kTrials], my_trials);
    if (my_new) atomicAdd(&ctl[kNew], my_new);
    __syncthreads();
    if (has_target) {
      // |A n A*| = popcount(burnt & reference) over the bitset
      gmem_cu32 *const ref = (gmem_cu32 *)tg.bits;
      uint32_t inter = 0;
      for (int w = tid; w < wwords; w += BLOCK) {
        const int gw = gw_of(w);
        inter += __popc(bload(w) & ~blocked[gw] & ref[gw]);
      }
      if (inter) atomicAdd(&ctl[kInter], inter);
      __syncthreads();
    }
    if (tid == 0) {
      fire_result r;
      r.burnt = 1u + ctl[kNew];
      r.steps = step;
      r.trials = ctl[kTrials];
      if (has_target) {
        const int64_t num = (int64_t)tg.n_ref + r.burnt - 2 * (int64_t)ctl[kInter];
        r.fitness = (double)num / (double)tg.n_ref;
      } else {
        r.fitness = __builtin_nan("");
      }
      a.out[sim] = r;
      if (a.times != nullptr && (int64_t)sim < a.times_cap)
        a.times[2 * (int64_t)sim + 1] = wall_clock64();
    }
    if (a.maps != nullptr) {
      uint32_t *m = a.maps + (int64_t)sim * a.map_words;
      for (int w = tid; w < words; w += BLOCK) {
        const int y = w / stride, xw = w % stride;
        const bool in = y >= wy0 && y < wy0 + wh && xw >= wx0w && xw < wx0w + ws;
        m[w] = in ? bload((y - wy0) * ws + (xw - wx0w)) & ~blocked[w] : 0u;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Wavefront-per-simulation kernel, for fronts of up to queue_cap cells.
//
// Each workgroup is one 64-lane wavefront that takes simulations from the
// same atomic work counter as sim_kernel and runs each alone, with no
// workgroup barrier: the parts of a step are ordered by program order
// within the wavefront (LDS operations of one wavefront are performed in
// issue order), and every count that decides control flow is wave-uniform.
// LDS per wavefront: burn bitset (whole lattice or window, as in
// sim_kernel) and two frontier queues of queue_cap entries.
// A step with up to 4 * 64 units (frontier entry, direction group) keeps
// up to four units per lane in registers and interleaves them: the entries,
// the targets' bits, the thresholds and the four Philox evaluations of all
// of a lane's units are issued before any result is needed, then the bits
// of the hit targets are set (every bit read of the step precedes every
// atomic, so eligibility is the burn state at the start of the step) and
// the cells whose bit a lane flipped are appended to the next frontier. A
// larger front first stores the hit nibbles of each entry in its queue
// word's top byte, then sets bits and appends in a second pass.
// A simulation whose next frontier would exceed queue_cap, or (with a
// window) whose fire comes within one cell of a window edge inside the
// lattice, stops and is listed in `retry` for the whole-lattice re-run
// launch of sim_kernel, which draws the same coins and so gives the same
// result.
// ---------------------------------------------------------------------------
constexpr int kWave = 64;
constexpr int kWaveRegUnits = 4;  // units per lane held in registers

// LDS words of one wavefront of simw_kernel.
__host__ __device__ constexpr int64_t simw_lds_words(int bitset_words, int queue_cap) {
  return (int64_t)bitset_words + 2 * (int64_t)queue_cap;
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <bool TABLE, bool WIN>
__global__ __launch_bounds__(kWave) void simw_kernel(SimArgs a) {
  extern __shared__ uint32_t lds[];
  const int bw = a.bitset_words;
  const uint32_t cap = (uint32_t)a.queue_cap;
  uint32_t *const bits = lds;
  uint32_t *const ql = lds + bw;  // queue q entry i: ql[q * cap + i]
  const int lane = threadIdx.x;

  for (;;) {
    uint32_t sim = 0;
    if (lane == 0) {
      const uint32_t k = atomicAdd(a.work, 1u);
      const uint32_t n = a.n_dev ? *a.n_dev : (uint32_t)a.n_sims;
      sim = k < n ? (a.order ? a.order[k] : k) : 0xFFFFFFFFu;
      if (a.times != nullptr && (int64_t)sim < a.times_cap)
        a.times[2 * (int64_t)sim] = wall_clock64();
    }
    sim = __builtin_amdgcn_readfirstlane(sim);
    if (sim == 0xFFFFFFFFu) break;
    const fire_sim sd = a.sims[sim];

    // -- descriptor checks, as in sim_kernel -------------------------------
    bool ok = sd.landscape_id >= 0 && sd.landscape_id < a.n_ls &&
              sd.param_index < (uint32_t)a.n_params;
    LandscapeDev L{};
    if (ok) {
      L = a.ls[sd.landscape_id];
      ok = L.valid && sd.ign_x >= 0 && sd.ign_x < L.W && sd.ign_y >= 0 &&
           sd.ign_y < L.H &&
           (WIN ? min(a.win, L.H) * min(a.win >> 5, L.stride) : L.H * L.stride) <=
               a.bitset_words &&
           (a.maps == nullptr || (int64_t)L.H * L.stride <= a.map_words) &&
           (a.tables == nullptr || a.table_ls == sd.landscape_id);
    }
    TargetDev tg{};
    const bool has_target = sd.target_id >= 0;
    if (ok && has_target) {
      ok = sd.target_id < a.n_tg;
      if (ok) {
        tg = a.tg[sd.target_id];
        ok = tg.valid && tg.landscape_id == sd.landscape_id;
      }
    } else if (ok) {
      ok = sd.target_id == -1;
    }
    if (!ok) {
      if (lane == 0) {
        fire_result r;
        r.burnt = 0; r.steps = 0xFFFFFFFFu; r.trials = 0;
        r.fitness = __builtin_nan("");
        a.out[sim] = r;
        if (a.times != nullptr && (int64_t)sim < a.times_cap)
          a.times[2 * (int64_t)sim + 1] = wall_clock64();
        atomicOr(a.error_flag, 1u);
      }
      continue;
    }
    const int W = L.W, H = L.H, stride = L.stride;
    const int words = H * stride;
    const int ix = sd.ign_x, iy = sd.ign_y;
    gmem_cu32 *const blocked = (gmem_cu32 *)L.blocked;
    if (((blocked[iy * stride + (ix >> 5)] >> (ix & 31)) & 1u) != 0) {
      // a non-burnable ignition burns nothing
      if (lane == 0) {
        fire_result r;
        r.burnt = 0; r.steps = 0; r.trials = 0;
        r.fitness = has_target ? 1.0 : __builtin_nan("");
        a.out[sim] = r;
        if (a.times != nullptr && (int64_t)sim < a.times_cap)
          a.times[2 * (int64_t)sim + 1] = wall_clock64();
      }
      if (a.maps != nullptr) {
        uint32_t *m = a.maps + (int64_t)sim * a.map_words;
        for (int w = lane; w < words; w += kWave) m[w] = 0u;
      }
      continue;
    }

    // -- window (whole lattice without one), as in sim_kernel --------------
    const int ws = WIN ? min(a.win >> 5, stride) : stride;
    const int wh = WIN ? min(a.win, H) : H;
    const int wx0w = WIN ? min(max((ix >> 5) - ws / 2, 0), stride - ws) : 0;
    const int wy0 = WIN ? min(max(iy - wh / 2, 0), H - wh) : 0;
    const int x_lo = wx0w > 0 ? 32 * wx0w + 1 : 0;
    const uint32_t x_span = (uint32_t)((wx0w + ws < stride ? 32 * (wx0w + ws) - 2 : 8191) - x_lo);
    const int y_lo = wy0 > 0 ? wy0 + 1 : 0;
    const uint32_t y_span = (uint32_t)((wy0 + wh < H ? wy0 + wh - 2 : 8191) - y_lo);
    const int w_off = wy0 * ws + wx0w;
    const int wwords = wh * ws;

    for (int w = lane; w < wwords; w += kWave)
      bits[w] = blocked[(wy0 + w / ws) * stride + wx0w + w % ws];
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    if (lane == 0) {
      bits[iy * ws + (ix >> 5) - w_off] |= 1u << (ix & 31);
      ql[0] = (uint32_t)ix | ((uint32_t)iy << 12);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    double beta[5];
    if (!TABLE) {
      const double *bp = a.betas + (int64_t)sd.param_index * 5;
#pragma unroll
      for (int i = 0; i < 5; ++i) beta[i] = bp[i];
    }
    gmem_cu32 *const table =
        TABLE ? (gmem_cu32 *)(a.tables + (int64_t)sd.param_index * a.table_stride) : nullptr;
    const uint32_t max_steps = sd.max_steps;
    const uint32_t sim_index = sd.sim_index;

    uint32_t n_cur = 1, cq = 0, step = 0, n_new = 0, my_trials = 0;
    bool stopped = false;

    // Targets of group g around a source at (x, y): (0, -s), (s, -s),
    // (s, 0), (s, s), s = +1 for g = 0 and -1 for g = 1. LDS words and bits
    // of the four; an edge that cannot be tried (target outside, or source
    // at a window edge) reads its source's own bit, which is set.
    struct Unit {
      uint32_t e, g, elig, hit;
      int base, xb;
      int wk[4], bk[4];
      bool edge;
    };
    auto unit_geom = [&](Unit &u, uint32_t e, uint32_t g, bool valid) {
      u.e = e;
      u.g = g;
      const int x = (int)(e & 0xFFFu), y = (int)((e >> 12) & 0xFFFu);
      u.edge = WIN && valid && ((uint32_t)(x - x_lo) > x_span || (uint32_t)(y - y_lo) > y_span);
      const int sg = g ? -1 : 1;
      const int sws = g ? -ws : ws;
      u.base = y * ws + (x >> 5) - w_off;
      u.xb = x & 31;
      const int xs = u.xb + sg;
      const int wo = xs >> 5, bs = xs & 31;
      u.wk[0] = u.base - sws;       u.bk[0] = u.xb;
      u.wk[1] = u.base - sws + wo;  u.bk[1] = bs;
      u.wk[2] = u.base + wo;        u.bk[2] = bs;
      u.wk[3] = u.base + sws + wo;  u.bk[3] = bs;
      const bool r1 = (unsigned)(y - sg) < (unsigned)H && !u.edge;
      const bool r2 = (unsigned)(y + sg) < (unsigned)H && !u.edge;
      const bool c1 = (unsigned)(x + sg) < (unsigned)W;
      const bool in[4] = {r1 && valid, r1 && c1 && valid, c1 && !u.edge && valid,
                          r2 && c1 && valid};
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (!in[q]) {
          u.wk[q] = u.base;
          u.bk[q] = u.xb;
        }
    };
    // the threshold of edge q (0..3) of the unit (TABLE: from the table)
    auto thresholds = [&](const Unit &u, uint32_t s_lin, uint32_t thr[4]) {
      if (TABLE) {
        const u32x4 t4 = load_x4(table + (int64_t)s_lin * 8 + 4 * u.g);
        thr[0] = t4.x; thr[1] = t4.y; thr[2] = t4.z; thr[3] = t4.w;
      } else {
        // Eq. 1 for the eligible edges; the covariates of the four targets
        // are read first (an ineligible edge reads its source's)
        const int sg = u.g ? -1 : 1;
        const int sW = u.g ? -W : W;
        const int tk[4] = {-sW, sg - sW, sg, sg + sW};
        uint32_t vu[4];
        double psi[4], slope[4], om[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int d = 4 * (int)u.g + q;
          const int64_t tl = ((u.elig >> q) & 1u) ? (int64_t)s_lin + tk[q] : (int64_t)s_lin;
          vu[q] = rec_word(L.rec, tl);
          psi[q] = ((gmem_cf64 *)L.ps)[2 * tl];
          slope[q] = ((gmem_cf64 *)L.ps)[2 * tl + 1];
          om[q] = ((gmem_cf64 *)L.omega)[8 * tl + d];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int d = 4 * (int)u.g + q;
          const uint32_t veg = vu[q] & 0xFFu;
          thr[q] = ((u.elig >> q) & 1u) && veg != 0
                       ? logistic_threshold(beta, veg == L.forest_class ? 1.0 : 0.0, psi[q],
                                            om[q], ((vu[q] >> (8 + d)) & 1u) ? slope[q] : 0.0)
                       : 0u;
        }
      }
    };
    // set the bits of the hit targets; the mask of targets whose bit this
    // lane flipped
    auto ignite = [&](const Unit &u, uint32_t hit) -> uint32_t {
      uint32_t old[4], bitv[4], fresh = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool h = (hit >> q) & 1u;
        bitv[q] = h ? 1u << u.bk[q] : 0u;
        old[q] = atomicOr(&bits[h ? u.wk[q] : u.base], bitv[q]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (bitv[q] && (old[q] & bitv[q]) == 0) fresh |= 1u << q;
      return fresh;
    };
    // append the fresh cells of every lane (wave prefix of per-lane counts
    // 0..4); `n_next` and `over` are wave-uniform
    auto append = [&](const Unit &u, uint32_t fresh, uint32_t &n_next, bool &over) {
      const uint32_t cnt = __popc(fresh);
      const uint64_t b0 = __ballot(cnt & 1u), b1 = __ballot(cnt & 2u), b2 = __ballot(cnt & 4u);
      const uint32_t total = (uint32_t)(__popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2));
      if (over || n_next + total > cap) {
        over = true;
      } else if (fresh) {
        uint32_t idx = n_next + lane_prefix(b0) + 2 * lane_prefix(b1) + 4 * lane_prefix(b2);
        const int x = (int)(u.e & 0xFFFu), y = (int)((u.e >> 12) & 0xFFFu);
        const int sg = u.g ? -1 : 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (!((fresh >> q) & 1u)) continue;
          const int tx = x + (q == 0 ? 0 : sg), ty = y + (q == 2 ? 0 : (q == 3 ? sg : -sg));
          ql[(cq ^ 1u) * cap + idx++] = (uint32_t)tx | ((uint32_t)ty << 12);
        }
      }
      n_next += total;
    };

    // a step whose units fit R per lane: everything in registers
    auto step_regs = [&](auto RC, uint32_t n_units, uint32_t &n_next, bool &over) -> bool {
      constexpr int R = decltype(RC)::value;
      Unit u[R];
      uint32_t rv[R][4], thr[R][4], s_lin[R], wv[R][4];
      bool valid[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t j = (uint32_t)(lane + kWave * r);
        valid[r] = j < n_units;
        // a lane without a unit takes entry 0 (a burning cell inside the
        // bitset) and reads only its own bit
        const uint32_t e = ql[cq * cap + (valid[r] ? j >> 1 : 0u)] & 0xFFFFFFu;
        unit_geom(u[r], e, j & 1u, valid[r]);
        s_lin[r] = (uint32_t)((int)((e >> 12) & 0xFFFu) * W + (int)(e & 0xFFFu));
#pragma unroll
        for (int q = 0; q < 4; ++q) wv[r][q] = bits[u[r].wk[q]];
      }
      if (TABLE) {
#pragma unroll
        for (int r = 0; r < R; ++r) thresholds(u[r], s_lin[r], thr[r]);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const Words4 w4 = philox10(sim_index, step, s_lin[r], u[r].g, a.key0, a.key1);
#pragma unroll
        for (int q = 0; q < 4; ++q) rv[r][q] = w4.v[q];
      }
      bool edge = false;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        uint32_t el = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) el |= ((wv[r][q] >> u[r].bk[q]) & 1u) == 0 ? 1u << q : 0u;
        u[r].elig = el;
        my_trials += __popc(el);
        edge = edge || u[r].edge;
      }
      if (WIN && __ballot(edge) != 0) return true;
      if (!TABLE) {
#pragma unroll
        for (int r = 0; r < R; ++r) thresholds(u[r], s_lin[r], thr[r]);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        uint32_t hit = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (((u[r].elig >> q) & 1u) && (thr[r][q] == kSaturated || rv[r][q] < thr[r][q]))
            hit |= 1u << q;
        u[r].hit = hit;
      }
      uint32_t fresh[R];
#pragma unroll
      for (int r = 0; r < R; ++r) fresh[r] = u[r].hit ? ignite(u[r], u[r].hit) : 0u;
#pragma unroll
      for (int r = 0; r < R; ++r) append(u[r], fresh[r], n_next, over);
      return false;
    };

    for (;;) {
      if (n_cur == 0 || step >= max_steps) break;
      const uint32_t n_units = 2 * n_cur;
      uint32_t n_next = 0;
      bool over = false, edge = false;
      if (n_units <= (uint32_t)(kWave * kWaveRegUnits)) {
        const uint32_t rounds = (n_units + kWave - 1) / kWave;
        if (rounds == 1) edge = step_regs(std::integral_constant<int, 1>{}, n_units, n_next, over);
        else if (rounds == 2) edge = step_regs(std::integral_constant<int, 2>{}, n_units, n_next, over);
        else if (rounds == 3) edge = step_regs(std::integral_constant<int, 3>{}, n_units, n_next, over);
        else edge = step_regs(std::integral_constant<int, 4>{}, n_units, n_next, over);
      } else {
        // large front: hit nibbles of both groups of an entry go to its
        // queue word's top byte, then a second pass sets bits and appends
        for (uint32_t base = 0; base < n_units; base += kWave) {
          const uint32_t j = base + (uint32_t)lane;
          const bool valid = j < n_units;
          Unit u;
          const uint32_t e = ql[cq * cap + (valid ? j >> 1 : 0u)] & 0xFFFFFFu;
          unit_geom(u, e, j & 1u, valid);
          const uint32_t s_lin = (uint32_t)((int)((e >> 12) & 0xFFFu) * W + (int)(e & 0xFFFu));
          uint32_t wv[4], thr[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) wv[q] = bits[u.wk[q]];
          if (TABLE) thresholds(u, s_lin, thr);
          const Words4 w4 = philox10(sim_index, step, s_lin, u.g, a.key0, a.key1);
          uint32_t el = 0;
#pragma unroll
          for (int q = 0; q < 4; ++q) el |= ((wv[q] >> u.bk[q]) & 1u) == 0 ? 1u << q : 0u;
          u.elig = el;
          my_trials += __popc(el);
          edge = edge || __ballot(u.edge) != 0;
          if (!TABLE) thresholds(u, s_lin, thr);
          uint32_t hit = 0;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (((el >> q) & 1u) && (thr[q] == kSaturated || w4.v[q] < thr[q])) hit |= 1u << q;
          const uint32_t other = (uint32_t)__shfl_xor((int)hit, 1);
          if (valid && (j & 1u) == 0 && (hit | other) != 0)
            ql[cq * cap + (j >> 1)] = e | ((hit | (other << 4)) << 24);
        }
        if (WIN && edge) {
          stopped = true;
          break;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        for (uint32_t base = 0; base < n_units; base += kWave) {
          const uint32_t j = base + (uint32_t)lane;
          const bool valid = j < n_units;
          const uint32_t q8 = ql[cq * cap + (valid ? j >> 1 : 0u)];
          Unit u;
          unit_geom(u, q8 & 0xFFFFFFu, j & 1u, valid);
          const uint32_t hit = valid ? (q8 >> (24 + 4 * (j & 1u))) & 15u : 0u;
          const uint32_t fresh = hit ? ignite(u, hit) : 0u;
          append(u, fresh, n_next, over);
        }
      }
      if (edge || over) {
        stopped = true;
        break;
      }
      n_new += n_next;
      n_cur = n_next;
      cq ^= 1u;
      ++step;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }

    if (stopped) {
      // outgrew the queues or reached the window edge: run again over the
      // whole lattice in the workgroup kernel
      if (lane == 0) a.retry[1 + atomicAdd(a.retry, 1u)] = sim;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      continue;
    }

    // -- result: counts, Eq. 2 over the window, map ------------------------
    const uint64_t trials = wave_sum(my_trials);
    uint64_t inter = 0;
    if (has_target) {
      gmem_cu32 *const ref = (gmem_cu32 *)tg.bits;
      uint32_t mine = 0;
      for (int w = lane; w < wwords; w += kWave) {
        const int gw = (wy0 + w / ws) * stride + wx0w + w % ws;
        mine += __popc(bits[w] & ~blocked[gw] & ref[gw]);
      }
      inter = wave_sum(mine);
    }
    if (lane == 0) {
      fire_result r;
      r.burnt = 1u + n_new;
      r.steps = step;
      r.trials = trials;
      if (has_target) {
        const int64_t num = (int64_t)tg.n_ref + r.burnt - 2 * (int64_t)inter;
        r.fitness = (double)num / (double)tg.n_ref;
      } else {
        r.fitness = __builtin_nan("");
      }
      a.out[sim] = r;
      if (a.times != nullptr && (int64_t)sim < a.times_cap)
        a.times[2 * (int64_t)sim + 1] = wall_clock64();
    }
    if (a.maps != nullptr) {
      uint32_t *m = a.maps + (int64_t)sim * a.map_words;
      for (int w = lane; w < words; w += kWave) {
        const int y = w / stride, xw = w % stride;
        const bool in = y >= wy0 && y < wy0 + wh && xw >= wx0w && xw < wx0w + ws;
        m[w] = in ? bits[(y - wy0) * ws + (xw - wx0w)] & ~blocked[w] : 0u;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
}

// ---------------------------------------------------------------------------
// Genetic-algorithm generation (Appendix B): elitism, tournament of two,
// one-point crossover of consecutive non-elite pairs, dynamic mutation.
// One workgroup, thread i owns slot i. Only exact IEEE operations.
// Workgroup b reads the parents from src and writes its offspring set to
// dst + b * dst_stride under key (k1:k0) + b * key_step (64-bit): one
// workgroup with src == dst is the in-place generation step; several give
// offspring sets of one parent population (gen_ptr is then NULL, and only
// workgroup 0 writes mean_fit).
__global__ void ga_step_kernel(const double *src, double *dst, int64_t dst_stride,
                               uint64_t key_step, const double *fit,
                               double *mean_fit, int P, int G, int R,
                               int elite, double pm0, GeneBox box, uint32_t gen_arg,
                               uint32_t *gen_ptr, uint32_t generations,
                               uint32_t key0, uint32_t key1) {
  extern __shared__ double sh[];
  double *mean = sh;            // [P]
  double *oldp = sh + P;        // [P][G]
  double *newp = oldp + P * G;  // [P][G]
  int *order = reinterpret_cast<int *>(newp + P * G);  // [P]
  const uint32_t gen = gen_ptr ? *gen_ptr : gen_arg;
  const int i = threadIdx.x;
  const uint64_t key = (((uint64_t)key1 << 32) | key0) + (uint64_t)blockIdx.x * key_step;
  const uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
  double *pop = dst + (int64_t)blockIdx.x * dst_stride;

  if (i < P) {
    double acc = 0.0;
    for (int r = 0; r < R; ++r) acc = acc + fit[(int64_t)i * R + r];
    mean[i] = acc / (double)R;
    for (int j = 0; j < G; ++j) oldp[i * G + j] = src[(int64_t)i * G + j];
  }
  __syncthreads();
  if (i < P) order[i] = i;
  __syncthreads();
  if (i < P) {
    // rank by (fitness, index)
    const double mi = mean[i];
    int rank = 0;
    for (int j = 0; j < P; ++j) {
      const double mj = mean[j];
      rank += (mj < mi || (mj == mi && j < i)) ? 1 : 0;
    }
    order[rank] = i;
  }
  __syncthreads();
  if (i < P) {
    int src;
    if (i < elite) {
      src = order[i];
    } else {
      const Words4 o = philox10(gen, (uint32_t)i, 0u, 0u, k0, k1);
      const int pa = (int)(((uint64_t)o.v[0] * (uint64_t)P) >> 32);
      const int pb = (int)(((uint64_t)o.v[1] * (uint64_t)P) >> 32);
      if (mean[pa] < mean[pb]) src = pa;
      else if (mean[pb] < mean[pa]) src = pb;
      else src = pa < pb ? pa : pb;
    }
    for (int j = 0; j < G; ++j) newp[i * G + j] = oldp[src * G + j];
  }
  __syncthreads();
  const int n_pairs = (P - elite) / 2;
  if (i < n_pairs) {
    const Words4 o = philox10(gen, (uint32_t)i, 1u, 0u, k0, k1);
    const int cut = 1 + (int)(((uint64_t)o.v[0] * (uint64_t)(G - 1)) >> 32);
    double *u = newp + (elite + 2 * i) * G;
    double *v = newp + (elite + 2 * i + 1) * G;
    for (int j = cut; j < G; ++j) {
      const double t = u[j];
      u[j] = v[j];
      v[j] = t;
    }
  }
  __syncthreads();
  if (i < P) {
    if (i >= elite) {
      const double pm = pm0 * (1.0 - (double)gen / (double)generations);
      for (int j = 0; j < G; ++j) {
        const Words4 o = philox10(gen, (uint32_t)i, 2u, (uint32_t)j, k0, k1);
        const double u0 = (double)o.v[0] * (1.0 / 4294967296.0);
        if (u0 < pm) {
          const double u1 = (double)o.v[1] * (1.0 / 4294967296.0);
          double g = newp[i * G + j] + box.h[j] * (2.0 * u1 - 1.0);
          if (g < box.lo[j]) g = box.lo[j];
          if (g > box.hi[j]) g = box.hi[j];
          newp[i * G + j] = g;
        }
      }
    }
    for (int j = 0; j < G; ++j) pop[(int64_t)i * G + j] = newp[i * G + j];
    if (mean_fit && blockIdx.x == 0) mean_fit[i] = mean[i];
  }
  __syncthreads();
  if (gen_ptr && i == 0) *gen_ptr = gen + 1;
}

// Descriptors of generation g: sim_index = (g*P + i)*R + r; also resets the
// work counter of the simulation kernel and records the population.
__global__ void ga_prepare_kernel(const uint32_t *gen_ptr, fire_sim *sims,
                                  int P, int R, uint32_t *work,
                                  const double *pop, int G, double *hist_pop) {
  const uint32_t gen = *gen_ptr;
  const int n = P * R;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += gridDim.x * blockDim.x) {
    sims[k].sim_index = (gen * (uint32_t)P + (uint32_t)(k / R)) * (uint32_t)R +
                        (uint32_t)(k % R);
  }
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < P * G;
       k += gridDim.x * blockDim.x)
    hist_pop[(int64_t)gen * P * G + k] = pop[k];
  if (blockIdx.x == 0 && threadIdx.x == 0) *work = 0u;
}

__global__ void ga_gather_kernel(const uint32_t *gen_ptr,
                                 const fire_result *res, int P, int R,
                                 double *fit, double *hist_fit) {
  const uint32_t gen = *gen_ptr;
  const int n = P * R;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += gridDim.x * blockDim.x) {
    const double f = res[k].fitness;
    fit[k] = f;
    hist_fit[(int64_t)gen * n + k] = f;
  }
}

// Descriptors of a generation whose individuals carry their ignition cell as
// genes 5 and 6: the cell is the nearest one (round half up), clamped to the
// lattice; genes 0..4 are copied to a [P][5] parameter array.
__global__ void sims_from_pop_kernel(const double *pop, int P, int G, int R,
                                     int32_t landscape_id, int32_t target_id, int W,
                                     int H, uint32_t gen_arg, const uint32_t *gen_ptr,
                                     fire_sim *sims, double *betas) {
  const uint32_t gen = gen_ptr ? *gen_ptr : gen_arg;
  const int n = P * R;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int i = k / R;
    const double *ind = pop + (int64_t)i * G;
    double fx = floor(ind[5] + 0.5), fy = floor(ind[6] + 0.5);
    fx = fx < 0.0 ? 0.0 : (fx > (double)(W - 1) ? (double)(W - 1) : fx);
    fy = fy < 0.0 ? 0.0 : (fy > (double)(H - 1) ? (double)(H - 1) : fy);
    fire_sim sd;
    sd.landscape_id = landscape_id;
    sd.target_id = target_id;
    sd.ign_x = (int32_t)fx;
    sd.ign_y = (int32_t)fy;
    sd.param_index = (uint32_t)i;
    sd.sim_index = (gen * (uint32_t)P + (uint32_t)i) * (uint32_t)R + (uint32_t)(k % R);
    sd.max_steps = 0xFFFFFFFFu;
    sims[k] = sd;
    if (k % R == 0)
      for (int j = 0; j < 5; ++j) betas[(int64_t)i * 5 + j] = ind[j];
  }
}

// ---------------------------------------------------------------------------
// Per-cell form of the step (an ablation of sim_kernel after the paper's own
// kernel): one thread per cell sweeps the whole lattice every step. A cell
// that is burnable and unburnt at the start of the step and has burning
// neighbours evaluates Eq. 1 for each of them (quantised like an edge
// threshold), multiplies (1 - p_i) in binary64 in direction order and draws
// one uniform, word 0 of Philox(sim_index, step, cell, 2); a saturated edge
// makes the ignition certain. State bytes: 0 unburnt, 1 burning (ignited at
// the previous step), 2 burnt out. counts[0] += cells ignited, counts[1] +=
// draws.
__global__ void dense_step_kernel(const uint8_t *__restrict__ cur, uint8_t *__restrict__ nxt,
                                  LandscapeDev L, const double *beta_dev, uint32_t sim_index,
                                  uint32_t step, uint32_t k0, uint32_t k1,
                                  unsigned long long *counts) {
  const int W = L.W, H = L.H;
  const int64_t n = (int64_t)W * H;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ignited = false, drew = false;
  if (t < n) {
    const uint8_t st = cur[t];
    uint8_t out = 0;
    const int x = (int)(t % W), y = (int)(t / W);
    if (st != 0) {
      out = 2;
    } else if (((L.blocked[(int64_t)y * L.stride + (x >> 5)] >> (x & 31)) & 1u) == 0) {
      uint32_t burning = 0;
      for (int d = 0; d < 8; ++d) {
        const int sx = x + dir_dx(d), sy = y + dir_dy(d);
        if ((unsigned)sx < (unsigned)W && (unsigned)sy < (unsigned)H &&
            cur[(int64_t)sy * W + sx] == 1)
          burning |= 1u << d;
      }
      if (burning) {
        double beta[5];
        for (int k = 0; k < 5; ++k) beta[k] = beta_dev[k];
        const uint32_t vu = rec_word(L.rec, t);
        double q = 1.0;
        bool sure = false;
        for (int d = 0; d < 8; ++d) {
          if (!((burning >> d) & 1u)) continue;
          // the edge from the neighbour in direction d points the other way
          const uint32_t thr = edge_threshold(beta, vu, L.ps, L.omega, t, (d + 4) & 7,
                                              L.forest_class);
          sure = sure || thr == kSaturated;
          q = q * (1.0 - (double)thr * (1.0 / 4294967296.0));
        }
        const Words4 r = philox10(sim_index, step, (uint32_t)t, 2u, k0, k1);
        const uint32_t thr_t = sure ? kSaturated : quantise(1.0 - q);
        ignited = thr_t == kSaturated || r.v[0] < thr_t;
        drew = true;
        out = ignited ? 1 : 0;
      }
    }
    nxt[t] = out;
  }
  const uint64_t bi = __ballot(ignited), bd = __ballot(drew);
  if ((threadIdx.x & 63) == 0 && (bi | bd)) {
    if (bi) atomicAdd(&counts[0], (unsigned long long)__popcll(bi));
    if (bd) atomicAdd(&counts[1], (unsigned long long)__popcll(bd));
  }
}

// State of a new simulation: the ignition burning if it is burnable;
// counts[0] = 1 (or 0 for a non-burnable ignition), counts[1] = 0.
__global__ void dense_init_kernel(uint8_t *st, LandscapeDev L, int ix, int iy,
                                  unsigned long long *counts) {
  const int64_t n = (int64_t)L.W * L.H;
  const int64_t ign = (int64_t)iy * L.W + ix;
  const bool ok = ((L.blocked[(int64_t)iy * L.stride + (ix >> 5)] >> (ix & 31)) & 1u) == 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    st[i] = (i == ign && ok) ? 1 : 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    counts[0] = ok ? 1ull : 0ull;
    counts[1] = 0ull;
  }
}

// Result of a finished per-cell simulation: packed map, |A*|, |A n A*| and
// Eq. 2 (one workgroup of kDenseResThreads threads, fixed-order sums of
// integers).
constexpr int kDenseResThreads = 1024;
__global__ __launch_bounds__(kDenseResThreads) void dense_result_kernel(
    const uint8_t *st, LandscapeDev L, const uint32_t *ref, uint32_t n_ref, int has_target,
    uint32_t steps, const unsigned long long *counts, fire_result *out, uint32_t *map) {
  __shared__ uint32_t sb[kDenseResThreads], si[kDenseResThreads];
  const int W = L.W, stride = L.stride;
  const int words = L.H * stride;
  uint32_t burnt = 0, inter = 0;
  for (int w = threadIdx.x; w < words; w += kDenseResThreads) {
    const int y = w / stride, x0 = (w % stride) * 32;
    uint32_t bits = 0;
    for (int b = 0; b < 32 && x0 + b < W; ++b)
      bits |= (st[(int64_t)y * W + x0 + b] != 0 ? 1u : 0u) << b;
    burnt += __popc(bits);
    if (has_target) inter += __popc(bits & ref[w]);
    if (map) map[w] = bits;
  }
  sb[threadIdx.x] = burnt;
  si[threadIdx.x] = inter;
  __syncthreads();
  for (int h = kDenseResThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sb[threadIdx.x] += sb[threadIdx.x + h];
      si[threadIdx.x] += si[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    fire_result r;
    r.burnt = sb[0];
    r.steps = steps;
    r.trials = counts[1];
    if (has_target) {
      const int64_t num = (int64_t)n_ref + sb[0] - 2 * (int64_t)si[0];
      r.fitness = (double)num / (double)n_ref;
    } else {
      r.fitness = __builtin_nan("");
    }
    *out = r;
  }
}

// ---------------------------------------------------------------------------
// Accepted-ensemble statistics: one workgroup of 1024 threads; every sum is
// reduced in a fixed tree order, so repeated runs give identical bits.
constexpr int kRedThreads = 1024;

__device__ double block_sum(double v, double *red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int off = kRedThreads / 2; off > 0; off >>= 1) {
    if (t < off) red[t] = red[t] + red[t + off];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kRedThreads) void ensemble_kernel(
    const double *params, const double *deltas, int N, int G, int R,
    double cutoff, int32_t *out_best, int32_t *out_n, double *out_mean,
    double *out_sd) {
  __shared__ double red[kRedThreads];
  __shared__ double bval[kRedThreads];
  __shared__ int bidx[kRedThreads];
  const int t = threadIdx.x;
  const int64_t total = (int64_t)N * R;
  // best single simulation (first index on ties) and accepted count
  double bv = INFINITY;
  int bi = 0x7FFFFFFF;
  double cnt = 0.0;
  for (int64_t k = t; k < total; k += kRedThreads) {
    const double d = deltas[k];
    if (d < bv) { bv = d; bi = (int)k; }
    if (d < cutoff) cnt += 1.0;
  }
  bval[t] = bv;
  bidx[t] = bi;
  __syncthreads();
  for (int off = kRedThreads / 2; off > 0; off >>= 1) {
    if (t < off) {
      const double ov = bval[t + off];
      const int oi = bidx[t + off];
      if (ov < bval[t] || (ov == bval[t] && oi < bidx[t])) {
        bval[t] = ov;
        bidx[t] = oi;
      }
    }
    __syncthreads();
  }
  const double n_acc = block_sum(cnt, red);
  if (t == 0) {
    *out_best = bidx[0] == 0x7FFFFFFF ? 0 : bidx[0] / R;
    *out_n = (int32_t)n_acc;
  }
  for (int j = 0; j < G; ++j) {
    double s = 0.0;
    for (int64_t k = t; k < total; k += kRedThreads)
      if (deltas[k] < cutoff) s = s + params[(k / R) * G + j];
    const double sum = block_sum(s, red);
    const double mean = n_acc > 0.0 ? sum / n_acc : __builtin_nan("");
    double q = 0.0;
    for (int64_t k = t; k < total; k += kRedThreads)
      if (deltas[k] < cutoff) {
        const double dv = params[(k / R) * G + j] - mean;
        q = q + dv * dv;
      }
    const double sq = block_sum(q, red);
    if (t == 0) {
      out_mean[j] = mean;
      out_sd[j] = n_acc > 1.0 ? sqrt(sq / (n_acc - 1.0)) : 0.0;
    }
  }
}

// Ignition scan: thread c reduces candidate c's replicates in order; the map
// normalisation is a fixed-order tree sum.
__global__ __launch_bounds__(kRedThreads) void scan_reduce_kernel(
    const double *deltas, int n_cand, int R, double cutoff, double tau,
    double *out_mean, double *out_sd, double *out_accept, double *out_post) {
  __shared__ double red[kRedThreads];
  const int t = threadIdx.x;
  double acc_local = 0.0, minm = INFINITY;
  for (int c = t; c < n_cand; c += kRedThreads) {
    const double *d = deltas + (int64_t)c * R;
    double s = 0.0;
    int na = 0;
    for (int r = 0; r < R; ++r) {
      s = s + d[r];
      na += d[r] < cutoff ? 1 : 0;
    }
    const double m = s / (double)R;
    double q = 0.0;
    for (int r = 0; r < R; ++r) {
      const double dv = d[r] - m;
      q = q + dv * dv;
    }
    out_mean[c] = m;
    out_sd[c] = R > 1 ? sqrt(q / (double)(R - 1)) : 0.0;
    out_accept[c] = (double)na / (double)R;
    acc_local = acc_local + out_accept[c];
    minm = fmin(minm, m);
  }
  const double acc_sum = block_sum(acc_local, red);
  // minimum mean (for the softmin fallback)
  red[t] = minm;
  __syncthreads();
  for (int off = kRedThreads / 2; off > 0; off >>= 1) {
    if (t < off) red[t] = fmin(red[t], red[t + off]);
    __syncthreads();
  }
  const double mmin = red[0];
  __syncthreads();
  if (acc_sum > 0.0) {
    for (int c = t; c < n_cand; c += kRedThreads) out_post[c] = out_accept[c] / acc_sum;
  } else {
    double w_local = 0.0;
    for (int c = t; c < n_cand; c += kRedThreads) {
      const double w = exp(-(out_mean[c] - mmin) / tau);
      out_post[c] = w;
      w_local = w_local + w;
    }
    const double ws = block_sum(w_local, red);
    for (int c = t; c < n_cand; c += kRedThreads) out_post[c] = out_post[c] / ws;
  }
}

int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers

hipError_t launch_preprocess(const uint8_t *veg, const float *elev,
                             const float *slope, const float *aspect,
                             const float *wind, int W, int H, int stride,
                             uint4 *rec, double *ps, double *omega, uint32_t *blocked,
                             hipStream_t s) {
  const int64_t n = (int64_t)W * H;
  hipLaunchKernelGGL(preprocess_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s,
                     veg, elev, slope, aspect, wind, W, H, stride, rec, ps, omega,
                     blocked);
  return hipGetLastError();
}

hipError_t launch_thresholds(const LandscapeDev *ls_dev_entry, int W, int H,
                             const double *beta_dev, uint32_t forest,
                             uint32_t *out, hipStream_t s) {
  return launch_thresholds_multi(ls_dev_entry, W, H, beta_dev, 1, forest, out, 0, s);
}

hipError_t launch_thresholds_multi(const LandscapeDev *ls_dev_entry, int W, int H,
                                   const double *betas_dev, int n_params, uint32_t forest,
                                   uint32_t *out, int64_t out_stride, hipStream_t s) {
  const int64_t n = (int64_t)W * H;
  const int groups = (n_params + kBetaPerThread - 1) / kBetaPerThread;
  hipLaunchKernelGGL(thresholds_kernel, dim3(grid_for(n, 256), groups), dim3(256), 0, s,
                     ls_dev_entry, W, H, betas_dev, n_params, forest, out, out_stride);
  return hipGetLastError();
}

hipError_t launch_dense_init(uint8_t *st, const LandscapeDev &L, int ix, int iy,
                             unsigned long long *counts, hipStream_t s) {
  hipLaunchKernelGGL(dense_init_kernel, dim3(grid_for((int64_t)L.W * L.H, 256)), dim3(256), 0, s,
                     st, L, ix, iy, counts);
  return hipGetLastError();
}

hipError_t launch_dense_step(const uint8_t *cur, uint8_t *nxt, const LandscapeDev &L,
                             const double *beta, uint32_t sim_index, uint32_t step, uint32_t k0,
                             uint32_t k1, unsigned long long *counts, hipStream_t s) {
  const int64_t n = (int64_t)L.W * L.H;
  hipLaunchKernelGGL(dense_step_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cur,
                     nxt, L, beta, sim_index, step, k0, k1, counts);
  return hipGetLastError();
}

hipError_t launch_dense_result(const uint8_t *st, const LandscapeDev &L, const uint32_t *ref,
                               uint32_t n_ref, bool has_target, uint32_t steps,
                               const unsigned long long *counts, fire_result *out,
                               uint32_t *map, hipStream_t s) {
  hipLaunchKernelGGL(dense_result_kernel, dim3(1), dim3(kDenseResThreads), 0, s, st, L, ref, n_ref,
                     has_target ? 1 : 0, steps, counts, out, map);
  return hipGetLastError();
}

hipError_t launch_set_life(uint4 *rec, int64_t n, const uint8_t *steps, hipStream_t s) {
  hipLaunchKernelGGL(set_life_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, rec, n, steps);
  return hipGetLastError();
}

hipError_t launch_zero_words(uint32_t *p0, uint32_t *p1, uint32_t *p2, hipStream_t s) {
  hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, p0, p1, p2);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s,
                     p, v, n);
  return hipGetLastError();
}

// Scratch of the no-allocation entry point (fire_run_dev_noalloc): its work
// counters, re-run list and frontier spill area, in a file-scope device
// array; every GPU the library runs on holds its own copy until the process
// ends. Host code uses the address hipGetSymbolAddress returns for the
// current device (noalloc_scratch), never the array's name.
static __device__ __align__(256) uint32_t scratch[kNoAllocScratchWords];

hipError_t noalloc_scratch(uint32_t **ptr) {
  static std::mutex mu;
  static std::map<int, uint32_t *> addr;  // device -> address of its copy
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    it = addr.emplace(dev, static_cast<uint32_t *>(p)).first;
  }
  *ptr = it->second;
  return hipSuccess;
}

hipError_t launch_simw(const SimArgs &a, bool table, int grid, size_t lds, hipStream_t s) {
  const bool win = a.win > 0;
  if (a.retry == nullptr) return hipErrorInvalidValue;
  if (table) {
    if (win) hipLaunchKernelGGL((simw_kernel<true, true>), dim3(grid), dim3(kWave), lds, s, a);
    else hipLaunchKernelGGL((simw_kernel<true, false>), dim3(grid), dim3(kWave), lds, s, a);
  } else {
    if (win) hipLaunchKernelGGL((simw_kernel<false, true>), dim3(grid), dim3(kWave), lds, s, a);
    else hipLaunchKernelGGL((simw_kernel<false, false>), dim3(grid), dim3(kWave), lds, s, a);
  }
  return hipGetLastError();
}

size_t simw_lds_bytes(int bitset_words, int queue_cap) {
  return sizeof(uint32_t) * (size_t)simw_lds_words(bitset_words, queue_cap);
}

int simw_occupancy(bool table, bool win, size_t lds_bytes) {
  int n = 0;
  hipError_t e;
  if (table)
    e = win ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, simw_kernel<true, true>, kWave, lds_bytes)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, simw_kernel<true, false>, kWave, lds_bytes);
  else
    e = win ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, simw_kernel<false, true>, kWave, lds_bytes)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, simw_kernel<false, false>, kWave, lds_bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

size_t simw_scratch_bytes(bool table, bool win) {
  hipFuncAttributes at{};
  const void *f = table ? (win ? reinterpret_cast<const void *>(&simw_kernel<true, true>)
                               : reinterpret_cast<const void *>(&simw_kernel<true, false>))
                        : (win ? reinterpret_cast<const void *>(&simw_kernel<false, true>)
                               : reinterpret_cast<const void *>(&simw_kernel<false, false>));
  if (hipFuncGetAttributes(&at, f) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return at.localSizeBytes;
}

template <int BLOCK, bool TABLE, bool DUR>
static void launch_one(const SimArgs &a, bool win, int grid, size_t lds, hipStream_t s) {
  if (win)
    hipLaunchKernelGGL((sim_kernel<BLOCK, TABLE, DUR, true>), dim3(grid), dim3(BLOCK), lds, s, a);
  else if (a.gbits)
    hipLaunchKernelGGL((sim_kernel<BLOCK, TABLE, DUR, false, true>), dim3(grid), dim3(BLOCK), lds,
                       s, a);
  else
    hipLaunchKernelGGL((sim_kernel<BLOCK, TABLE, DUR, false>), dim3(grid), dim3(BLOCK), lds, s, a);
}

template <int BLOCK>
static hipError_t launch_sim_block(const SimArgs &a, bool table, bool dur, int grid,
                                   size_t lds, hipStream_t s) {
  const bool win = a.win > 0;
  if (dur) {
    if (table) launch_one<BLOCK, true, true>(a, win, grid, lds, s);
    else launch_one<BLOCK, false, true>(a, win, grid, lds, s);
  } else {
    if (table) launch_one<BLOCK, true, false>(a, win, grid, lds, s);
    else launch_one<BLOCK, false, false>(a, win, grid, lds, s);
  }
  return hipGetLastError();
}

template <int BLOCK, bool TABLE, bool DUR>
static int occupancy_one(size_t lds, bool win, bool gb) {
  int n = 0;
  hipError_t e = win  ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &n, sim_kernel<BLOCK, TABLE, DUR, true>, BLOCK, lds)
                 : gb ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &n, sim_kernel<BLOCK, TABLE, DUR, false, true>, BLOCK, lds)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &n, sim_kernel<BLOCK, TABLE, DUR, false>, BLOCK, lds);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

template <int BLOCK>
static int occupancy_block(bool table, bool dur, bool win, bool gb, size_t lds) {
  if (dur) return table ? occupancy_one<BLOCK, true, true>(lds, win, gb)
                        : occupancy_one<BLOCK, false, true>(lds, win, gb);
  return table ? occupancy_one<BLOCK, true, false>(lds, win, gb)
               : occupancy_one<BLOCK, false, false>(lds, win, gb);
}

template <int BLOCK, bool TABLE, bool DUR>
static size_t scratch_one(bool win, bool gb) {
  hipFuncAttributes at{};
  const void *f =
      win  ? reinterpret_cast<const void *>(&sim_kernel<BLOCK, TABLE, DUR, true>)
      : gb ? reinterpret_cast<const void *>(&sim_kernel<BLOCK, TABLE, DUR, false, true>)
           : reinterpret_cast<const void *>(&sim_kernel<BLOCK, TABLE, DUR, false>);
  hipError_t e = hipFuncGetAttributes(&at, f);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return at.localSizeBytes;
}

template <int BLOCK>
static size_t scratch_block(bool table, bool dur, bool win, bool gb) {
  if (dur) return table ? scratch_one<BLOCK, true, true>(win, gb)
                        : scratch_one<BLOCK, false, true>(win, gb);
  return table ? scratch_one<BLOCK, true, false>(win, gb) : scratch_one<BLOCK, false, false>(win, gb);
}

size_t sim_scratch_bytes(int threads, bool table, bool dur, bool win, bool gb) {
  switch (threads) {
    case 64: return scratch_block<64>(table, dur, win, gb);
    case 128: return scratch_block<128>(table, dur, win, gb);
    case 256: return scratch_block<256>(table, dur, win, gb);
    case 512: return scratch_block<512>(table, dur, win, gb);
    case 1024: return scratch_block<1024>(table, dur, win, gb);
    default: return 0;
  }
}

int sim_occupancy(int threads, bool table, bool dur, bool win, size_t lds_bytes, bool gb) {
  switch (threads) {
    case 64: return occupancy_block<64>(table, dur, win, gb, lds_bytes);
    case 128: return occupancy_block<128>(table, dur, win, gb, lds_bytes);
    case 256: return occupancy_block<256>(table, dur, win, gb, lds_bytes);
    case 512: return occupancy_block<512>(table, dur, win, gb, lds_bytes);
    case 1024: return occupancy_block<1024>(table, dur, win, gb, lds_bytes);
    default: return 0;
  }
}

hipError_t launch_sim(const SimArgs &a, int threads, bool table, bool dur, int grid,
                      size_t lds_bytes, hipStream_t s) {
  if (dur && a.ovf_life == nullptr) return hipErrorInvalidValue;
  if (a.win > 0 && a.retry == nullptr) return hipErrorInvalidValue;
  switch (threads) {
    case 64: return launch_sim_block<64>(a, table, dur, grid, lds_bytes, s);
    case 128: return launch_sim_block<128>(a, table, dur, grid, lds_bytes, s);
    case 256: return launch_sim_block<256>(a, table, dur, grid, lds_bytes, s);
    case 512: return launch_sim_block<512>(a, table, dur, grid, lds_bytes, s);
    case 1024: return launch_sim_block<1024>(a, table, dur, grid, lds_bytes, s);
    default: return hipErrorInvalidValue;
  }
}

template <int BLOCK, bool TABLE, bool DUR>
static hipError_t set_limit_one(size_t bytes) {
  hipError_t e = hipFuncSetAttribute(
      reinterpret_cast<const void *>(&sim_kernel<BLOCK, TABLE, DUR, false>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void *>(&sim_kernel<BLOCK, TABLE, DUR, false, true>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&sim_kernel<BLOCK, TABLE, DUR, true>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int BLOCK>
static hipError_t set_limit_block(size_t bytes) {
  hipError_t e;
  if ((e = set_limit_one<BLOCK, true, false>(bytes)) != hipSuccess) return e;
  if ((e = set_limit_one<BLOCK, false, false>(bytes)) != hipSuccess) return e;
  if ((e = set_limit_one<BLOCK, true, true>(bytes)) != hipSuccess) return e;
  return set_limit_one<BLOCK, false, true>(bytes);
}

hipError_t set_sim_lds_limit(size_t bytes) {
  hipError_t e;
  const void *wk[4] = {reinterpret_cast<const void *>(&simw_kernel<true, true>),
                       reinterpret_cast<const void *>(&simw_kernel<true, false>),
                       reinterpret_cast<const void *>(&simw_kernel<false, true>),
                       reinterpret_cast<const void *>(&simw_kernel<false, false>)};
  for (const void *f : wk)
    if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) !=
        hipSuccess)
      return e;
  if ((e = set_limit_block<64>(bytes)) != hipSuccess) return e;
  if ((e = set_limit_block<128>(bytes)) != hipSuccess) return e;
  if ((e = set_limit_block<256>(bytes)) != hipSuccess) return e;
  if ((e = set_limit_block<512>(bytes)) != hipSuccess) return e;
  return set_limit_block<1024>(bytes);
}

GeneBox uniform_box(double lo, double hi, double h) {
  GeneBox b;
  for (int j = 0; j < kMaxGenes; ++j) {
    b.lo[j] = lo;
    b.hi[j] = hi;
    b.h[j] = h;
  }
  return b;
}

hipError_t launch_sims_from_pop(const double *pop, int P, int G, int R,
                                int32_t landscape_id, int32_t target_id, int W,
                                int H, uint32_t gen, const uint32_t *gen_ptr, fire_sim *sims,
                                double *betas, hipStream_t s) {
  hipLaunchKernelGGL(sims_from_pop_kernel, dim3(grid_for((int64_t)P * R, 256)), dim3(256), 0, s,
                     pop, P, G, R, landscape_id, target_id, W, H, gen, gen_ptr, sims, betas);
  return hipGetLastError();
}

hipError_t launch_ga_step(double *pop, const double *fit, double *mean_fit,
                          int P, int G, int R, int elite, double pm0,
                          const GeneBox &box, uint32_t gen,
                          uint32_t *gen_ptr, uint32_t generations,
                          uint32_t key0, uint32_t key1, hipStream_t s) {
  const int threads = ((P + 63) / 64) * 64;
  const size_t lds = ga_step_lds(P, G);
  hipLaunchKernelGGL(ga_step_kernel, dim3(1), dim3(threads), lds, s, pop, pop, (int64_t)0,
                     (uint64_t)0, fit, mean_fit, P, G, R, elite, pm0, box, gen, gen_ptr,
                     generations, key0, key1);
  return hipGetLastError();
}

hipError_t launch_ga_offspring(const double *pop, const double *fit, int P, int G, int R,
                               int elite, double pm0, const GeneBox &box, uint32_t gen,
                               uint32_t generations, uint64_t seed, uint64_t seed_step,
                               int n_sets, double *out_sets, hipStream_t s) {
  const int threads = ((P + 63) / 64) * 64;
  const size_t lds = ga_step_lds(P, G);
  hipLaunchKernelGGL(ga_step_kernel, dim3(n_sets), dim3(threads), lds, s, pop, out_sets,
                     (int64_t)P * G, seed_step, fit, nullptr, P, G, R, elite, pm0, box, gen,
                     nullptr, generations, (uint32_t)seed, (uint32_t)(seed >> 32));
  return hipGetLastError();
}

hipError_t launch_ga_prepare(const uint32_t *gen_ptr, fire_sim *sims, int P,
                             int R, uint32_t *work, const double *pop, int G,
                             double *hist_pop, hipStream_t s) {
  hipLaunchKernelGGL(ga_prepare_kernel, dim3(grid_for((int64_t)P * R, 256)),
                     dim3(256), 0, s, gen_ptr, sims, P, R, work, pop, G,
                     hist_pop);
  return hipGetLastError();
}

hipError_t launch_ga_gather(const uint32_t *gen_ptr, const fire_result *res,
                            int P, int R, double *fit, double *hist_fit,
                            hipStream_t s) {
  hipLaunchKernelGGL(ga_gather_kernel, dim3(grid_for((int64_t)P * R, 256)),
                     dim3(256), 0, s, gen_ptr, res, P, R, fit, hist_fit);
  return hipGetLastError();
}

hipError_t launch_ensemble(const double *params, const double *deltas, int N,
                           int G, int R, double cutoff, int32_t *out_best,
                           int32_t *out_n, double *out_mean, double *out_sd,
                           hipStream_t s) {
  hipLaunchKernelGGL(ensemble_kernel, dim3(1), dim3(kRedThreads), 0, s, params,
                     deltas, N, G, R, cutoff, out_best, out_n, out_mean,
                     out_sd);
  return hipGetLastError();
}

hipError_t launch_scan_reduce(const double *deltas, int n_cand, int R,
                              double cutoff, double tau, double *out_mean,
                              double *out_sd, double *out_accept,
                              double *out_post, hipStream_t s) {
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(1), dim3(kRedThreads), 0, s,
                     deltas, n_cand, R, cutoff, tau, out_mean, out_sd,
                     out_accept, out_post);
  return hipGetLastError();
}

}  // namespace firegpu
