// HIP kernels (gfx950) of the stochastic CA fire model of Denham & Laneri,
// arXiv 1701.03549: landscape preprocessing, Eq. 1 thresholds, the batched
// simulation kernel with the Eq. 2 fitness fused in, and the device-side
// operators of the parameter search (Appendix B genetic algorithm,
// accepted-ensemble statistics, ignition-scan reduction).
//
// Built with -ffp-contract=off: every binary64 + - * / below is a single
// correctly rounded operation, so the only floating-point differences from
// another IEEE implementation come from exp and cos.

#include <hip/hip_runtime.h>
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
    const uint32_t lo0 = 0xD2511F53u * c0;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo2 = 0xCD9E8D57u * c2;
    const uint32_t hi2 = __umulhi(0xCD9E8D57u, c2);
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
// vegetation, psi precomputed from its slope and aspect, omega from its wind
// direction against the edge's compass angle, sigma from its slope when it
// lies strictly higher than the source (bit d of its up mask).
__device__ __forceinline__ uint32_t quantise(double p) {
  if (!(p < 1.0)) return kSaturated;
  if (!(p > 0.0)) return 0u;
  const double scaled = rint(p * 4294967296.0);
  if (scaled >= 4294967295.0) return kSaturated;
  return (uint32_t)scaled;
}

__device__ __forceinline__ uint32_t edge_threshold(const double *beta,
                                                   uint4 rec_t, double psi_t,
                                                   int d, uint32_t forest) {
  const uint32_t veg = rec_t.w & 0xFFu;
  if (veg == 0) return 0u;
  const bool up = ((rec_t.w >> (8 + d)) & 1u) != 0;
  const double slope = (double)__uint_as_float(rec_t.x);
  const double wind = (double)__uint_as_float(rec_t.z);
  const double i_f = veg == forest ? 1.0 : 0.0;
  const double omega = cos((wind - 45.0 * (double)d) * kDegToRad);
  const double sigma = up ? slope / 100.0 : 0.0;
  double x = beta[0];
  x = x + beta[1] * i_f;
  x = x + beta[2] * psi_t;
  x = x + beta[3] * omega;
  x = x + beta[4] * sigma;
  return quantise(1.0 / (1.0 + exp(-x)));
}

// ---------------------------------------------------------------------------
// Landscape preprocessing: per-cell 16-byte record, aspect covariate and the
// packed non-burnable map (padding bits past W count as non-burnable).
__global__ void preprocess_kernel(const uint8_t *veg, const float *elev,
                                  const float *slope, const float *aspect,
                                  const float *wind, int W, int H, int stride,
                                  uint4 *rec, double *psi, uint32_t *blocked) {
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
    psi[c] = (double)sl > 5.0
                 ? cos(((double)aspect[c] - 315.0) * kDegToRad)
                 : 0.0;
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

// One thread per source cell writes its 8 thresholds (two 16-byte stores).
__global__ void thresholds_kernel(const LandscapeDev *lsd, int W, int H,
                                  const double *beta_dev, uint32_t forest,
                                  uint32_t *out) {
  const LandscapeDev L = *lsd;
  double beta[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) beta[i] = beta_dev[i];
  const int64_t n = (int64_t)W * H;
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(s % W), y = (int)(s / W);
    uint32_t t8[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      const int tx = x + kDx[d], ty = y + kDy[d];
      uint32_t v = 0;
      if (tx >= 0 && tx < W && ty >= 0 && ty < H) {
        const int64_t t = (int64_t)ty * W + tx;
        v = edge_threshold(beta, L.rec[t], L.psi[t], d, forest);
      }
      t8[d] = v;
    }
    uint4 *o = reinterpret_cast<uint4 *>(out + s * 8);
    o[0] = make_uint4(t8[0], t8[1], t8[2], t8[3]);
    o[1] = make_uint4(t8[4], t8[5], t8[6], t8[7]);
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
//   * each step runs in two phases separated by barriers. Phase 1 reads the
//     bitset only (so eligibility is judged against the burn state at the
//     start of the step), draws the coins of the eligible edges of every
//     frontier cell and stores the mask of successful directions in the
//     entry's top byte. Phase 2 sets the bits of the successful targets with
//     atomic ORs; the lane whose OR flipped a bit owns that new cell and
//     appends it to the next frontier (wave ballot prefix sums give the
//     offsets, one LDS atomic per wave reserves the space), counting it and
//     its overlap with the reference map for Eq. 2.
// Every coin is a pure function of (sim_index, step, source cell, direction)
// and ignition is an OR, so the burnt set, step count, trial count and
// fitness do not depend on thread order or on the schedule.
// ---------------------------------------------------------------------------

template <int BLOCK>
__device__ __forceinline__ uint32_t q_get(const uint32_t *lq, const uint32_t *gq,
                                          uint32_t cap, uint32_t i) {
  return i < cap ? lq[i] : gq[i - cap];
}

template <int BLOCK>
__device__ __forceinline__ void q_put(uint32_t *lq, uint32_t *gq, uint32_t cap,
                                      uint32_t i, uint32_t v) {
  if (i < cap) lq[i] = v;
  else gq[i - cap] = v;
}

__device__ __forceinline__ uint32_t lane_prefix(uint64_t ballot) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(ballot >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)ballot, 0u));
}

enum CtlSlot { kSim = 0, kLen0 = 1, kTrials = 4, kNew = 5, kInter = 6, kCtlWords = 8 };

template <int BLOCK, bool TABLE>
__global__ __launch_bounds__(BLOCK) void sim_kernel(SimArgs a) {
  extern __shared__ uint32_t lds[];
  uint32_t *const bits = lds;
  uint32_t *qa = lds + a.bitset_words;
  uint32_t *qb = qa + a.queue_cap;
  uint32_t *const ctl = qb + a.queue_cap;
  uint32_t *ga = a.ovf + (int64_t)blockIdx.x * 2 * a.ovf_cap;
  uint32_t *gb = ga + a.ovf_cap;
  const uint32_t cap = (uint32_t)a.queue_cap;
  const int tid = threadIdx.x;
  const int lane = tid & 63;

  for (;;) {
    if (tid == 0) ctl[kSim] = atomicAdd(a.work, 1u);
    __syncthreads();
    const uint32_t sim = ctl[kSim];
    if (sim >= (uint32_t)a.n_sims) break;
    const fire_sim sd = a.sims[sim];

    // -- descriptor checks (uniform over the workgroup) --------------------
    bool ok = sd.landscape_id >= 0 && sd.landscape_id < a.n_ls &&
              sd.param_index < (uint32_t)a.n_params;
    LandscapeDev L{};
    if (ok) {
      L = a.ls[sd.landscape_id];
      ok = L.valid && sd.ign_x >= 0 && sd.ign_x < L.W && sd.ign_y >= 0 &&
           sd.ign_y < L.H && L.H * L.stride <= a.bitset_words &&
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
        atomicOr(a.error_flag, 1u);
      }
      __syncthreads();
      continue;
    }

    const int W = L.W, H = L.H, stride = L.stride;
    const int words = H * stride;
    const int ix = sd.ign_x, iy = sd.ign_y;
    const bool burnable =
        ((L.blocked[iy * stride + (ix >> 5)] >> (ix & 31)) & 1u) == 0;
    if (!burnable) {
      // a non-burnable ignition burns nothing
      if (tid == 0) {
        fire_result r;
        r.burnt = 0; r.steps = 0; r.trials = 0;
        r.fitness = has_target ? 1.0 : __builtin_nan("");
        a.out[sim] = r;
      }
      if (a.maps != nullptr) {
        uint32_t *m = a.maps + (int64_t)sim * a.map_words;
        for (int w = tid; w < words; w += BLOCK) m[w] = 0u;
      }
      __syncthreads();
      continue;
    }

    // -- init: bitset = non-burnable map, ignition burnt -------------------
    for (int w = tid; w < words; w += BLOCK) bits[w] = L.blocked[w];
    if (tid == 0) {
      ctl[kLen0 + 0] = 0; ctl[kLen0 + 1] = 0; ctl[kLen0 + 2] = 0;
      ctl[kTrials] = 0; ctl[kNew] = 0; ctl[kInter] = 0;
    }
    __syncthreads();
    if (tid == 0) {
      bits[iy * stride + (ix >> 5)] |= 1u << (ix & 31);
      q_put<BLOCK>(qa, ga, cap, 0, (uint32_t)ix | ((uint32_t)iy << 12));
    }
    double beta[5];
    const double *bp = a.betas + (int64_t)sd.param_index * 5;
#pragma unroll
    for (int i = 0; i < 5; ++i) beta[i] = bp[i];
    const uint32_t *table =
        TABLE ? a.tables + (int64_t)sd.param_index * a.table_stride : nullptr;
    const uint32_t *tbits = has_target ? tg.bits : nullptr;
    __syncthreads();

    uint32_t *cur = qa, *nxt = qb, *gcur = ga, *gnxt = gb;
    uint32_t n_cur = 1, step = 0;
    uint32_t my_trials = 0, my_new = 0, my_inter = 0;
    const uint32_t max_steps = sd.max_steps;

    while (n_cur != 0 && step < max_steps) {
      const int nslot = kLen0 + (int)((step + 1) % 3);
      if (tid == 0) ctl[nslot] = 0;

      // -- phase 1: eligibility against the step-start state, coins -------
      for (uint32_t i = tid; i < n_cur; i += BLOCK) {
        const uint32_t e = q_get<BLOCK>(cur, gcur, cap, i);
        const int x = (int)(e & 0xFFFu), y = (int)((e >> 12) & 0xFFFu);
        uint32_t elig = 0;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
          const int tx = x + kDx[d], ty = y + kDy[d];
          if (tx >= 0 && tx < W && ty >= 0 && ty < H &&
              ((bits[ty * stride + (tx >> 5)] >> (tx & 31)) & 1u) == 0)
            elig |= 1u << d;
        }
        if (elig == 0) continue;
        my_trials += __popc(elig);
        const uint32_t s_lin = (uint32_t)(y * W + x);
        uint32_t succ = 0;
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          const uint32_t m = (elig >> (4 * g)) & 0xFu;
          if (m == 0) continue;
          const Words4 r = philox10(sd.sim_index, step, s_lin, (uint32_t)g,
                                    a.key0, a.key1);
          uint32_t thr[4];
          if (TABLE) {
            const uint4 t4 =
                reinterpret_cast<const uint4 *>(table + (int64_t)s_lin * 8)[g];
            thr[0] = t4.x; thr[1] = t4.y; thr[2] = t4.z; thr[3] = t4.w;
          } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              thr[k] = 0;
              if ((m >> k) & 1u) {
                const int d = 4 * g + k;
                const int64_t t = (int64_t)(y + kDy[d]) * W + (x + kDx[d]);
                thr[k] = edge_threshold(beta, L.rec[t], L.psi[t], d,
                                        L.forest_class);
              }
            }
          }
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const bool hit = ((m >> k) & 1u) &&
                             (thr[k] == kSaturated || r.v[k] < thr[k]);
            succ |= (hit ? 1u : 0u) << (4 * g + k);
          }
        }
        if (succ != 0) q_put<BLOCK>(cur, gcur, cap, i, e | (succ << 24));
      }
      __syncthreads();

      // -- phase 2: apply ignitions, compact the next frontier --------------
      for (uint32_t base = 0; base < n_cur; base += BLOCK) {
        const uint32_t i = base + (uint32_t)tid;
        const uint32_t e = i < n_cur ? q_get<BLOCK>(cur, gcur, cap, i) : 0u;
        uint32_t succ = e >> 24;
        const int x = (int)(e & 0xFFFu), y = (int)((e >> 12) & 0xFFFu);
        uint32_t newm = 0;
        while (succ) {
          const int d = __ffs(succ) - 1;
          succ &= succ - 1;
          const int tx = x + kDx[d], ty = y + kDy[d];
          const uint32_t bit = 1u << (tx & 31);
          const uint32_t old = atomicOr(&bits[ty * stride + (tx >> 5)], bit);
          if ((old & bit) == 0) newm |= 1u << d;
        }
        const uint32_t cnt = __popc(newm);
        uint32_t excl = 0, total = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const uint64_t bal = __ballot((cnt >> b) & 1u);
          excl += lane_prefix(bal) << b;
          total += (uint32_t)__popcll(bal) << b;
        }
        if (total != 0) {
          uint32_t wbase = 0;
          if (lane == 0) wbase = atomicAdd(&ctl[nslot], total);
          wbase = __builtin_amdgcn_readfirstlane(wbase);
          uint32_t pos = wbase + excl;
          while (newm) {
            const int d = __ffs(newm) - 1;
            newm &= newm - 1;
            const int tx = x + kDx[d], ty = y + kDy[d];
            q_put<BLOCK>(nxt, gnxt, cap, pos++, (uint32_t)tx | ((uint32_t)ty << 12));
            ++my_new;
            if (tbits != nullptr)
              my_inter += (tbits[ty * stride + (tx >> 5)] >> (tx & 31)) & 1u;
          }
        }
      }
      __syncthreads();
      n_cur = ctl[nslot];
      uint32_t *t0 = cur; cur = nxt; nxt = t0;
      uint32_t *t1 = gcur; gcur = gnxt; gnxt = t1;
      ++step;
    }

    // -- result: counts, Eq. 2, optional map --------------------------------
    if (my_trials) atomicAdd(&ctl[kTrials], my_trials);
    if (my_new) atomicAdd(&ctl[kNew], my_new);
    if (my_inter) atomicAdd(&ctl[kInter], my_inter);
    __syncthreads();
    if (tid == 0) {
      fire_result r;
      r.burnt = 1u + ctl[kNew];
      r.steps = step;
      r.trials = ctl[kTrials];
      if (has_target) {
        const uint32_t ign_in_ref = (tbits[iy * stride + (ix >> 5)] >> (ix & 31)) & 1u;
        const int64_t inter = (int64_t)ign_in_ref + ctl[kInter];
        const int64_t num = (int64_t)tg.n_ref + r.burnt - 2 * inter;
        r.fitness = (double)num / (double)tg.n_ref;
      } else {
        r.fitness = __builtin_nan("");
      }
      a.out[sim] = r;
    }
    if (a.maps != nullptr) {
      uint32_t *m = a.maps + (int64_t)sim * a.map_words;
      for (int w = tid; w < words; w += BLOCK) m[w] = bits[w] & ~L.blocked[w];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Genetic-algorithm generation (Appendix B): elitism, tournament of two,
// one-point crossover of consecutive non-elite pairs, dynamic mutation.
// One workgroup, thread i owns slot i. Only exact IEEE operations.
__global__ void ga_step_kernel(double *pop, const double *fit,
                               double *mean_fit, int P, int G, int R,
                               int elite, double pm0, double h, double lo,
                               double hi, uint32_t gen_arg,
                               uint32_t *gen_ptr, uint32_t generations,
                               uint32_t k0, uint32_t k1) {
  extern __shared__ double sh[];
  double *mean = sh;            // [P]
  double *oldp = sh + P;        // [P][G]
  double *newp = oldp + P * G;  // [P][G]
  int *order = reinterpret_cast<int *>(newp + P * G);  // [P]
  const uint32_t gen = gen_ptr ? *gen_ptr : gen_arg;
  const int i = threadIdx.x;

  if (i < P) {
    double acc = 0.0;
    for (int r = 0; r < R; ++r) acc = acc + fit[(int64_t)i * R + r];
    mean[i] = acc / (double)R;
    for (int j = 0; j < G; ++j) oldp[i * G + j] = pop[(int64_t)i * G + j];
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
          double g = newp[i * G + j] + h * (2.0 * u1 - 1.0);
          if (g < lo) g = lo;
          if (g > hi) g = hi;
          newp[i * G + j] = g;
        }
      }
    }
    for (int j = 0; j < G; ++j) pop[(int64_t)i * G + j] = newp[i * G + j];
    if (mean_fit) mean_fit[i] = mean[i];
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
                             uint4 *rec, double *psi, uint32_t *blocked,
                             hipStream_t s) {
  const int64_t n = (int64_t)W * H;
  hipLaunchKernelGGL(preprocess_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s,
                     veg, elev, slope, aspect, wind, W, H, stride, rec, psi,
                     blocked);
  return hipGetLastError();
}

hipError_t launch_thresholds(const LandscapeDev *ls_dev_entry, int W, int H,
                             const double *beta_dev, uint32_t forest,
                             uint32_t *out, hipStream_t s) {
  const int64_t n = (int64_t)W * H;
  hipLaunchKernelGGL(thresholds_kernel, dim3(grid_for(n, 256)), dim3(256), 0,
                     s, ls_dev_entry, W, H, beta_dev, forest, out);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s,
                     p, v, n);
  return hipGetLastError();
}

template <int BLOCK>
static hipError_t launch_sim_block(const SimArgs &a, bool table, int grid,
                                   size_t lds, hipStream_t s) {
  if (table)
    hipLaunchKernelGGL((sim_kernel<BLOCK, true>), dim3(grid), dim3(BLOCK), lds,
                       s, a);
  else
    hipLaunchKernelGGL((sim_kernel<BLOCK, false>), dim3(grid), dim3(BLOCK),
                       lds, s, a);
  return hipGetLastError();
}

hipError_t launch_sim(const SimArgs &a, int threads, bool table, int grid,
                      size_t lds_bytes, hipStream_t s) {
  switch (threads) {
    case 64: return launch_sim_block<64>(a, table, grid, lds_bytes, s);
    case 128: return launch_sim_block<128>(a, table, grid, lds_bytes, s);
    case 256: return launch_sim_block<256>(a, table, grid, lds_bytes, s);
    case 512: return launch_sim_block<512>(a, table, grid, lds_bytes, s);
    case 1024: return launch_sim_block<1024>(a, table, grid, lds_bytes, s);
    default: return hipErrorInvalidValue;
  }
}

template <int BLOCK>
static hipError_t set_limit_block(size_t bytes) {
  hipError_t e = hipFuncSetAttribute(
      reinterpret_cast<const void *>(&sim_kernel<BLOCK, true>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(
      reinterpret_cast<const void *>(&sim_kernel<BLOCK, false>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t set_sim_lds_limit(size_t bytes) {
  hipError_t e;
  if ((e = set_limit_block<64>(bytes)) != hipSuccess) return e;
  if ((e = set_limit_block<128>(bytes)) != hipSuccess) return e;
  if ((e = set_limit_block<256>(bytes)) != hipSuccess) return e;
  if ((e = set_limit_block<512>(bytes)) != hipSuccess) return e;
  return set_limit_block<1024>(bytes);
}

hipError_t launch_ga_step(double *pop, const double *fit, double *mean_fit,
                          int P, int G, int R, int elite, double pm0,
                          double h, double lo, double hi, uint32_t gen,
                          uint32_t *gen_ptr, uint32_t generations,
                          uint32_t key0, uint32_t key1, hipStream_t s) {
  const int threads = ((P + 63) / 64) * 64;
  const size_t lds = sizeof(double) * ((size_t)P + 2 * (size_t)P * G) +
                     sizeof(int) * (size_t)P;
  hipLaunchKernelGGL(ga_step_kernel, dim3(1), dim3(threads), lds, s, pop, fit,
                     mean_fit, P, G, R, elite, pm0, h, lo, hi, gen, gen_ptr,
                     generations, key0, key1);
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
