// Internal declarations shared by the host ABI layer and the kernel file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fire.h"

namespace firegpu {

constexpr int kMaxDim = 4096;          // 12-bit x and y in frontier entries
constexpr uint32_t kSaturated = 0xFFFFFFFFu;

// Device-side landscape entry (one per loaded landscape id).
struct LandscapeDev {
  int32_t W, H, stride, valid;  // stride = ceil(W/32) words per bitset row
  const uint4 *rec;             // [H*W] {slope f32, aspect f32, wind f32,
                                //        veg | up_mask << 8 | turn-off << 16}
  const double *ps;             // [H*W][2] binary64: psi, slope / 100 of each cell
  const double *omega;          // [H*W][8] binary64: omega of each cell as the
                                // target of an edge in direction 0..7
  const uint32_t *blocked;      // [H*stride] 1 = non-burnable or padding
  const uint8_t *burn_steps;    // NULL (one step for every type) or [256]
                                // active steps of a burning cell by veg value
  uint32_t forest_class;
  uint32_t pad0;
};

struct TargetDev {
  int32_t landscape_id, valid;
  uint32_t n_ref, pad0;
  const uint32_t *bits;  // [H*stride]
};

struct SimArgs {
  const LandscapeDev *ls;
  int32_t n_ls;
  const TargetDev *tg;
  int32_t n_tg;
  const double *betas;
  int32_t n_params;
  const fire_sim *sims;
  const uint32_t *order;   // NULL, or the n_sims indices into sims[] to run
  int32_t n_sims;
  uint32_t key0, key1;
  const uint32_t *tables;  // NULL or [n_params][table_stride]
  int64_t table_stride;
  int32_t table_ls;        // landscape the tables belong to
  fire_result *out;
  uint32_t *maps;
  int64_t map_words;
  uint32_t *work;          // work-stealing counter (zeroed before launch)
  uint32_t *error_flag;    // set to 1 on an invalid descriptor
  uint32_t *ovf;           // per workgroup: 2 * ovf_cap frontier entries
  uint8_t *ovf_life;       // turn-off-time kernels: per workgroup 2 * ovf_cap
                           // remaining-life bytes of the spilled entries
  int64_t ovf_cap;
  int32_t queue_cap;       // frontier entries per queue held in LDS
  int32_t bitset_words;    // words of the burn bitset: in LDS, or per workgroup in gbits
  uint32_t *gbits;         // NULL (bitset in LDS), or [gridDim][bitset_words] in global
                           // memory for lattices whose bitset does not fit LDS (no window)
  int32_t win;             // 0, or the side (cells, multiple of 32) of the
                           // LDS window a simulation runs in
  uint32_t *retry;         // window runs: [0] count, [1..] simulations whose
                           // fire reached the window edge
  const uint32_t *n_dev;   // NULL, or the device count of simulations (else n_sims)
  uint32_t *stat_out;      // NULL, or a host-mapped word that receives *n_dev
  uint64_t *times;         // NULL, or per simulation i < times_cap: [2i] wall clock
  int64_t times_cap;       // when a workgroup took it, [2i + 1] when its result was
                           // written (100 MHz ticks)
};

// Launchers (fire_kernels.hip). Each returns the hipError_t of its launch.
hipError_t launch_preprocess(const uint8_t *veg, const float *elev,
                             const float *slope, const float *aspect,
                             const float *wind, int W, int H, int stride,
                             uint4 *rec, double *ps, double *omega, uint32_t *blocked,
                             hipStream_t s);
hipError_t launch_thresholds(const LandscapeDev *ls_dev_entry, int W, int H,
                             const double *beta_dev, uint32_t forest,
                             uint32_t *out, hipStream_t s);
// one table per parameter vector (betas_dev [n_params][5]), table p at
// out + p * out_stride
hipError_t launch_thresholds_multi(const LandscapeDev *ls_dev_entry, int W, int H,
                                   const double *betas_dev, int n_params, uint32_t forest,
                                   uint32_t *out, int64_t out_stride, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_zero_words(uint32_t *p0, uint32_t *p1, uint32_t *p2, hipStream_t s);
hipError_t launch_set_life(uint4 *rec, int64_t n, const uint8_t *steps, hipStream_t s);
hipError_t launch_sim(const SimArgs &a, int threads, bool table, bool dur, int grid,
                      size_t lds_bytes, hipStream_t s);
hipError_t set_sim_lds_limit(size_t bytes);
// Device scratch of the no-allocation entry point: kNoAllocScratchWords
// words per GPU (64 MiB), a file-scope array in fire_kernels.hip. `ptr`
// receives the current device's copy (looked up once per device).
constexpr size_t kNoAllocScratchWords = (size_t)16 << 20;
hipError_t noalloc_scratch(uint32_t **ptr);
// wavefront-per-simulation kernel (one 64-lane workgroup per simulation,
// LDS-only queues; a.retry receives the simulations it could not finish)
hipError_t launch_simw(const SimArgs &a, bool table, int grid, size_t lds, hipStream_t s);
size_t simw_lds_bytes(int bitset_words, int queue_cap);
int simw_occupancy(bool table, bool win, size_t lds_bytes);
size_t simw_scratch_bytes(bool table, bool win);
// workgroups of the simulation kernel resident per compute unit for this
// launch shape (registers and LDS), 0 if unknown
int sim_occupancy(int threads, bool table, bool dur, bool win, size_t lds_bytes,
                  bool gb = false);
// per-lane scratch (register spills) of a simulation-kernel variant, bytes
size_t sim_scratch_bytes(int threads, bool table, bool dur, bool win, bool gb = false);
// per-cell (paper-style) ablation path
hipError_t launch_dense_init(uint8_t *st, const LandscapeDev &L, int ix, int iy,
                             unsigned long long *counts, hipStream_t s);
hipError_t launch_dense_step(const uint8_t *cur, uint8_t *nxt, const LandscapeDev &L,
                             const double *beta, uint32_t sim_index, uint32_t step, uint32_t k0,
                             uint32_t k1, unsigned long long *counts, hipStream_t s);
hipError_t launch_dense_result(const uint8_t *st, const LandscapeDev &L, const uint32_t *ref,
                               uint32_t n_ref, bool has_target, uint32_t steps,
                               const unsigned long long *counts, fire_result *out,
                               uint32_t *map, hipStream_t s);
constexpr int kMaxGenes = 16;
// per-gene clamp box and mutation half-width
struct GeneBox {
  double lo[kMaxGenes], hi[kMaxGenes], h[kMaxGenes];
};
GeneBox uniform_box(double lo, double hi, double h);
// LDS of the one-workgroup GA step: means, old and new population, ranking
inline size_t ga_step_lds(int P, int G) {
  return sizeof(double) * ((size_t)P + 2 * (size_t)P * G) + sizeof(int) * (size_t)P;
}

hipError_t launch_ga_step(double *pop, const double *fit, double *mean_fit,
                          int P, int G, int R, int elite, double pm0,
                          const GeneBox &box, uint32_t gen,
                          uint32_t *gen_ptr, uint32_t generations,
                          uint32_t key0, uint32_t key1, hipStream_t s);
hipError_t launch_ga_offspring(const double *pop, const double *fit, int P, int G, int R,
                               int elite, double pm0, const GeneBox &box, uint32_t gen,
                               uint32_t generations, uint64_t seed, uint64_t seed_step,
                               int n_sets, double *out_sets, hipStream_t s);
hipError_t launch_sims_from_pop(const double *pop, int P, int G, int R,
                                int32_t landscape_id, int32_t target_id, int W,
                                int H, uint32_t gen, const uint32_t *gen_ptr,
                                fire_sim *sims, double *betas, hipStream_t s);
hipError_t launch_ga_prepare(const uint32_t *gen_ptr, fire_sim *sims, int P,
                             int R, uint32_t *work, const double *pop, int G,
                             double *hist_pop, hipStream_t s);
hipError_t launch_ga_gather(const uint32_t *gen_ptr, const fire_result *res,
                            int P, int R, double *fit, double *hist_fit,
                            hipStream_t s);
hipError_t launch_ensemble(const double *params, const double *deltas, int N,
                           int G, int R, double cutoff, int32_t *out_best,
                           int32_t *out_n, double *out_mean, double *out_sd,
                           hipStream_t s);
hipError_t launch_scan_reduce(const double *deltas, int n_cand, int R,
                              double cutoff, double tau, double *out_mean,
                              double *out_sd, double *out_accept,
                              double *out_post, hipStream_t s);

}  // namespace firegpu
