/*
 * fire.h -- C ABI of the MI355X (gfx950) library for the stochastic
 * cellular-automaton fire model of Denham & Laneri (arXiv 1701.03549).
 *
 * The library runs thousands of seeded fire simulations at once on one GPU,
 * scores each simulated burn map against a reference map (Eq. 2), and
 * provides the device-side operators of the parameter search that those
 * scores drive (genetic algorithm, ignition scan, ensemble statistics).
 *
 * Conventions used by every entry point
 * -------------------------------------
 * Lattice: W x H cells, row 0 is north, x grows east; cell (x, y) has
 *   linear index y*W + x. Cells outside the lattice are non-burnable.
 *   1 <= W, H <= 4096.
 * Directions d from a burning source to a target, with compass angle 45*d:
 *   d = 0 N (0,-1), 1 NE (+1,-1), 2 E (+1,0), 3 SE (+1,+1),
 *       4 S (0,+1), 5 SW (-1,+1), 6 W (-1,0),  7 NW (-1,-1).
 * Packed burn maps: uint32 words, row-major, ceil(W/32) words per row;
 *   cell (x, y) is bit x%32 of word y*ceil(W/32) + x/32; padding bits 0.
 * Threshold tables: uint32 T[(y*W + x)*8 + d] for the directed edge from
 *   source (x, y) in direction d; a coin r succeeds iff T == 0xFFFFFFFF or
 *   r < T (so T/2^32 is the spread probability, Eq. 1, quantised by
 *   round-half-even of p*2^32, saturating at 0xFFFFFFFF); T = 0 when the
 *   target is outside the lattice or non-burnable.
 * Coins: word (d % 4) of Philox4x32-10 (Salmon et al., SC'11; the
 *   generator the paper's CUDA-implementation section names) with counter
 *   (sim_index, step, y*W + x, d / 4) and key (seed low 32, seed high 32).
 * Memory: "host" pointers are ordinary CPU memory, "device" pointers are
 *   GPU memory of the context's device (e.g. a torch tensor's data_ptr()).
 *   The caller owns every buffer it passes; landscapes and targets are
 *   copied into context-owned device memory at load time.
 * Streams: `stream` is a hipStream_t (NULL = the null stream). Device work
 *   is enqueued on it and ordered with the caller's other work there;
 *   device buffers passed in must stay alive until that work completes.
 * Errors: every call returns a fire_status; nothing throws or aborts across
 *   the ABI. Argument checks run before any device work is enqueued, and a
 *   failing call leaves its outputs untouched. fire_last_error() describes
 *   the last failure of a context. Asynchronous device errors surface as
 *   FIRE_E_DEVICE at the next fire_sync().
 * Threads: a context is not thread-safe; use one per host thread.
 */
#ifndef FIRE_H_
#define FIRE_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fire_ctx fire_ctx; /* opaque */

typedef enum {
  FIRE_OK = 0,
  FIRE_E_INVALID = -1,     /* bad argument or unknown id                 */
  FIRE_E_OOM = -2,         /* device or host allocation failed           */
  FIRE_E_DEVICE = -3,      /* HIP runtime / kernel error                 */
  FIRE_E_UNSUPPORTED = -4  /* valid request the library cannot serve    */
} fire_status;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device`; *out receives the handle. */
fire_status fire_ctx_create(int device, fire_ctx **out);
/* Destroy a context and free every device object it owns (waits for the
 * device first). NULL is ignored. */
void fire_ctx_destroy(fire_ctx *ctx);
/* Text of the last failure on this context ("" if none). Owned by the
 * context, valid until its next call. */
const char *fire_last_error(const fire_ctx *ctx);
/* Wait for `stream` and report any asynchronous device error, including
 * descriptors rejected by device-side validation in fire_run_dev(). */
fire_status fire_sync(fire_ctx *ctx, void *stream);
/* Library version string, e.g. "1.0.0 gfx950". */
const char *fire_version(void);

/* ---- landscapes and reference maps (Methods, "Forest Fire Spread
 *      Simulation": vegetation, slope, aspect and wind rasters; Eq. 2's
 *      reference map A) ---------------------------------------------- */

typedef struct {
  int32_t width, height;     /* W, H                                     */
  float cell_m;              /* cell size in metres (informational)      */
  const uint8_t *veg;        /* [H][W] 0 = non-burnable, else burnable   */
  const float *elev_m;       /* [H][W] elevation; decides sigma's gate   */
  const float *slope_deg;    /* [H][W] slope in degrees                  */
  const float *aspect_deg;   /* [H][W] compass degrees the slope faces   */
  const float *wind_to_deg;  /* [H][W] compass degrees wind blows toward */
  uint8_t forest_class;      /* I_f = (veg == forest_class); 0 -> 1      */
  int32_t on_device;         /* 0: host pointers, 1: device pointers     */
} fire_landscape_desc;

/* Copy a landscape into the context and precompute its per-cell record
 * (raw covariate inputs, the 8-bit "target higher than source" mask, the
 * aspect covariate in binary64 and the packed non-burnable map).
 * FIRE_E_INVALID on W or H outside [1, 4096], NULL layers or a non-finite
 * value. Synchronous. *out_id receives a small non-negative id. */
fire_status fire_landscape_load(fire_ctx *ctx, const fire_landscape_desc *desc,
                                int32_t *out_id);
fire_status fire_landscape_free(fire_ctx *ctx, int32_t landscape_id);

/* Turn-off times (Methods: burnt cells are active or inactive, and a
 * burning cell turns inactive after a time set by its vegetation type; the
 * paper's results use one step for forest and shrubland). steps: NULL, or a
 * host array [256] where steps[v] is the number of consecutive steps a cell
 * of vegetation value v tries to ignite its unburnt neighbours after it
 * ignites (entry 0 is ignored; entries 1..255 must be >= 1, else
 * FIRE_E_INVALID). NULL or all ones restores the one-step model. Applies to
 * every later simulation on the landscape; waits for the device. */
fire_status fire_landscape_set_burn_steps(fire_ctx *ctx, int32_t landscape_id,
                                          const uint8_t *steps);

/* Copy a packed reference burn map (host pointer, H*ceil(W/32) words) for
 * landscape `landscape_id`. Padding bits are ignored. FIRE_E_INVALID when
 * the map is empty (Eq. 2 divides by |A|). Synchronous. */
fire_status fire_target_load(fire_ctx *ctx, int32_t landscape_id,
                             const uint32_t *bits, int32_t *out_target_id);
fire_status fire_target_free(fire_ctx *ctx, int32_t target_id);

/* ---- Eq. 1 thresholds ------------------------------------------------- */

/* Threshold table of landscape `landscape_id` under parameters beta[5]
 * (host, finite) into out_T (device, W*H*8 uint32, layout above), in
 * binary64: x = b0 + b1*I_f + b2*psi + b3*omega + b4*sigma summed left to
 * right without contraction, p = 1/(1+exp(-x)), with the covariates of the
 * target cell (psi = cos(aspect - 315 deg) if slope > 5 deg else 0;
 * omega = cos(wind_to - 45*d deg); sigma = slope/100 if the target is
 * strictly higher than the source else 0). Stream-ordered. */
fire_status fire_thresholds(fire_ctx *ctx, int32_t landscape_id,
                            const double beta[5], uint32_t *out_T,
                            void *stream);

/* As fire_thresholds, for n_params parameter vectors already on the device
 * (betas_dev: n_params x 5 binary64, row-major): table k goes to
 * out_T + k * W*H*8 (device, 16-byte aligned, n_params tables). One launch,
 * no host synchronisation and no allocation, so it can be captured into a
 * graph. The parameters are not checked on the host: a non-finite value
 * makes p NaN, which quantises to the saturated threshold (certain
 * ignition). FIRE_E_INVALID for a null pointer, n_params < 1, an unknown
 * landscape or a misaligned out_T. */
fire_status fire_thresholds_dev(fire_ctx *ctx, int32_t landscape_id, const double *betas_dev,
                                int32_t n_params, uint32_t *out_T, void *stream);

/* ---- simulations (Methods: propagation rules; Eq. 2 fitness) ---------- */

typedef struct {
  int32_t landscape_id;
  int32_t target_id;     /* -1: no reference map, fitness = NaN          */
  int32_t ign_x, ign_y;  /* ignition cell, inside the lattice            */
  uint32_t param_index;  /* row of betas[] (and of thresholds_override)  */
  uint32_t sim_index;    /* Philox counter word 0                        */
  uint32_t max_steps;    /* step cap; 0xFFFFFFFF = run to extinction     */
} fire_sim;              /* 28 bytes */

typedef struct {
  uint32_t burnt;   /* |A*|: burnt cells including the ignition          */
  uint32_t steps;   /* CA steps executed                                 */
  uint64_t trials;  /* coin draws: (burning source, unburnt burnable
                       in-lattice target) pairs over all steps           */
  double fitness;   /* Eq. 2: (|A| + |A*| - 2|A n A*|) / |A|, NaN
                       without target                                    */
} fire_result;      /* 24 bytes */

/* Run n_sims independent simulations. Each one: if the ignition cell is
 * non-burnable it burns nothing (burnt = steps = trials = 0, fitness 1.0
 * with a target). Otherwise the ignition burns at step 0; at every step
 * each cell that ignited at the previous step tries once, with its own
 * coin, to ignite each unburnt burnable neighbour, and a target ignites if
 * any of those coins succeeds; it stops when no cell ignited or after
 * max_steps steps.
 *   betas  host [n_params][5] binary64, finite
 *   sims   host [n_sims] descriptors (checked on the host)
 *   seed   Philox key
 *   thresholds_override  NULL, or device [n_params][W*H*8] tables to use
 *          instead of Eq. 1 (every sim must then use one landscape)
 *   out    device [n_sims] results, written in sims[] order
 *   out_maps  NULL, or device [n_sims][map_words] packed maps; sim i's
 *          map starts at out_maps + i*map_words
 *   map_words  words reserved per map; must be >= H*ceil(W/32) of every
 *          sim's landscape when out_maps != NULL
 * With one parameter vector, simulations are grouped by landscape (by
 * size when more than 8 landscapes are used) and each group runs as its
 * own persistent launch with LDS sized for it, on internal streams forked
 * from and joined back to `stream`. With several parameter vectors the
 * batch runs as one persistent launch whose simulations start in
 * decreasing order of expected fire size (burnable cells times the Eq. 1
 * probability averaged over the landscape's forest and other burnable
 * cells, each at the landscape's mean aspect and slope terms), so that
 * the longest fires do not start last. Results do not depend on the
 * schedule (threads, queue sizes, threshold mode), the grouping or the
 * order in which simulations run. Stream-ordered; calls on one context
 * must not overlap on different streams (they share staging and scratch
 * buffers). Not for stream capture: descriptors are staged through pinned
 * host memory that a graph would read at replay time, so under capture
 * this returns FIRE_E_UNSUPPORTED (use fire_run_dev).
 * Burn state: a simulation runs in one workgroup, whose LDS holds its
 * burn bitset (H*ceil(W/32) words, or a window of it) and two frontier
 * queues. A lattice whose whole bitset does not fit LDS (more than 40816
 * words with 160 KiB on gfx950, e.g. beyond 1024 x 1275 cells) keeps each
 * workgroup's bitset in global memory instead (at most 1 GiB of such
 * bitsets per launch, which bounds its resident simulations); results are
 * the same. */
fire_status fire_run(fire_ctx *ctx, const double *betas, int32_t n_params,
                     const fire_sim *sims, int32_t n_sims, uint64_t seed,
                     const uint32_t *thresholds_override, fire_result *out,
                     uint32_t *out_maps, int64_t map_words, void *stream);

/* Longest-expected-first order of a batch (host pointers, no device work):
 * out_order [n_sims] receives the indices of sims [n_sims] sorted by
 * decreasing expected fire size, the order fire_run starts a batch with
 * several parameter vectors in (burnable cells times the Eq. 1 probability
 * averaged over the landscape's forest and other burnable cells, each at
 * the landscape's mean aspect and slope terms; ties keep input order).
 * For fire_run_dev callers, e.g. a batch captured into a graph: upload the
 * descriptors in this order and row k of the results belongs to
 * sims[out_order[k]]. Results of a simulation do not depend on its place
 * in the batch. Descriptors are checked as by fire_run (FIRE_E_INVALID);
 * betas [n_params][5] must be finite. */
fire_status fire_order_sims(fire_ctx *ctx, const double *betas, int32_t n_params,
                            const fire_sim *sims, int32_t n_sims, int32_t *out_order);

/* Per-cell form of the simulation, after the paper's own kernel, kept as
 * an ablation and paper-style baseline of fire_run (CUDA-implementation
 * section; Methods, propagation rules): one thread per cell sweeps the
 * whole lattice every step, a burnable cell unburnt at the start of the
 * step with burning neighbours evaluates Eq. 1 for each of them (quantised
 * like an edge threshold), accumulates prod(1 - p_i) in binary64 in
 * direction order and draws one uniform (word 0 of Philox(sim_index, step,
 * y*W + x, 2) under `seed`) against 1 - prod; a saturated edge ignites
 * surely. The law of the burn equals fire_run's; the realisations differ.
 * Simulations run one after another, one launch per step, the host reading
 * the count of new cells after each step. trials = per-cell draws.
 * Arguments as fire_run (betas and sims on the host, out and out_maps on
 * the device); landscapes with turn-off times are FIRE_E_UNSUPPORTED.
 * Returns after every simulation's last step has been read back; the
 * results are written stream-ordered. */
fire_status fire_run_dense(fire_ctx *ctx, const double *betas, int32_t n_params,
                           const fire_sim *sims, int32_t n_sims, uint64_t seed,
                           fire_result *out, uint32_t *out_maps,
                           int64_t map_words, void *stream);

/* As fire_run, with betas and sims already in device memory (no host
 * staging). Descriptors are checked on the device: an invalid one yields
 * {0, 0xFFFFFFFF, 0, NaN} and makes the next fire_sync() return
 * FIRE_E_INVALID.
 * Stream capture: allowed once an identical call (same landscapes, batch
 * size and schedule) has run eagerly on this context, so that every
 * context scratch buffer (frontier spill area, retry list, threshold
 * tables) is already large enough; a call that would have to grow one
 * during capture returns FIRE_E_UNSUPPORTED. After a capture, buffers that
 * later calls outgrow are kept allocated (not freed) until
 * fire_ctx_destroy, so a captured graph stays valid for the context's
 * lifetime. Replays share the context's scratch with eager calls: keep
 * them stream-ordered with every other call on the context. */
fire_status fire_run_dev(fire_ctx *ctx, const double *betas_dev,
                         int32_t n_params, const fire_sim *sims_dev,
                         int32_t n_sims, uint64_t seed,
                         const uint32_t *thresholds_override,
                         fire_result *out, uint32_t *out_maps,
                         int64_t map_words, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * fire_run_dev, but every scratch buffer of the call (work counters, the
 * list of simulations run again, the frontier spill area) lives in one
 * 64 MiB device array that the library holds per GPU for the life of the
 * process, and the call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine). Thresholds come from thresholds_override or
 * are evaluated per trial (no context tables). The launch grids shrink so
 * that the spill area fits; a batch that cannot fit even one workgroup's
 * spill area (about 2 * W * H words for the largest loaded landscape, plus
 * n_sims + 65 words), or whose lattice needs its burn bitsets in global
 * memory (see fire_run), is rejected with FIRE_E_INVALID before any device
 * work. Every call on one GPU shares that GPU's array and leaves its
 * contents behind (counters are cleared by each call): calls that overlap
 * on one GPU, on any stream or context, race and must not be issued.
 * Results are identical to fire_run_dev's. */
fire_status fire_run_dev_noalloc(fire_ctx *ctx, const double *betas_dev,
                                 int32_t n_params, const fire_sim *sims_dev,
                                 int32_t n_sims, uint64_t seed,
                                 const uint32_t *thresholds_override,
                                 fire_result *out, uint32_t *out_maps,
                                 int64_t map_words, void *stream);

/* Per-simulation clocks, for load-balance analysis of the persistent
 * launches (not a passage of the paper: a diagnostic of the batch
 * scheduler). While set, every simulation launch of the context writes, for
 * batch index i < capacity, times_dev[2i] = the device's constant 100 MHz
 * wall clock when a workgroup took simulation i and times_dev[2i + 1] = the
 * clock when its result was written; a simulation that is run again over
 * the whole lattice (LDS windows) keeps the second run's pair. times_dev is
 * the caller's device buffer of 2 * capacity uint64 words, 8-byte aligned,
 * and must stay allocated while launches that use it run; launches already
 * captured into a graph keep the buffer they were captured with. NULL stops
 * the writes. FIRE_E_INVALID for capacity < 1 with a buffer. */
fire_status fire_set_sim_timing(fire_ctx *ctx, uint64_t *times_dev, int64_t capacity);

/* ---- schedule (autotuner hooks) --------------------------------------- */

typedef struct {
  int32_t threads;       /* workgroup size: 64, 128, 256, 512 or 1024     */
  int32_t queue_cap;     /* frontier entries kept in LDS per queue (>=64) */
  int32_t table_mode;    /* 1: precomputed threshold table per parameter,
                            0: thresholds evaluated per trial             */
  int32_t wg_per_cu;     /* persistent workgroups per compute unit (>=1)  */
  int32_t window;        /* -1: built-in choice; 0: every simulation keeps
                            the whole lattice's burn bitset in LDS; a
                            multiple of 32 in [64, 4096]: each simulation
                            first runs in an LDS window of that many cells
                            a side around its ignition, and one whose fire
                            comes within a cell of a window edge inside the
                            lattice is run again over the whole lattice
                            (same coins, so the same result); smaller LDS
                            footprints keep more simulations resident.
                            Ignored (whole lattice) with 1024 threads.    */
  int32_t wave;          /* 0: one simulation per workgroup of `threads`
                            lanes; 1: one simulation per 64-lane wavefront
                            (threads and wg_per_cu ignored) with its
                            frontier queues held in LDS only (queue_cap
                            entries each): its steps need no workgroup
                            barrier and draw coins only for units with an
                            eligible edge; a fire whose front outgrows
                            queue_cap (or a window) is run again by the
                            workgroup kernel over the whole lattice, with
                            the same coins and so the same result. The
                            built-in choice uses it for batches of at most
                            8 parameter vectors without turn-off times
                            while such re-runs stay absent.               */
} fire_schedule;

/* Fix the schedule used by later fire_run/fire_run_dev calls; NULL
 * restores the built-in choice. FIRE_E_INVALID when a field is out of
 * range or the LDS budget cannot hold it. */
fire_status fire_set_schedule(fire_ctx *ctx, const fire_schedule *s);
/* Schedule for one size class and kind of batch: runs whose landscapes
 * have between 2^(b-1)+1 and 2^b cells, b = ceil(log2(max_cells)), and
 * whose batch is of `kind` -- 0: at most 8 parameter vectors (replicate
 * batches); 1: more vectors with at least 8 simulations each (GA
 * populations); 2: other batches (Monte Carlo draws, random-parameter
 * batches) -- use `s` unless a fixed schedule is set; runs with turn-off
 * times keep the built-in choice. Its window and wave fields may be -1
 * (built-in choice). NULL removes the class entry. FIRE_E_INVALID for a
 * kind outside 0..2 or a field out of range. Used by the autotuner. */
fire_status fire_set_class_schedule(fire_ctx *ctx, int64_t max_cells, int32_t kind,
                                    const fire_schedule *s);
/* The schedule a batch of `n_sims` simulations with `n_params` parameter
 * vectors on a square lattice of `max_cells` cells would use (window: the
 * LDS window side of its first launch, 0 for none). */
fire_status fire_get_schedule(fire_ctx *ctx, int64_t max_cells,
                              int32_t n_params, int32_t n_sims,
                              fire_schedule *out);

/* ---- genetic algorithm (Appendix B) ----------------------------------- */

typedef struct {
  int32_t elite;         /* individuals copied unchanged (e.g. 2)         */
  double pm0;            /* mutation probability at generation 0          */
  double mut_h;          /* mutation step half-width                      */
  double lo, hi;         /* gene box, mutated genes are clamped to it     */
  uint32_t generations;  /* p_m(g) = pm0 * (1 - g / generations)          */
} fire_ga_cfg;

/* One generation in place on the device. pop: device [P][G] binary64,
 * replaced by the next population; fit: device [P][R] Eq. 2 values of the
 * current population; mean_fit: NULL or device [P], receives the mean
 * fitness (sum in replicate order / R). Fitness of an individual is its
 * mean; the `elite` best (ties by index) are kept; every other slot i is
 * the winner of a 2-tournament drawn from Philox counter (gen, i, 0, 0)
 * under key ga_seed (indices (out0*P)>>32 and (out1*P)>>32, lower fitness
 * wins, tie to lower index); non-elite slots elite+2k, elite+2k+1 swap
 * genes [c, G) with c = 1 + ((out0*(G-1))>>32), counter (gen, k, 1, 0);
 * gene j of non-elite slot i mutates iff out0*2^-32 < p_m(gen), counter
 * (gen, i, 2, j), by mut_h*(2*out1*2^-32 - 1), clamped to [lo, hi].
 * 1 <= P <= 1024, 2 <= G <= 16, R >= 1, and the population must fit the
 * LDS of one workgroup (8*(P + 2*P*G) + 4*P bytes <= the device's LDS per
 * workgroup, 160 KiB on gfx950). Stream-ordered. */
fire_status fire_ga_step(fire_ctx *ctx, double *pop, const double *fit,
                         double *mean_fit, int32_t P, int32_t G, int32_t R,
                         const fire_ga_cfg *cfg, uint32_t gen,
                         uint64_t ga_seed, void *stream);

/* Offspring sets of one parent population (Appendix B operators, as
 * fire_ga_step): set o of out_sets [n_sets][P][G] (device) is the
 * population fire_ga_step would make from pop and fit at generation gen
 * under seed ga_seed + o * seed_step (mod 2^64), with pop left unchanged;
 * used to draw several candidate offspring sets for screening in one
 * launch. out_sets must not overlap pop. 1 <= n_sets <= 1024; sizes and
 * configuration as fire_ga_step. Stream-ordered. */
fire_status fire_ga_offspring(fire_ctx *ctx, const double *pop, const double *fit,
                              int32_t P, int32_t G, int32_t R,
                              const fire_ga_cfg *cfg, uint32_t gen,
                              uint64_t ga_seed, uint64_t seed_step,
                              int32_t n_sets, double *out_sets, void *stream);

/* fire_ga_step with a box and a mutation half-width per gene (host arrays
 * lo[G], hi[G], h[G]); used when genes have different ranges, e.g. the
 * ignition cell carried as genes 5 and 6 (Appendix B: 7 parameters when
 * the ignition point is estimated). 2 <= G <= 16. */
fire_status fire_ga_step_genes(fire_ctx *ctx, double *pop, const double *fit,
                               double *mean_fit, int32_t P, int32_t G, int32_t R,
                               int32_t elite, double pm0, const double *lo,
                               const double *hi, const double *h,
                               uint32_t generations, uint32_t gen,
                               uint64_t ga_seed, void *stream);

/* Descriptors of one generation whose individuals carry their ignition as
 * genes 5 and 6 (device pop [P][G], G >= 7): out_sims [P*R] (device) with
 * sims[i*R + r] = {landscape_id, target_id, ignition (floor(g5 + 0.5),
 * floor(g6 + 0.5)) clamped to the lattice, param_index i, sim_index
 * (gen*P + i)*R + r, run to extinction}; out_betas [P][5] (device) = genes
 * 0..4. Stream-ordered. */
fire_status fire_ga_sims_from_pop(fire_ctx *ctx, const double *pop, int32_t P,
                                  int32_t G, int32_t R, int32_t landscape_id,
                                  int32_t target_id, uint32_t gen,
                                  fire_sim *out_sims, double *out_betas,
                                  void *stream);

/* A whole GA calibration on one landscape and reference map (5 genes, the
 * betas): for g in [0, generations): evaluate every individual by R
 * simulations (sim_index = (g*P + i)*R + r, ignition (ign_x, ign_y),
 * run to extinction), then fire_ga_step with gen = g. One generation is
 * captured once as a HIP graph and replayed.
 *   pop0      host [P][5] initial population
 *   hist_pop  device [generations][P][5]: population evaluated at g
 *   hist_fit  device [generations][P][R]: its Eq. 2 values
 * Stream-ordered; FIRE_E_UNSUPPORTED if graph capture fails. */
fire_status fire_ga_run(fire_ctx *ctx, int32_t landscape_id,
                        int32_t target_id, int32_t ign_x, int32_t ign_y,
                        const double *pop0, int32_t P, int32_t R,
                        const fire_ga_cfg *cfg, uint64_t sim_seed,
                        uint64_t ga_seed, double *hist_pop, double *hist_fit,
                        void *stream);

/* ---- ensemble statistics (Methods rules; Appendix D) ------------------ */

/* Accepted-ensemble statistics over N individuals with G parameters each
 * (device params [N][G]) evaluated by R simulations (device deltas [N][R]):
 * a simulation is accepted iff its fitness < cutoff; out_best (device,
 * int32[1]) = individual of the minimum single fitness (first on ties);
 * out_n (device, int32[1]) = accepted simulations; out_mean and out_sd
 * (device [G]) = mean and standard deviation (n-1 denominator, 0 if n<2)
 * of the parameters over the accepted simulations (each accepted
 * replicate counts its individual once). Stream-ordered. */
fire_status fire_ensemble(fire_ctx *ctx, const double *params,
                          const double *deltas, int32_t N, int32_t G,
                          int32_t R, double cutoff, int32_t *out_best,
                          int32_t *out_n, double *out_mean, double *out_sd,
                          void *stream);

/* A whole GA calibration with the ignition point estimated (Appendix B:
 * 7 parameters, beta[5] then the ignition x, y): as fire_ga_run, but each
 * generation's simulations start at the cell of the individual's genes 5
 * and 6 (floor(g + 0.5), clamped to the lattice; a non-burnable cell burns
 * nothing and scores 1). lo, hi, h: host arrays [7], the clamp box and
 * mutation half-width of each gene. pop0: host [P][7]; hist_pop: device
 * [generations][P][7]; hist_fit: device [generations][P][R]. Returns after
 * the last generation has finished. */
fire_status fire_ga_run_ignition(fire_ctx *ctx, int32_t landscape_id,
                                 int32_t target_id, const double *pop0,
                                 int32_t P, int32_t R, int32_t elite,
                                 double pm0, uint32_t generations,
                                 const double *lo, const double *hi,
                                 const double *h, uint64_t sim_seed,
                                 uint64_t ga_seed, double *hist_pop,
                                 double *hist_fit, void *stream);

/* Ignition-scan reduction (Methods: ignition points; cutoff rule of the
 * CUDA-implementation section) over device deltas [n_cand][R]: per
 * candidate the mean, standard deviation (n-1) and acceptance rate
 * #(delta < cutoff)/R, and a map acceptance/sum(acceptance), or, when no
 * replicate is accepted anywhere, exp(-(mean - min mean)/tau) normalised
 * to 1. All outputs device [n_cand] binary64. Stream-ordered. */
fire_status fire_scan_reduce(fire_ctx *ctx, const double *deltas,
                             int32_t n_cand, int32_t R, double cutoff,
                             double tau, double *out_mean, double *out_sd,
                             double *out_accept, double *out_post,
                             void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FIRE_H_ */
