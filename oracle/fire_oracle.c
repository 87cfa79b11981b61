/*
 * CPU oracle for the stochastic cellular-automaton fire model of Denham &
 * Laneri, "Using efficient parallelization in Graphic Processing Units to
 * parameterize stochastic fire propagation models" (arXiv 1701.03549).
 *
 * TEST INFRASTRUCTURE. This is the plain, slow, obviously-correct reference
 * that the GPU library is checked against. Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it; the product
 * library never links, includes or calls anything here, and nothing here is
 * taken from the GPU sources.
 *
 * Floating point: IEEE binary64 everywhere (the paper fixes no precision).
 * Build with -ffp-contract=off and without fast-math so that every + - * /
 * below is exactly one correctly rounded operation; exp and cos come from
 * the host libm.
 *
 * Readings of the paper that the code below fixes (the paper is silent or
 * garbled on these points):
 *   - Grid: row 0 is north, x grows east; cell (x, y) has linear index
 *     y*W + x. Cells outside the lattice are treated as non-burnable.
 *   - The 8 directions d, from a burning source to its target:
 *       d : 0   1   2   3   4   5   6   7
 *           N   NE  E   SE  S   SW  W   NW
 *       dx: 0  +1  +1  +1   0  -1  -1  -1
 *       dy:-1  -1   0  +1  +1  +1   0  -1
 *     and the compass angle of the source->target direction is 45*d degrees.
 *   - Every covariate of Eq. 1 is taken at the TARGET cell; the wind map
 *     holds the compass direction the wind blows toward; sigma uses the
 *     target's slope in degrees divided by 100 when the target is strictly
 *     higher than the source; psi is 0 when the slope is 5 degrees or less.
 *   - The garbled ignition rule (one minus a product over burning
 *     neighbours) is realised by one independent coin per directed edge
 *     (burning source, unburnt target): the target ignites if any coin
 *     succeeds, which gives exactly 1 - prod(1 - p_i).
 *   - A cell burns for exactly one step, so each directed edge is tried at
 *     most once.
 *   - The uniform in [0, 1] is a 32-bit Philox output compared against
 *     p quantised to 32 bits (see quantise_p below).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Philox4x32-10: the counter-based generator of Salmon, Moraes, Dror and
 * Shaw (SC'11, "Parallel random numbers: as easy as 1, 2, 3"), the
 * generator the paper names in its CUDA implementation section. One call
 * maps a 128-bit counter and a 64-bit key to 128 random bits by ten
 * rounds; each round multiplies counter words 0 and 2 by two fixed
 * odd constants, mixes the high halves with words 1 and 3 and the key,
 * and the key is advanced by two Weyl constants between rounds.          */

static const uint32_t PHILOX_MUL_A = 0xD2511F53u;  /* multiplies word 0 */
static const uint32_t PHILOX_MUL_B = 0xCD9E8D57u;  /* multiplies word 2 */
static const uint32_t PHILOX_WEYL_A = 0x9E3779B9u; /* golden ratio       */
static const uint32_t PHILOX_WEYL_B = 0xBB67AE85u; /* sqrt(3) - 1        */

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                          uint32_t out[4]) {
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_WEYL_A;
      k1 += PHILOX_WEYL_B;
    }
    uint64_t prod_a = (uint64_t)PHILOX_MUL_A * (uint64_t)c[0];
    uint64_t prod_b = (uint64_t)PHILOX_MUL_B * (uint64_t)c[2];
    uint32_t hi_a = (uint32_t)(prod_a >> 32), lo_a = (uint32_t)prod_a;
    uint32_t hi_b = (uint32_t)(prod_b >> 32), lo_b = (uint32_t)prod_b;
    uint32_t n0 = hi_b ^ c[1] ^ k0;
    uint32_t n1 = lo_b;
    uint32_t n2 = hi_a ^ c[3] ^ k1;
    uint32_t n3 = lo_a;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* ---------------------------------------------------------------------- */
/* Lattice geometry                                                        */

static const int DIR_DX[8] = {0, 1, 1, 1, 0, -1, -1, -1};
static const int DIR_DY[8] = {-1, -1, 0, 1, 1, 1, 0, -1};

static int in_lattice(int W, int H, int x, int y) {
  return x >= 0 && x < W && y >= 0 && y < H;
}

static double deg_to_rad(double a) { return a * (M_PI / 180.0); }

/* ---------------------------------------------------------------------- */
/* Covariates of Eq. 1 (Methods, "Forest Fire Spread Simulation").        */

/* I_f: 1 for a forest cell, 0 otherwise. */
static double cov_forest(uint8_t veg_t, uint8_t forest_class) {
  return veg_t == forest_class ? 1.0 : 0.0;
}

/* psi = cos(theta - 315 deg) for cells steeper than 5 degrees, theta the
 * aspect; 1 for a north-west facing cell, -1 for a south-east facing one. */
static double cov_aspect(float slope_t, float aspect_t) {
  if (!((double)slope_t > 5.0)) return 0.0;
  return cos(deg_to_rad((double)aspect_t - 315.0));
}

/* omega = cos(phi_w - phi_c): phi_w the wind direction at the target,
 * phi_c the direction from the burning cell to the target; 1 downwind. */
static double cov_wind(float wind_to_t, int d) {
  return cos(deg_to_rad((double)wind_to_t - 45.0 * (double)d));
}

/* sigma = slope / 100 when the target is higher than the source, else 0. */
static double cov_slope(float slope_t, float elev_t, float elev_s) {
  if (elev_t > elev_s) return (double)slope_t / 100.0;
  return 0.0;
}

/* Eq. 1: p = 1 / (1 + exp(-(b0 + b1 I_f + b2 psi + b3 omega + b4 sigma))),
 * the sum taken left to right. */
double oracle_spread_probability(const double beta[5], double i_f, double psi,
                                 double omega, double sigma) {
  double x = beta[0];
  x = x + beta[1] * i_f;
  x = x + beta[2] * psi;
  x = x + beta[3] * omega;
  x = x + beta[4] * sigma;
  return 1.0 / (1.0 + exp(-x));
}

/* p quantised to a 32-bit threshold T: a coin r (uniform on 0..2^32-1)
 * succeeds iff T == 0xFFFFFFFF or r < T, so T / 2^32 is the realised
 * probability. p * 2^32 is exact in binary64, so the only rounding is the
 * round-half-to-even of rint (default rounding mode). */
uint32_t oracle_quantise_p(double p) {
  if (!(p < 1.0)) return 0xFFFFFFFFu;
  if (!(p > 0.0)) return 0u;
  double scaled = rint(p * 4294967296.0);
  if (scaled >= 4294967295.0) return 0xFFFFFFFFu;
  return (uint32_t)scaled;
}

/* Threshold table T[(y*W + x)*8 + d] for the directed edge from source
 * (x, y) to its neighbour in direction d; 0 when the target lies outside
 * the lattice or is non-burnable (veg == 0). Returns 0 on success. */
int oracle_thresholds(int W, int H, const uint8_t *veg, const float *elev,
                      const float *slope, const float *aspect,
                      const float *wind_to, uint8_t forest_class,
                      const double beta[5], uint32_t *T) {
  if (W <= 0 || H <= 0) return -1;
  for (int y = 0; y < H; ++y) {
    for (int x = 0; x < W; ++x) {
      long s = (long)y * W + x;
      for (int d = 0; d < 8; ++d) {
        int tx = x + DIR_DX[d], ty = y + DIR_DY[d];
        uint32_t thr = 0;
        if (in_lattice(W, H, tx, ty)) {
          long t = (long)ty * W + tx;
          if (veg[t] != 0) {
            double p = oracle_spread_probability(
                beta, cov_forest(veg[t], forest_class),
                cov_aspect(slope[t], aspect[t]), cov_wind(wind_to[t], d),
                cov_slope(slope[t], elev[t], elev[s]));
            thr = oracle_quantise_p(p);
          }
        }
        T[s * 8 + d] = thr;
      }
    }
  }
  return 0;
}

/* ---------------------------------------------------------------------- */
/* One simulation (Methods, fire ignition and propagation rules).
 *
 * Cells are unburnable (veg == 0), burnable, burnt and active, or burnt and
 * inactive (the four states of the Methods). A cell that ignites is active
 * for burn_steps[veg] consecutive steps (its turn-off time, set by its
 * vegetation; the paper's results use 1 step for every type, which is what
 * burn_steps == NULL gives) and then inactive. At every step each active
 * cell tries each neighbour that is burnable and unburnt at the start of the
 * step once; the cells ignited during a step become active from the next
 * step on (synchronous update).
 *
 * The coin for the directed edge (source s -> direction d) tried at step k
 * of simulation sim_index is word (d mod 4) of
 *   Philox4x32-10(counter = (sim_index, k, s, d div 4),
 *                 key     = (seed mod 2^32, seed div 2^32)).
 * With static_edges != 0 the step word is forced to 0 (a test mode: every
 * directed edge then has one fixed coin, so the final burn equals the set
 * reachable from the ignition through open edges).
 *
 * Outputs: map_bits (optional, H rows of ceil(W/32) words, cell (x, y) is
 * bit x%32 of word y*ceil(W/32) + x/32), number of burnt cells, number of
 * steps executed (steps with at least one active cell, up to max_steps) and
 * number of coin trials. Returns 0 on success, -1 on a bad argument
 * (including a burn_steps entry of 0 for a vegetation value present in the
 * landscape), -2 on allocation failure.                                   */
int oracle_simulate(int W, int H, const uint8_t *veg, const uint32_t *T,
                    int ign_x, int ign_y, uint32_t sim_index, uint64_t seed,
                    uint32_t max_steps, int static_edges,
                    const uint8_t *burn_steps, uint32_t *map_bits,
                    uint32_t *out_burnt, uint32_t *out_steps,
                    uint64_t *out_trials) {
  if (W <= 0 || H <= 0 || !in_lattice(W, H, ign_x, ign_y)) return -1;
  long n = (long)W * H;
  long stride = (W + 31) / 32;
  if (burn_steps)
    for (long c = 0; c < n; ++c)
      if (veg[c] != 0 && burn_steps[veg[c]] == 0) return -1;
  if (map_bits) memset(map_bits, 0, sizeof(uint32_t) * stride * H);
  *out_burnt = 0;
  *out_steps = 0;
  *out_trials = 0;
  long ign = (long)ign_y * W + ign_x;
  if (veg[ign] == 0) return 0; /* a non-burnable ignition burns nothing */

  uint8_t *burnt = calloc(n, 1);     /* burnt at the start of this step   */
  uint8_t *is_new = calloc(n, 1);    /* ignited during this step          */
  int *life = calloc(n, sizeof(int)); /* active steps left (0: inactive)  */
  long *active = malloc(sizeof(long) * n);
  long *next = malloc(sizeof(long) * n);
  if (!burnt || !is_new || !life || !active || !next) {
    free(burnt); free(is_new); free(life); free(active); free(next);
    return -2;
  }
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};

  burnt[ign] = 1;
  life[ign] = burn_steps ? burn_steps[veg[ign]] : 1;
  active[0] = ign;
  long n_active = 1;
  uint32_t n_burnt = 1;
  uint32_t step = 0;
  uint64_t trials = 0;

  while (n_active > 0 && step < max_steps) {
    long n_next = 0;
    for (long i = 0; i < n_active; ++i) {
      long s = active[i];
      int sx = (int)(s % W), sy = (int)(s / W);
      uint32_t coins[2][4];
      int have_coins[2] = {0, 0};
      for (int d = 0; d < 8; ++d) {
        int tx = sx + DIR_DX[d], ty = sy + DIR_DY[d];
        if (!in_lattice(W, H, tx, ty)) continue;
        long t = (long)ty * W + tx;
        if (veg[t] == 0 || burnt[t]) continue;
        trials++;
        int g = d / 4;
        if (!have_coins[g]) {
          uint32_t ctr[4] = {sim_index, static_edges ? 0u : step,
                             (uint32_t)s, (uint32_t)g};
          oracle_philox4x32_10(ctr, key, coins[g]);
          have_coins[g] = 1;
        }
        uint32_t r = coins[g][d % 4];
        uint32_t thr = T[s * 8 + d];
        if (thr == 0xFFFFFFFFu || r < thr) {
          if (!is_new[t]) {
            is_new[t] = 1;
            next[n_next++] = t;
          }
        }
      }
    }
    n_burnt += (uint32_t)n_next;
    /* synchronous update: the new cells burn from the next step on, the
     * active ones lose one step of life */
    for (long i = 0; i < n_next; ++i) {
      long t = next[i];
      burnt[t] = 1;
      is_new[t] = 0;
      life[t] = burn_steps ? burn_steps[veg[t]] : 1;
    }
    for (long i = 0; i < n_active; ++i) {
      long s = active[i];
      life[s] -= 1;
      if (life[s] > 0) next[n_next++] = s;
    }
    long *tmp = active; active = next; next = tmp;
    n_active = n_next;
    step++;
  }

  if (map_bits) {
    for (long c = 0; c < n; ++c) {
      if (burnt[c]) {
        int x = (int)(c % W), y = (int)(c / W);
        map_bits[(long)y * stride + x / 32] |= 1u << (x % 32);
      }
    }
  }
  *out_burnt = n_burnt;
  *out_steps = step;
  *out_trials = trials;
  free(burnt); free(is_new); free(life); free(active); free(next);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* The per-target form of the propagation rule (Methods, propagation rules;
 * CUDA-implementation section): at each step every burnable cell that is
 * unburnt at the start of the step and has at least one burning neighbour
 * draws one uniform and ignites with probability 1 - prod_i (1 - p_i) over
 * its burning neighbours i. Each p_i is the quantised edge probability
 * T(i -> target) / 2^32 of the table, so the law of the final burn equals
 * the per-edge model's (independent coins, one per directed edge). The
 * product runs over the target's neighbours in direction order d = 0..7 in
 * binary64; a saturated edge (T = 0xFFFFFFFF) makes the probability 1; the
 * probability is quantised like an edge probability and compared with word 0
 * of Philox4x32-10(counter = (sim_index, step, target y*W + x, 2), key =
 * seed). A "trial" here is one such per-target draw. One-step burn.
 * Arguments and returns as oracle_simulate.                               */
int oracle_simulate_dense(int W, int H, const uint8_t *veg, const uint32_t *T,
                          int ign_x, int ign_y, uint32_t sim_index,
                          uint64_t seed, uint32_t max_steps,
                          uint32_t *map_bits, uint32_t *out_burnt,
                          uint32_t *out_steps, uint64_t *out_trials) {
  if (W <= 0 || H <= 0 || !in_lattice(W, H, ign_x, ign_y)) return -1;
  long n = (long)W * H;
  long stride = (W + 31) / 32;
  if (map_bits) memset(map_bits, 0, sizeof(uint32_t) * stride * H);
  *out_burnt = 0;
  *out_steps = 0;
  *out_trials = 0;
  long ign = (long)ign_y * W + ign_x;
  if (veg[ign] == 0) return 0;

  /* 0 unburnt, 1 burning (ignited at the previous step), 2 burnt out */
  uint8_t *state = calloc(n, 1);
  uint8_t *next = calloc(n, 1);
  if (!state || !next) { free(state); free(next); return -2; }
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  state[ign] = 1;
  uint32_t n_burnt = 1, step = 0;
  long n_burning = 1;
  uint64_t trials = 0;
  while (n_burning > 0 && step < max_steps) {
    n_burning = 0;
    for (int y = 0; y < H; ++y) {
      for (int x = 0; x < W; ++x) {
        long t = (long)y * W + x;
        if (state[t] != 0) { next[t] = 2; continue; }
        next[t] = 0;
        if (veg[t] == 0) continue;
        double q = 1.0;
        int any = 0, sure = 0;
        for (int d = 0; d < 8; ++d) {
          int sx = x + DIR_DX[d], sy = y + DIR_DY[d];
          if (!in_lattice(W, H, sx, sy)) continue;
          long s = (long)sy * W + sx;
          if (state[s] != 1) continue;
          any = 1;
          uint32_t thr = T[s * 8 + (d + 4) % 8]; /* edge s -> t */
          if (thr == 0xFFFFFFFFu) sure = 1;
          q = q * (1.0 - (double)thr * (1.0 / 4294967296.0));
        }
        if (!any) continue;
        trials++;
        uint32_t ctr[4] = {sim_index, step, (uint32_t)t, 2u}, out[4];
        oracle_philox4x32_10(ctr, key, out);
        uint32_t thr_t = sure ? 0xFFFFFFFFu : oracle_quantise_p(1.0 - q);
        if (thr_t == 0xFFFFFFFFu || out[0] < thr_t) {
          next[t] = 1;
          n_burning++;
        }
      }
    }
    n_burnt += (uint32_t)n_burning;
    uint8_t *tmp = state; state = next; next = tmp;
    step++;
  }
  if (map_bits)
    for (long c = 0; c < n; ++c)
      if (state[c]) {
        int x = (int)(c % W), y = (int)(c / W);
        map_bits[(long)y * stride + x / 32] |= 1u << (x % 32);
      }
  *out_burnt = n_burnt;
  *out_steps = step;
  *out_trials = trials;
  free(state); free(next);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Eq. 2 fitness: delta = (|A u A*| - |A n A*|) / |A|, A the reference map,
 * A* the simulated one, both packed as in oracle_simulate. Counts are taken
 * cell by cell; returns NaN when the reference is empty.                  */
double oracle_fitness(int W, int H, const uint32_t *sim_bits,
                      const uint32_t *ref_bits) {
  long stride = (W + 31) / 32;
  long n_union = 0, n_inter = 0, n_ref = 0;
  for (int y = 0; y < H; ++y) {
    for (int x = 0; x < W; ++x) {
      long w = (long)y * stride + x / 32;
      int a = (ref_bits[w] >> (x % 32)) & 1;
      int b = (sim_bits[w] >> (x % 32)) & 1;
      n_union += (a | b);
      n_inter += (a & b);
      n_ref += a;
    }
  }
  if (n_ref == 0) return NAN;
  return (double)(n_union - n_inter) / (double)n_ref;
}

/* ---------------------------------------------------------------------- */
/* Genetic-algorithm generation (Appendix B). The paper states the operators
 * (elitism, tournament of two, one-point crossover, per-gene mutation whose
 * probability decreases with the generation, a small random gene change)
 * but not their constants or random draws; the oracle fixes them:
 *   - fitness of individual i = mean over its R replicate deltas, summed in
 *     replicate order;
 *   - the `elite` best individuals (ordered by fitness, ties by index) are
 *     copied unchanged to slots 0..elite-1;
 *   - every other slot i holds the winner of a tournament between two
 *     individuals drawn with Philox counter (gen, i, 0, 0) under key
 *     ga_seed: a = (out0 * P) >> 32, b = (out1 * P) >> 32; lower fitness
 *     wins, a tie goes to the lower index;
 *   - slots elite+2k and elite+2k+1 are crossed at one point: counter
 *     (gen, k, 1, 0), cut c = 1 + ((out0 * (G-1)) >> 32), genes c..G-1
 *     swapped; an odd slot left over is not crossed;
 *   - each gene j of a non-elite slot i is mutated with counter
 *     (gen, i, 2, j): it mutates iff out0 * 2^-32 < pm0 * (1 - gen /
 *     generations), by delta = h[j] * (2 * out1 * 2^-32 - 1), and the result
 *     is clamped to [lo[j], hi[j]]. Each gene has its own box and width so
 *     that the 7-parameter search of Appendix B (beta[5] and the ignition
 *     x, y) keeps the coordinates on the lattice.
 * Only + - * / and comparisons are used, so any IEEE implementation gives
 * the same bits. pop is [P][G], fit is [P][R], new_pop is [P][G].         */

typedef struct {
  double fitness;
  int index;
} ranked_t;

static int rank_cmp(const void *a, const void *b) {
  const ranked_t *x = a, *y = b;
  if (x->fitness < y->fitness) return -1;
  if (x->fitness > y->fitness) return 1;
  return x->index - y->index;
}

int oracle_ga_step(const double *pop, const double *fit, int P, int G, int R,
                   int elite, double pm0, const double *h, const double *lo,
                   const double *hi,
                   uint32_t gen, uint32_t generations, uint64_t ga_seed,
                   double *new_pop, double *out_mean_fitness) {
  if (P <= 0 || G <= 1 || R <= 0 || elite < 0 || elite > P) return -1;
  const uint32_t key[2] = {(uint32_t)ga_seed, (uint32_t)(ga_seed >> 32)};
  double *mean = malloc(sizeof(double) * P);
  ranked_t *order = malloc(sizeof(ranked_t) * P);
  if (!mean || !order) { free(mean); free(order); return -2; }

  for (int i = 0; i < P; ++i) {
    double acc = 0.0;
    for (int r = 0; r < R; ++r) acc = acc + fit[(long)i * R + r];
    mean[i] = acc / (double)R;
    order[i].fitness = mean[i];
    order[i].index = i;
    if (out_mean_fitness) out_mean_fitness[i] = mean[i];
  }
  qsort(order, P, sizeof(ranked_t), rank_cmp);

  /* elitism */
  for (int e = 0; e < elite; ++e)
    memcpy(&new_pop[(long)e * G], &pop[(long)order[e].index * G],
           sizeof(double) * G);

  /* tournament selection of two */
  for (int i = elite; i < P; ++i) {
    uint32_t ctr[4] = {gen, (uint32_t)i, 0u, 0u}, out[4];
    oracle_philox4x32_10(ctr, key, out);
    int a = (int)(((uint64_t)out[0] * (uint64_t)P) >> 32);
    int b = (int)(((uint64_t)out[1] * (uint64_t)P) >> 32);
    int win;
    if (mean[a] < mean[b]) win = a;
    else if (mean[b] < mean[a]) win = b;
    else win = a < b ? a : b;
    memcpy(&new_pop[(long)i * G], &pop[(long)win * G], sizeof(double) * G);
  }

  /* one-point crossover of consecutive non-elite pairs */
  int n_pairs = (P - elite) / 2;
  for (int k = 0; k < n_pairs; ++k) {
    uint32_t ctr[4] = {gen, (uint32_t)k, 1u, 0u}, out[4];
    oracle_philox4x32_10(ctr, key, out);
    int cut = 1 + (int)(((uint64_t)out[0] * (uint64_t)(G - 1)) >> 32);
    double *u = &new_pop[(long)(elite + 2 * k) * G];
    double *v = &new_pop[(long)(elite + 2 * k + 1) * G];
    for (int j = cut; j < G; ++j) {
      double t = u[j]; u[j] = v[j]; v[j] = t;
    }
  }

  /* dynamic mutation */
  double pm = pm0 * (1.0 - (double)gen / (double)generations);
  for (int i = elite; i < P; ++i) {
    for (int j = 0; j < G; ++j) {
      uint32_t ctr[4] = {gen, (uint32_t)i, 2u, (uint32_t)j}, out[4];
      oracle_philox4x32_10(ctr, key, out);
      double u0 = (double)out[0] * (1.0 / 4294967296.0);
      if (u0 < pm) {
        double u1 = (double)out[1] * (1.0 / 4294967296.0);
        double g = new_pop[(long)i * G + j] + h[j] * (2.0 * u1 - 1.0);
        if (g < lo[j]) g = lo[j];
        if (g > hi[j]) g = hi[j];
        new_pop[(long)i * G + j] = g;
      }
    }
  }
  free(mean);
  free(order);
  return 0;
}
