/*
 * fire_nn.h -- C ABI of the learned surrogate of the fire simulator
 * (MI355X / gfx950), used to pre-screen genetic-algorithm offspring and
 * candidate ignition points before exact simulation.
 *
 * The surrogate is not part of the paper's method; the paper's fitting
 * (Methods, "Model fitting"; Appendix B) evaluates every candidate by
 * simulation. Here a network trained on simulator output predicts, for a
 * parameter vector beta[5] and an ignition cell (x, y) on one fixed
 * landscape, (a) t = log(1 + delta) with delta the Eq. 2 fitness against one
 * fixed reference map, and (b) a burn-probability map on a 128x128 grid.
 * Every candidate it keeps is re-scored by exact simulation (fire.h).
 *
 * Network (every matrix product and every decoder convolution takes bf16
 * operands -- activations, weights, back-propagated errors -- and
 * accumulates in fp32, on MFMA except for the gradients of the last
 * convolution, whose one output channel would fill one row of a 16-row
 * MFMA tile: those are summed on VALU over the input's grid, the error
 * first summed over the 2x2 blocks each tap reads; master weights and Adam
 * state fp32):
 *   input  x = (b0/30, ..., b4/30, 2x/W - 1, 2y/H - 1), zero-padded to 16
 *   h1 = relu(x  W1 + c1)    W1 16x256  (rows 7..15 unused, kept zero)
 *   h2 = relu(h1 W2 + c2)    W2 256x256
 *   h3 = relu(h2 W3 + c3)    W3 256x256
 *   t  = h3 Wf + cf          Wf 256x1
 *   d0 = relu(h3 Wd + cd)    Wd 256x2048, viewed as 8 channels x 16x16
 *   d1 = relu(U(d0) * K1)    3x3 conv, 8 -> 8, after 2x nearest upsampling (32x32)
 *   d2 = relu(U(d1) * K2)    8 -> 8 (64x64)
 *   z  = U(d2) * K3          8 -> 1 (128x128 logits); map = sigmoid(z)
 * Convolutions use zero padding and a per-output-channel bias; their
 * bias gradients are sums of the bf16 errors.
 * Loss per batch: mean((t - y_t)^2) + w_map * mean(BCE-with-logits(z, y_map)).
 *
 * Parameters are flattened (fp32) in this order: W1 [16][256], c1 [256],
 * W2 [256][256], c2, W3 [256][256], c3, Wf [256][1], cf [1],
 * Wd [256][2048], cd [2048], K1 [8][8][3][3], k1 [8], K2 [8][8][3][3],
 * k2 [8], K3 [1][8][3][3], k3 [1]; matrices row-major [in][out], conv
 * kernels [out][in][ky][kx].
 *
 * Conventions: device pointers unless stated; `stream` is a hipStream_t;
 * errors are returned, never thrown; a handle is not thread-safe.
 */
#ifndef FIRE_NN_H_
#define FIRE_NN_H_

#include <stdint.h>

#include "fire.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fire_nn fire_nn; /* opaque */

#define FIRE_NN_IN 7
#define FIRE_NN_MAP 128

typedef struct {
  int32_t max_batch;   /* largest batch any call will use (>= 1)           */
  int32_t lattice_w;   /* W, H of the landscape the ignition refers to      */
  int32_t lattice_h;
  float w_map;         /* weight of the map loss (0 disables the decoder's
                          loss; the decoder still runs in forward())       */
  float adam_b1, adam_b2, adam_eps;
} fire_nn_cfg;

/* Create a surrogate on `device` with parameters drawn from Philox under
 * `seed` (weights uniform in +-sqrt(6/(fan_in+fan_out)), biases 0). */
fire_status fire_nn_create(int device, const fire_nn_cfg *cfg, uint64_t seed,
                           fire_nn **out);
void fire_nn_destroy(fire_nn *nn);
const char *fire_nn_last_error(const fire_nn *nn);
/* Number of fp32 parameters (layout in the header comment). */
int64_t fire_nn_num_params(const fire_nn *nn);
/* Copy the fp32 master parameters out of / into the handle (device
 * pointers, num_params floats). Setting also refreshes the bf16 copies. */
fire_status fire_nn_get_params(fire_nn *nn, float *out, void *stream);
fire_status fire_nn_set_params(fire_nn *nn, const float *in, void *stream);

/* Forward pass for B <= max_batch candidates. x: [B][7] fp32 raw inputs
 * (beta[5], ignition x, y in cells); out_t: [B] fp32 predicted log(1+delta);
 * out_map: NULL (the decoder is then not run) or [B][128][128] fp32 burn
 * probabilities. */
fire_status fire_nn_forward(fire_nn *nn, const float *x, int32_t B,
                            float *out_t, float *out_map, void *stream);

/* Loss and gradients without updating: y_t [B] targets log(1+delta),
 * y_map NULL or [B][128][128] uint8 {0,1}; out_loss [2] fp32 (fitness
 * loss, map loss); out_grads NULL or [num_params] fp32, d(loss)/d(param). */
fire_status fire_nn_gradients(fire_nn *nn, const float *x, const float *y_t,
                              const uint8_t *y_map, int32_t B, float *out_loss,
                              float *out_grads, void *stream);

/* One Adam step (step >= 1, bias-corrected) on the batch. */
fire_status fire_nn_train_step(fire_nn *nn, const float *x, const float *y_t,
                               const uint8_t *y_map, int32_t B, float lr,
                               int32_t step, float *out_loss, void *stream);

/* Building block, exposed for tests: C = op(A) op(B) (+ bias[n]) (+ C if
 * accumulate), optionally ReLU, with A, B bf16 (uint16 storage) addressed
 * as A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn]; C fp32 [M][ldc];
 * Cb NULL or bf16 copy [M][ldc]. MFMA 32x32x16 bf16, fp32 accumulation. */
fire_status fire_gemm_bf16(int M, int N, int K, const uint16_t *A, int64_t sam,
                           int64_t sak, const uint16_t *Bm, int64_t sbk,
                           int64_t sbn, float *C, int64_t ldc, const float *bias,
                           int relu, int accumulate, uint16_t *Cb, void *stream);

/* Max-pool of packed burn maps (fire.h layout, W x H, map_words per map)
 * onto an out_w x out_h grid of uint8 {0,1}: cell (X, Y) is 1 iff any
 * burnt cell falls in [X*W/out_w, (X+1)*W/out_w) x [Y*H/out_h, ...). */
fire_status fire_pool_maps(const uint32_t *maps, int32_t n, int32_t W,
                           int32_t H, int64_t map_words, int32_t out_w,
                           int32_t out_h, uint8_t *out, void *stream);

/* Building block, exposed for tests: column sums out[n] = sum_m d[m*N + n]
 * of a row-major fp32 matrix d [M][N] (device pointers), the bias-gradient
 * reduction of the backward pass, in a fixed order: rows m = r, r + 16,
 * r + 32, ... are summed in order for each r = 0..15, and the sixteen
 * partial sums are then added pairwise, (p0 + p1), (p2 + p3), ..., then
 * those results pairwise in the same way down to one, so repeated calls
 * give identical bits. M >= 1, N >= 1. */
fire_status fire_colsum_f32(const float *d, int32_t M, int32_t N, float *out, void *stream);

/* Screening selection for oversampled GA offspring: out [k][G] receives
 * the first `keep` rows of cand unchanged (the elites), then the k - keep
 * rows of cand[keep..n) with the lowest score, in ascending score order
 * (ties by row index); out_idx [k] (NULL allowed) their row numbers.
 * cand [n][G] binary64, score [n] fp32 (non-finite scores rank last);
 * 1 <= k <= n <= 4096, 0 <= keep <= k. */
fire_status fire_nn_select(const double *cand, const float *score, int32_t n,
                           int32_t G, int32_t keep, int32_t k, double *out,
                           int32_t *out_idx, void *stream);

/* Training rows from simulator runs (device pointers). Row i of out_x
 * [n][7] fp32 is the network input of run i: parameter row i / reps of
 * params [*][5] binary64 (rounded to nearest fp32), then the ignition
 * (ign [n][2] fp32, or the constant pair ign_x, ign_y when ign is NULL);
 * out_y [n] fp32 receives log(1 + delta) of results[i].fitness (Eq. 2,
 * binary64 log1p rounded to fp32), the surrogate's fitness target;
 * out_fit [n] binary64 the fitness itself. Any output may be NULL (params
 * only when out_x is). n >= 0, reps >= 1. Stream-ordered. */
fire_status fire_nn_rows_from_results(const double *params, int32_t reps,
                                      const float *ign, float ign_x, float ign_y,
                                      const fire_result *results, int32_t n,
                                      float *out_x, float *out_y,
                                      double *out_fit, void *stream);

/* Row gather (device pointers): row k of dst [n][row_bytes] is row
 * rows[k] of src; used for shuffled minibatches of training rows, targets
 * and maps. row_bytes a positive multiple of 4; rows [n] int64 must index
 * rows of src (not checked on the device); dst must not overlap src.
 * n >= 0. Stream-ordered. */
fire_status fire_gather_rows(const void *src, int64_t row_bytes,
                             const int64_t *rows, int32_t n, void *dst,
                             void *stream);

/* Screening candidates from n_sets offspring sets drawn from one parent
 * population (sets [n_sets][P][5] binary64, e.g. n_sets calls of
 * fire_ga_step on copies of the population): cand receives all P rows of
 * set 0, then rows E..P-1 of sets 1..n_sets-1 (their rows 0..E-1 are the
 * same elites), P + (n_sets - 1)(P - E) rows of 5 values; x the matching
 * network inputs [rows][7] fp32 (parameters rounded to nearest, then the
 * constant ignition). n_sets >= 1, 0 <= E < P. Stream-ordered. */
fire_status fire_nn_candidates(const double *sets, int32_t n_sets, int32_t P,
                               int32_t E, float ign_x, float ign_y,
                               double *cand, float *x, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FIRE_NN_H_ */
