// Learned surrogate of the fire simulator (include/fire_nn.h): bf16 GEMMs on
// MFMA (v_mfma_f32_32x32x16_bf16, fp32 accumulation) for the MLP and the
// decoder's dense layer, fp32 upsample+3x3-convolution layers for the
// decoder, fused losses, Adam with fp32 master weights.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "fire_nn.h"

namespace firenn {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

// fp32 -> bf16 with round-to-nearest-even (inputs are finite)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

int blocks_for(int64_t n, int t = 256) {
  int64_t b = (n + t - 1) / t;
  if (b < 1) b = 1;
  if (b > 65535) b = 65535;
  return (int)b;
}

// ---------------------------------------------------------------------------
// GEMM: 64x64 output tile per workgroup of 4 waves, each wave one 32x32 MFMA
// tile; K staged through two LDS buffers 32 at a time (the next tile's
// global loads are in flight while the current one is multiplied). Both
// operands are stored in LDS as [row][k] (A rows are m, B rows are n), so
// that each lane's 8 consecutive k of a fragment are contiguous. A thread
// moves 8 bf16 of each operand per tile; how depends on the operand's
// strides (LoadMode).
constexpr int kTM = 64, kTN = 64, kTK = 32, kLdt = kTK + 8;

// kAlongK: k is contiguous (stride 1) and rows start on 16-byte boundaries:
//   one 16-byte load per thread, one 16-byte LDS store.
// kAlongRows: rows are contiguous and k-slices start on 16-byte boundaries:
//   one 16-byte load of 8 rows at one k, 8 two-byte LDS stores.
// kElementwise: any strides, 8 two-byte loads.
enum LoadMode { kElementwise = 0, kAlongK = 1, kAlongRows = 2 };

template <int MODE>
__device__ __forceinline__ void tile_load(const uint16_t *base, int64_t sr, int64_t sk, int row0,
                                          int rows, int k0, int kdim, int t, uint16_t v[8]) {
  if (MODE == kAlongK) {
    const int row = row0 + (t >> 2), k = k0 + (t & 3) * 8;
    if (row < rows && k + 8 <= kdim) {
      const uint4 q = *reinterpret_cast<const uint4 *>(base + (int64_t)row * sr + k);
      const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[2 * j] = (uint16_t)(w[j] & 0xFFFFu);
        v[2 * j + 1] = (uint16_t)(w[j] >> 16);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        v[i] = (row < rows && k + i < kdim) ? base[(int64_t)row * sr + k + i] : (uint16_t)0;
    }
  } else if (MODE == kAlongRows) {
    const int k = k0 + (t >> 3), row = row0 + (t & 7) * 8;
    if (k < kdim && row + 8 <= rows) {
      const uint4 q = *reinterpret_cast<const uint4 *>(base + (int64_t)k * sk + row);
      const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[2 * j] = (uint16_t)(w[j] & 0xFFFFu);
        v[2 * j + 1] = (uint16_t)(w[j] >> 16);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        v[i] = (k < kdim && row + i < rows) ? base[(int64_t)k * sk + row + i] : (uint16_t)0;
    }
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = t + 256 * i;
      const int row = row0 + (e >> 5), k = k0 + (e & 31);
      v[i] = (row < rows && k < kdim) ? base[(int64_t)row * sr + (int64_t)k * sk] : (uint16_t)0;
    }
  }
}

template <int MODE>
__device__ __forceinline__ void tile_store(uint16_t *S, int t, const uint16_t v[8]) {
  if (MODE == kAlongK) {
    uint4 q;
    q.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
    q.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
    q.z = (uint32_t)v[4] | ((uint32_t)v[5] << 16);
    q.w = (uint32_t)v[6] | ((uint32_t)v[7] << 16);
    *reinterpret_cast<uint4 *>(&S[(t >> 2) * kLdt + (t & 3) * 8]) = q;
  } else if (MODE == kAlongRows) {
    const int kk = t >> 3, r = (t & 7) * 8;
#pragma unroll
    for (int i = 0; i < 8; ++i) S[(r + i) * kLdt + kk] = v[i];
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = t + 256 * i;
      S[(e >> 5) * kLdt + (e & 31)] = v[i];
    }
  }
}

template <int AM, int BM>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, const uint16_t *A,
                                                   int64_t sam, int64_t sak, const uint16_t *B,
                                                   int64_t sbk, int64_t sbn, float *C,
                                                   int64_t ldc, const float *bias, int relu,
                                                   int accumulate, uint16_t *Cb) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][kTM * kLdt];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][kTN * kLdt];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  f32x16_t acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  uint16_t va[8], vb[8];
  tile_load<AM>(A, sam, sak, m0, M, 0, K, tid, va);
  tile_load<BM>(B, sbn, sbk, n0, N, 0, K, tid, vb);
  tile_store<AM>(As[0], tid, va);
  tile_store<BM>(Bs[0], tid, vb);
  __syncthreads();
  const int half = lane >> 5, r = lane & 31;
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += kTK) {
    const bool more = k0 + kTK < K;
    if (more) {
      tile_load<AM>(A, sam, sak, m0, M, k0 + kTK, K, tid, va);
      tile_load<BM>(B, sbn, sbk, n0, N, k0 + kTK, K, tid, vb);
    }
#pragma unroll
    for (int kk = 0; kk < kTK; kk += 16) {
      const bf16x8_t a =
          *reinterpret_cast<const bf16x8_t *>(&As[buf][(wr + r) * kLdt + kk + half * 8]);
      const bf16x8_t b =
          *reinterpret_cast<const bf16x8_t *>(&Bs[buf][(wc + r) * kLdt + kk + half * 8]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    if (more) {
      // the other buffer was last read before the previous barrier
      tile_store<AM>(As[buf ^ 1], tid, va);
      tile_store<BM>(Bs[buf ^ 1], tid, vb);
    }
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = wr + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int j = wc + (lane & 31);
    const int m = m0 + i, n = n0 + j;
    if (m < M && n < N) {
      float val = acc[v];
      if (bias) val += bias[n];
      if (accumulate) val += C[(int64_t)m * ldc + n];
      if (relu) val = fmaxf(val, 0.0f);
      C[(int64_t)m * ldc + n] = val;
      if (Cb) Cb[(int64_t)m * ldc + n] = f2bf(val);
    }
  }
}

// how an operand of `rows` x `kdim` with strides (sr, sk) is loaded
int load_mode(const uint16_t *p, int64_t sr, int64_t sk) {
  if ((reinterpret_cast<uintptr_t>(p) & 15u) != 0) return kElementwise;
  if (sk == 1 && sr % 8 == 0) return kAlongK;
  if (sr == 1 && sk % 8 == 0) return kAlongRows;
  return kElementwise;
}

template <int AM>
hipError_t gemm_b(int bm, dim3 grid, hipStream_t s, int M, int N, int K, const uint16_t *A,
                  int64_t sam, int64_t sak, const uint16_t *B, int64_t sbk, int64_t sbn, float *C,
                  int64_t ldc, const float *bias, int relu, int accumulate, uint16_t *Cb) {
  if (bm == kAlongK)
    hipLaunchKernelGGL((gemm_kernel<AM, kAlongK>), grid, dim3(256), 0, s, M, N, K, A, sam, sak,
                       B, sbk, sbn, C, ldc, bias, relu, accumulate, Cb);
  else if (bm == kAlongRows)
    hipLaunchKernelGGL((gemm_kernel<AM, kAlongRows>), grid, dim3(256), 0, s, M, N, K, A, sam,
                       sak, B, sbk, sbn, C, ldc, bias, relu, accumulate, Cb);
  else
    hipLaunchKernelGGL((gemm_kernel<AM, kElementwise>), grid, dim3(256), 0, s, M, N, K, A, sam,
                       sak, B, sbk, sbn, C, ldc, bias, relu, accumulate, Cb);
  return hipGetLastError();
}

hipError_t gemm(int M, int N, int K, const uint16_t *A, int64_t sam, int64_t sak,
                const uint16_t *B, int64_t sbk, int64_t sbn, float *C, int64_t ldc,
                const float *bias, int relu, int accumulate, uint16_t *Cb, hipStream_t s) {
  dim3 grid((N + kTN - 1) / kTN, (M + kTM - 1) / kTM);
  const int am = load_mode(A, sam, sak), bm = load_mode(B, sbn, sbk);
  if (am == kAlongK)
    return gemm_b<kAlongK>(bm, grid, s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, relu,
                           accumulate, Cb);
  if (am == kAlongRows)
    return gemm_b<kAlongRows>(bm, grid, s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, relu,
                              accumulate, Cb);
  return gemm_b<kElementwise>(bm, grid, s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, relu,
                              accumulate, Cb);
}

// ---------------------------------------------------------------------------
// Elementwise and reduction kernels

__global__ void to_bf16_kernel(const float *x, uint16_t *y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = f2bf(x[i]);
}

// raw [B][7] -> bf16 [B][16]: beta/30, ignition scaled to [-1, 1], zero pad
__global__ void prep_input_kernel(const float *x, int B, float inv_w, float inv_h, uint16_t *xb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * 16) return;
  const int b = i >> 4, k = i & 15;
  float v = 0.0f;
  if (k < 5) v = x[b * 7 + k] * (1.0f / 30.0f);
  else if (k == 5) v = 2.0f * x[b * 7 + 5] * inv_w - 1.0f;
  else if (k == 6) v = 2.0f * x[b * 7 + 6] * inv_h - 1.0f;
  xb[i] = f2bf(v);
}

// g <- g * (h > 0) (ReLU backward, in place) and its bf16 copy
__global__ void relu_bwd_kernel(float *g, const float *h, uint16_t *gb, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float v = h[i] > 0.0f ? g[i] : 0.0f;
    g[i] = v;
    gb[i] = f2bf(v);
  }
}

// column sums of d [M][N] (bias gradients) in a fixed order: a workgroup of
// 256 threads takes 16 columns; row group r (0..15) sums rows r, r+16, ...
// in order, then the 16 partial sums are added pairwise:
// p0+p1, p2+p3, ..., then those pairwise, down to one
constexpr int kColsumCols = 16, kColsumGroups = 16;
__global__ __launch_bounds__(256) void colsum_kernel(const float *d, int M, int N, float *out) {
  __shared__ float part[kColsumGroups][kColsumCols];
  const int c = threadIdx.x % kColsumCols, rg = threadIdx.x / kColsumCols;
  const int n = blockIdx.x * kColsumCols + c;
  float s = 0.0f;
  if (n < N)
    for (int m = rg; m < M; m += kColsumGroups) s += d[(int64_t)m * N + n];
  part[rg][c] = s;
  __syncthreads();
  if (rg == 0 && n < N) {
    float p[kColsumGroups];
#pragma unroll
    for (int i = 0; i < kColsumGroups; ++i) p[i] = part[i][c];
#pragma unroll
    for (int w = kColsumGroups; w > 1; w >>= 1)
#pragma unroll
      for (int i = 0; i < w / 2; ++i) p[i] = p[2 * i] + p[2 * i + 1];
    out[n] = p[0];
  }
}

int colsum_blocks(int N) { return (N + kColsumCols - 1) / kColsumCols; }

__device__ float block_reduce(float v, float *red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  const float r = red[0];
  __syncthreads();
  return r;
}

// fitness head: loss = mean((t - y)^2), dt = 2 (t - y) / B
__global__ __launch_bounds__(256) void loss_fit_kernel(const float *t, const float *y, int B,
                                                       float *dt, uint16_t *dtb, float *loss) {
  __shared__ float red[256];
  float acc = 0.0f;
  for (int b = threadIdx.x; b < B; b += 256) {
    const float e = t[b] - y[b];
    acc += e * e;
    const float g = 2.0f * e / (float)B;
    dt[b] = g;
    dtb[b] = f2bf(g);
  }
  const float s = block_reduce(acc, red);
  if (threadIdx.x == 0) loss[0] = s / (float)B;
}

// map head: BCE with logits, dz = w (sigmoid(z) - y) / (B P); per-block
// partial losses reduced afterwards in fixed order
__global__ __launch_bounds__(256) void loss_map_kernel(const float *z, const uint8_t *y,
                                                       int64_t n, float w, float *dz,
                                                       float *partial) {
  __shared__ float red[256];
  float acc = 0.0f;
  const float inv_n = 1.0f / (float)n;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float zi = z[i], yi = y[i] ? 1.0f : 0.0f;
    acc += fmaxf(zi, 0.0f) - zi * yi + log1pf(expf(-fabsf(zi)));
    const float sg = 1.0f / (1.0f + expf(-zi));
    dz[i] = w * (sg - yi) * inv_n;
  }
  const float s = block_reduce(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const float *p, int n, float scale,
                                                           float *out) {
  __shared__ float red[256];
  float acc = 0.0f;
  for (int i = threadIdx.x; i < n; i += 256) acc += p[i];
  const float s = block_reduce(acc, red);
  if (threadIdx.x == 0) out[0] = s * scale;
}

__global__ void sigmoid_kernel(const float *z, float *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 1.0f / (1.0f + expf(-z[i]));
}

// ---------------------------------------------------------------------------
// Decoder convolutions on MFMA (v_mfma_f32_16x16x32_bf16: A 16x32 with lane
// l holding row l%16 and k 8*(l/16)..+8; B 32x16 with lane l holding column
// l%16 and the same k; D 16x16 with lane l holding column l%16 and rows
// 4*(l/16)..+4). A layer is out = conv3x3(up2(in)) with zero padding, in
// [Ci=8][S][S] and out [Co][2S][2S]; the products take bf16 operands
// (activations, kernels, back-propagated errors) and accumulate in fp32.
// One workgroup of 4 waves per sample stages that sample's planes in LDS.
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;
typedef uint16_t u16x8_t __attribute__((ext_vector_type(8)));
constexpr int kConvCi = 8, kConvTaps = 9, kConvK = kConvCi * kConvTaps;  // 72
constexpr int kWgradCols = 80;  // 72 kernel taps, the bias column, padding
constexpr int kWgradRows = 16;  // output channels, padded
constexpr int kWgradParts = 2048;

__device__ __forceinline__ bf16x8_t as_bf16x8(u16x8_t v) { return __builtin_bit_cast(bf16x8_t, v); }

// Stage n bf16 values (n a multiple of 8, 16-byte aligned) into LDS.
__device__ __forceinline__ void stage_bf16(uint16_t *dst, const uint16_t *src, int n) {
  for (int i = threadIdx.x; i < n / 8; i += blockDim.x)
    reinterpret_cast<uint4 *>(dst)[i] = reinterpret_cast<const uint4 *>(src)[i];
}

// Forward (UP) or data gradient (!UP) of one layer, 16-pixel tiles of the
// 2S x 2S grid:
//   UP:  out[co][y][x] = bias[co] + sum_k A[p][k] B[k][co],
//        A[p][k] = in[ci][(y+dy-1)/2][(x+dx-1)/2], B[k][co] = K[co][ci][dy][dx];
//        written fp32 (and bf16) after an optional ReLU;
//  !UP:  dU[ci][u][v] = sum_k A[p][k] B[k][ci],
//        A[p][k] = g[co][u-dy+1][v-dx+1], B[k][ci] = K[co][ci][dy][dx];
//        the 2x2 blocks of dU are summed into din[ci][u/2][v/2], which is
//        zeroed where act <= 0.
// src: UP the layer input [8][S][S], !UP the error g [8][2S][2S] (bf16;
// the one-channel data gradient of the last layer runs in
// upconv_grads_co1_kernel). The 8 source planes are staged
// channel-interleaved, [row][col][channel], and k = tap * 8 + channel: a
// lane's 8 k-values of a step are the 8 channels of one source cell, one
// 16-byte LDS read.
template <bool UP>
__global__ __launch_bounds__(256) void upconv_mfma_kernel(const uint16_t *src, const uint16_t *Kb,
                                                          const float *bias, int S, int Co,
                                                          int relu, const float *act, float *out,
                                                          uint16_t *out_b) {
  extern __shared__ __attribute__((aligned(16))) uint16_t plane[];
  const int b = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int O = 2 * S;
  const int srcR = UP ? S : O;
  const uint16_t *sp = src + (int64_t)b * kConvCi * srcR * srcR;
  {
    const int n = srcR * srcR;
    for (int i = threadIdx.x; i < kConvCi * n; i += blockDim.x)
      plane[(i % n) * kConvCi + i / n] = sp[i];
  }
  const int col = lane & 15, kq = lane >> 4;
  const int ncols = UP ? Co : kConvCi;  // columns of the result
  const int nk = kConvTaps * kConvCi;
  const int steps = (nk + 31) / 32;
  // B fragments of the (up to) three k-steps
  bf16x8_t bw[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    u16x8_t v;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = 32 * s + 8 * kq + i;
      const int t = k / kConvCi, c = k % kConvCi;
      // UP: column col is co, k runs over (tap, ci). !UP: column col is ci,
      // k runs over (tap, co)
      const bool ok = k < nk && col < ncols;
      const int widx = UP ? (col * kConvCi + c) * kConvTaps + t : (c * kConvCi + col) * kConvTaps + t;
      v[i] = ok ? Kb[widx] : (uint16_t)0;
    }
    bw[s] = as_bf16x8(v);
  }
  const float bcol = (UP && col < ncols && bias) ? bias[col] : 0.0f;
  __syncthreads();
  // tile: 16 consecutive columns x0.. of one row; for !UP a wave takes the
  // two rows of a 2x2 block together
  const int per_row = O / 16;
  const int rows_per_item = UP ? 1 : 2;
  const int items = (O / rows_per_item) * per_row;
  const int sgn = UP ? 1 : -1;
  for (int it = wave; it < items; it += 4) {
    const int y0 = (it / per_row) * rows_per_item, x0 = (it % per_row) * 16;
    const int x = x0 + (lane & 15);
    f32x4_t acc[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) acc[r] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (r >= rows_per_item) break;
      const int y = y0 + r;
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        if (s >= steps) break;
        u16x8_t a;
        // tap 4 s + kq, the 8 channels of one source cell
        const int t = 4 * s + kq;
        const int yy = y + sgn * (t / 3 - 1), xx = x + sgn * (t % 3 - 1);
        const bool in = t < kConvTaps && (unsigned)yy < (unsigned)O && (unsigned)xx < (unsigned)O;
        const int sy = UP ? (yy >> 1) : yy, sx = UP ? (xx >> 1) : xx;
        if (in) {
          a = *reinterpret_cast<const u16x8_t *>(&plane[(sy * srcR + sx) * kConvCi]);
        } else {
#pragma unroll
          for (int i = 0; i < 8; ++i) a[i] = 0;
        }
        acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a), bw[s], acc[r], 0, 0, 0);
      }
    }
    if (col >= ncols) continue;
    if (UP) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float val = acc[0][v] + bcol;
        if (relu) val = fmaxf(val, 0.0f);
        const int64_t o = (((int64_t)b * Co + col) * O + y0) * O + x0 + 4 * kq + v;
        out[o] = val;
        if (out_b) out_b[o] = f2bf(val);
      }
    } else {
      // lane holds dU[col][y0 + r][x0 + 4kq + v]: pairs of columns in the
      // lane, the two rows in acc[0] and acc[1]
      const int sy = y0 >> 1;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float sum = (acc[0][2 * h] + acc[0][2 * h + 1]) + (acc[1][2 * h] + acc[1][2 * h + 1]);
        const int sx = (x0 >> 1) + 2 * kq + h;
        const int64_t o = (((int64_t)b * kConvCi + col) * S + sy) * S + sx;
        const float val = act[o] > 0.0f ? sum : 0.0f;
        out[o] = val;
        if (out_b) out_b[o] = f2bf(val);
      }
    }
  }
}

// Kernel and bias gradients of one layer: for every sample handled by this
// workgroup (b = blockIdx.x, + gridDim.x, ...) the contraction over its
// (2S)^2 pixels, 32 per MFMA step:
//   P[co][k] += sum_p A[co][p] B[p][k],  A[co][p] = g[co][p] (bf16 error),
//   B[p][k] = in[ci][(y+dy-1)/2][(x+dx-1)/2] for k = ci*9 + dy*3 + dx < 72,
//   1 for k = 72 (the bias gradient), 0 beyond;
// the four waves' sums are added in wave order and the workgroup writes its
// partial [16][80] to part; wgrad_finish_kernel adds the partials.
__global__ __launch_bounds__(256) void upconv_wgrad_mfma_kernel(const uint16_t *g_b,
                                                                const uint16_t *in_b, int B, int S,
                                                                int Co, float *part) {
  extern __shared__ __attribute__((aligned(16))) uint16_t lds16[];
  __shared__ float red[4][kWgradRows * kWgradCols];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int O = 2 * S;
  uint16_t *gpl = lds16;                        // [Co][O][O]
  uint16_t *ipl = lds16 + (Co * O * O + 7) / 8 * 8;  // [8][S][S]
  const int row = lane & 15, kq = lane >> 4;
  // each lane's B column per n-tile: k = 16 n + row
  int bc[5], bdy[5], bdx[5];
#pragma unroll
  for (int n = 0; n < 5; ++n) {
    const int k = 16 * n + row;
    bc[n] = k < kConvK ? k / kConvTaps : (k == kConvK ? -2 : -1);
    bdy[n] = (k % kConvTaps) / 3;
    bdx[n] = (k % kConvTaps) % 3;
  }
  f32x4_t acc[5];
#pragma unroll
  for (int n = 0; n < 5; ++n) acc[n] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
  const int chunks = O * O / 32;
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    __syncthreads();
    stage_bf16(gpl, g_b + (int64_t)b * Co * O * O, Co * O * O);
    stage_bf16(ipl, in_b + (int64_t)b * kConvCi * S * S, kConvCi * S * S);
    __syncthreads();
    for (int ch = wave; ch < chunks; ch += 4) {
      const int p0 = ch * 32 + 8 * kq;  // this lane's 8 pixels (one row)
      const int y = p0 / O, x0 = p0 % O;
      u16x8_t a;
      if (row < Co) {
        a = *reinterpret_cast<const u16x8_t *>(&gpl[(row * O + y) * O + x0]);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = 0;
      }
      const bf16x8_t av = as_bf16x8(a);
#pragma unroll
      for (int n = 0; n < 5; ++n) {
        u16x8_t bv;
        const int c = bc[n];
        const int yy = y + bdy[n] - 1;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int xx = x0 + i + bdx[n] - 1;
          uint16_t v = 0;
          if (c >= 0) {
            if ((unsigned)yy < (unsigned)O && (unsigned)xx < (unsigned)O)
              v = ipl[(c * S + (yy >> 1)) * S + (xx >> 1)];
          } else if (c == -2) {
            v = 0x3F80u;  // 1.0
          }
          bv[i] = v;
        }
        acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, as_bf16x8(bv), acc[n], 0, 0, 0);
      }
    }
  }
  // D layout: lane holds column (16 n + row) and rows (co) 4 kq + v
#pragma unroll
  for (int n = 0; n < 5; ++n)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave][(4 * kq + v) * kWgradCols + 16 * n + row] = acc[n][v];
  __syncthreads();
  for (int i = threadIdx.x; i < kWgradRows * kWgradCols; i += blockDim.x)
    part[(int64_t)blockIdx.x * kWgradRows * kWgradCols + i] =
        ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
}

__device__ __forceinline__ float bf16_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Kernel, bias and data gradients of a layer with one output channel (the
// last decoder layer), on the input's own grid. With nearest 2x upsampling,
// tap (dy, dx) of output pixel (y, x) reads input cell
// ((y + dy - 1) >> 1, (x + dx - 1) >> 1), so
//   dK[c][dy][dx] = sum over input cells (Y, X) of in[c][Y][X] times the
//                   sum of g over output rows {2Y+1-dy, 2Y+2-dy} and
//                   columns {2X+1-dx, 2X+2-dx} (pixels outside the output
//                   contribute nothing),
// a quarter of the multiply-adds of the per-pixel form and no im2col; the
// bias gradient is the sum of g over the 2x2 blocks {2Y, 2Y+1} x
// {2X, 2X+1}. With one output channel an MFMA tile would use one of its 16
// rows, so this runs on VALU. Thread item: one sample's input cells
// (Y, 2j) and (Y, 2j + 1); their error windows, rows 2Y-1 .. 2Y+2 and
// columns 4j-1 .. 4j+4, are three 8-byte loads per row, their inputs one
// 4-byte load per channel. Items are spread over the grid; each thread
// keeps 73 sums, reduced over the wave (a fixed shuffle tree) and then over
// the four waves in order, so the result does not depend on timing.
// Partials [gridDim.x][16][80] (row 0) as the MFMA form. S even, S <= 64.
// The same box sums also give the layer's data gradient: the
// error of input cell (Y, X), summed over its 2x2 upsampling block, is
// sum over taps of K[c][dy][dx] times box (dy, dx); it is zeroed where the
// layer input's activation act <= 0 and written to din (fp32) and din_b
// (bf16), as the MFMA data-gradient kernel writes it.
__global__ __launch_bounds__(256) void upconv_grads_co1_kernel(const uint16_t *g_b,
                                                               const uint16_t *in_b, int B, int S,
                                                               float *part, const uint16_t *Kb,
                                                               const float *act, float *din,
                                                               uint16_t *din_b) {
  __shared__ float red[4][kConvK + 1];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int O = 2 * S, half = S / 2;
  float acc[kConvK + 1];
#pragma unroll
  for (int k = 0; k <= kConvK; ++k) acc[k] = 0.0f;
  float kw[kConvK];
#pragma unroll
  for (int k = 0; k < kConvK; ++k) kw[k] = bf16_f32(Kb[k]);
  const int64_t items = (int64_t)B * S * half;
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + t; it < items;
       it += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(it / (S * half)), pr = (int)(it % (S * half));
    const int Y = pr / half, j = pr % half;
    const uint16_t *gp = g_b + (int64_t)b * O * O;
    // w[i][m]: error at row 2Y - 1 + i, column 4j - 1 + m (0 outside)
    float w[4][6];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int y = 2 * Y - 1 + i;
      uint2 q0 = make_uint2(0u, 0u), q1 = make_uint2(0u, 0u), q2 = make_uint2(0u, 0u);
      if ((unsigned)y < (unsigned)O) {
        const uint2 *row = reinterpret_cast<const uint2 *>(gp + (int64_t)y * O);
        if (j > 0) q0 = row[j - 1];
        q1 = row[j];
        if (j + 1 < half) q2 = row[j + 1];
      }
      w[i][0] = __uint_as_float(q0.y & 0xFFFF0000u);
      w[i][1] = __uint_as_float(q1.x << 16);
      w[i][2] = __uint_as_float(q1.x & 0xFFFF0000u);
      w[i][3] = __uint_as_float(q1.y << 16);
      w[i][4] = __uint_as_float(q1.y & 0xFFFF0000u);
      w[i][5] = __uint_as_float(q2.x << 16);
    }
    float v0[kConvCi], v1[kConvCi];
#pragma unroll
    for (int c = 0; c < kConvCi; ++c) {
      const uint32_t pv =
          *reinterpret_cast<const uint32_t *>(in_b + ((int64_t)(b * kConvCi + c) * S + Y) * S + 2 * j);
      v0[c] = __uint_as_float(pv << 16);
      v1[c] = __uint_as_float(pv & 0xFFFF0000u);
    }
    float dsum[2][kConvCi];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      // cell (Y, 2j + h): window columns 2h .. 2h + 3 of w
      float cp[4][3];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) cp[i][dx] = w[i][2 * h + 2 - dx] + w[i][2 * h + 3 - dx];
      float box[kConvTaps];
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) box[3 * dy + dx] = cp[2 - dy][dx] + cp[3 - dy][dx];
#pragma unroll
      for (int c = 0; c < kConvCi; ++c) {
        const float v = h ? v1[c] : v0[c];
        float d = 0.0f;
#pragma unroll
        for (int tap = 0; tap < kConvTaps; ++tap) {
          acc[c * kConvTaps + tap] = fmaf(box[tap], v, acc[c * kConvTaps + tap]);
          d = fmaf(kw[c * kConvTaps + tap], box[tap], d);
        }
        dsum[h][c] = d;
      }
      acc[kConvK] += (w[1][2 * h + 1] + w[1][2 * h + 2]) + (w[2][2 * h + 1] + w[2][2 * h + 2]);
    }
#pragma unroll
    for (int c = 0; c < kConvCi; ++c) {
      const int64_t o = ((int64_t)(b * kConvCi + c) * S + Y) * S + 2 * j;
      const float2 a = *reinterpret_cast<const float2 *>(act + o);
      const float r0 = a.x > 0.0f ? dsum[0][c] : 0.0f, r1 = a.y > 0.0f ? dsum[1][c] : 0.0f;
      *reinterpret_cast<float2 *>(din + o) = make_float2(r0, r1);
      *reinterpret_cast<uint32_t *>(din_b + o) = (uint32_t)f2bf(r0) | ((uint32_t)f2bf(r1) << 16);
    }
  }
#pragma unroll
  for (int k = 0; k <= kConvK; ++k) {
    float v = acc[k];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off);
    acc[k] = v;
  }
  if (lane == 0)
#pragma unroll
    for (int k = 0; k <= kConvK; ++k) red[wave][k] = acc[k];
  __syncthreads();
  float *out = part + (int64_t)blockIdx.x * kWgradRows * kWgradCols;
  for (int i = t; i < kWgradRows * kWgradCols; i += blockDim.x) {
    const int r = i / kWgradCols, k = i % kWgradCols;
    out[i] = (r == 0 && k <= kConvK) ? ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k] : 0.0f;
  }
}

// dK[co][ci][dy][dx] and dkb[co] from the partials of `parts` workgroups:
// one workgroup per output; thread t adds partials t, t + 256, ... in
// order, then a pairwise tree over the 256 threads.
__global__ __launch_bounds__(256) void wgrad_finish_kernel(const float *part, int parts, int Co,
                                                           float *dK, float *dkb) {
  __shared__ float red[256];
  const int o = blockIdx.x;  // co * 73 + k
  const int co = o / (kConvK + 1), k = o % (kConvK + 1);
  float s = 0.0f;
  for (int p = threadIdx.x; p < parts; p += 256)
    s += part[(int64_t)p * kWgradRows * kWgradCols + co * kWgradCols + k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (k < kConvK) dK[co * kConvK + k] = red[0];
    else dkb[co] = red[0];
  }
}

// ---------------------------------------------------------------------------
// Adam (bias-corrected), fp32 master weights; wb receives the bf16 copy of
// the updated weights the matrix products read
__global__ void adam_kernel(float *w, uint16_t *wb, float *m, float *v, const float *g, int64_t n,
                            float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
  }
}

// Philox4x32-10 word 0 as the uniform source of the initial weights
__device__ uint32_t philox_word0(uint32_t c0, uint32_t c1, uint32_t k0, uint32_t k1) {
  uint32_t c2 = 0, c3 = 0;
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p2 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p2 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p2;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c0;
}

__global__ void init_uniform_kernel(float *w, int64_t n, float limit, uint32_t tensor,
                                    uint32_t k0, uint32_t k1, int rows_used, int cols) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t u = philox_word0((uint32_t)i, tensor, k0, k1);
    const float v = (2.0f * ((float)(u >> 8) * (1.0f / 16777216.0f)) - 1.0f) * limit;
    w[i] = (rows_used > 0 && (int)(i / cols) >= rows_used) ? 0.0f : v;
  }
}

__global__ void fill_f32_kernel(float *p, float v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// maps: packed burn maps -> coarse uint8 occupancy grid
__global__ void pool_maps_kernel(const uint32_t *maps, int n, int W, int H, int64_t map_words,
                                 int ow, int oh, uint8_t *out) {
  const int64_t total = (int64_t)n * ow * oh;
  const int stride = (W + 31) / 32;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int X = (int)(i % ow), Y = (int)((i / ow) % oh), k = (int)(i / ((int64_t)ow * oh));
    const int x0 = (int)((int64_t)X * W / ow), x1 = (int)((int64_t)(X + 1) * W / ow);
    const int y0 = (int)((int64_t)Y * H / oh), y1 = (int)((int64_t)(Y + 1) * H / oh);
    const uint32_t *m = maps + (int64_t)k * map_words;
    uint8_t any = 0;
    for (int y = y0; y < y1 && !any; ++y)
      for (int x = x0; x < x1; ++x)
        if ((m[(int64_t)y * stride + (x >> 5)] >> (x & 31)) & 1u) { any = 1; break; }
    out[i] = any;
  }
}

// rank of each non-elite candidate by (score, index); one workgroup
__global__ __launch_bounds__(1024) void select_kernel(const double *cand, const float *score,
                                                      int n, int G, int keep, int k, double *out,
                                                      int32_t *out_idx) {
  // the scores are staged in LDS (n <= 4096): every thread reads all of
  // them, the same one at a time (a broadcast)
  __shared__ float sc[4096];
  for (int i = threadIdx.x; i < n; i += 1024) sc[i] = score[i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 1024) {
    int slot;
    if (i < keep) {
      slot = i;
    } else {
      const float si = sc[i];
      const bool fi = isfinite(si);
      int rank = 0;
      for (int j = keep; j < n; ++j) {
        const float sj = sc[j];
        const bool fj = isfinite(sj);
        const bool before = (fj && !fi) || (fj == fi && ((fi && sj < si) || ((!fi || sj == si) && j < i)));
        rank += before ? 1 : 0;
      }
      slot = keep + rank;
    }
    if (slot < k) {
      for (int c = 0; c < G; ++c) out[(int64_t)slot * G + c] = cand[(int64_t)i * G + c];
      if (out_idx) out_idx[slot] = i;
    }
  }
}

// ---------------------------------------------------------------------------
// Training rows from simulation results: row i takes parameter row
// i / reps (binary64 -> fp32, round to nearest), the ignition (a row of
// `ign` or the constant pair) and the target log(1 + delta) of result i's
// Eq. 2 fitness (binary64 log1p, then rounded to fp32); delta itself is
// copied to out_fit. Any output may be NULL.
__global__ void rows_from_results_kernel(const double *params, int reps, const float *ign,
                                         float ign_x, float ign_y, const fire_result *res, int n,
                                         float *out_x, float *out_y, double *out_fit) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double delta = res[i].fitness;
    if (out_fit) out_fit[i] = delta;
    if (out_y) out_y[i] = (float)log1p(delta);
    if (out_x) {
      const double *b = params + 5 * (int64_t)(i / reps);
      float *x = out_x + 7 * (int64_t)i;
      for (int k = 0; k < 5; ++k) x[k] = (float)b[k];
      x[5] = ign ? ign[2 * (int64_t)i] : ign_x;
      x[6] = ign ? ign[2 * (int64_t)i + 1] : ign_y;
    }
  }
}

// dst row k = src row rows[k]; rows of `words` 32-bit words, copied with
// 16-byte moves when `vec` (rows and both bases 16-byte aligned).
__global__ void gather_rows_kernel(const uint32_t *src, int64_t words, const int64_t *rows, int n,
                                   uint32_t *dst, int vec) {
  const int64_t per = vec ? words / 4 : words;
  const int64_t total = (int64_t)n * per;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = t / per, w = t % per;
    const int64_t r = rows[k];
    if (vec) {
      reinterpret_cast<uint4 *>(dst + k * words)[w] =
          reinterpret_cast<const uint4 *>(src + r * words)[w];
    } else {
      dst[k * words + w] = src[r * words + w];
    }
  }
}

// Screening candidates from `n_sets` offspring sets [n_sets][P][5]: all of
// set 0, then rows E..P-1 of every later set (its first E rows are the
// elites again); binary64 rows to cand, fp32 network inputs (parameters,
// then the constant ignition) to x.
__global__ void candidates_kernel(const double *sets, int n_sets, int P, int E, float ign_x,
                                  float ign_y, double *cand, float *x) {
  const int n = P + (n_sets - 1) * (P - E);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int src = i;
    if (i >= P) {
      const int o = 1 + (i - P) / (P - E), j = E + (i - P) % (P - E);
      src = o * P + j;
    }
    for (int k = 0; k < 5; ++k) {
      const double v = sets[5 * (int64_t)src + k];
      cand[5 * (int64_t)i + k] = v;
      x[7 * (int64_t)i + k] = (float)v;
    }
    x[7 * (int64_t)i + 5] = ign_x;
    x[7 * (int64_t)i + 6] = ign_y;
  }
}

}  // namespace
}  // namespace firenn

using namespace firenn;

// ---------------------------------------------------------------------------
// Handle

namespace {
constexpr int kH = 256, kIn = 16, kD0C = 8, kD0S = 16, kDec = kD0C * kD0S * kD0S;
constexpr int kP = FIRE_NN_MAP * FIRE_NN_MAP;

struct Seg {
  int64_t off, n;
  int rows, cols;
};

struct Layout {
  Seg W1, c1, W2, c2, W3, c3, Wf, cf, Wd, cd, K1, k1, K2, k2, K3, k3;
  int64_t total;
  Layout() {
    int64_t o = 0;
    auto add = [&](int rows, int cols) { Seg s{o, (int64_t)rows * cols, rows, cols}; o += s.n; return s; };
    W1 = add(kIn, kH); c1 = add(1, kH);
    W2 = add(kH, kH); c2 = add(1, kH);
    W3 = add(kH, kH); c3 = add(1, kH);
    Wf = add(kH, 1); cf = add(1, 1);
    Wd = add(kH, kDec); cd = add(1, kDec);
    K1 = add(kD0C * kD0C, 9); k1 = add(1, kD0C);
    K2 = add(kD0C * kD0C, 9); k2 = add(1, kD0C);
    K3 = add(1 * kD0C, 9); k3 = add(1, 1);
    total = o;
  }
};
}  // namespace

struct fire_nn {
  int device = 0;
  fire_nn_cfg cfg{};
  std::string err;
  Layout L;
  float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;  // [total]
  uint16_t *wb = nullptr;                                        // bf16 copy [total]
  // activations (max_batch rows)
  uint16_t *xb = nullptr, *h1b = nullptr, *h2b = nullptr, *h3b = nullptr, *d0b = nullptr, *dtb = nullptr;
  float *h1 = nullptr, *h2 = nullptr, *h3 = nullptr, *t = nullptr, *d0 = nullptr, *d1 = nullptr,
        *d2 = nullptr, *z = nullptr;
  float *gt = nullptr, *gd0 = nullptr, *gd1 = nullptr, *gd2 = nullptr, *gz = nullptr, *gh = nullptr;
  uint16_t *ghb = nullptr;
  // bf16 copies the decoder's MFMA convolutions read
  uint16_t *d1b = nullptr, *d2b = nullptr, *gzb = nullptr, *gd1b = nullptr, *gd2b = nullptr;
  float *partial = nullptr, *loss = nullptr;
  float *wpart = nullptr;  // kernel-gradient partials [kWgradParts][16][80]
  std::vector<void *> allocs;
};

namespace {
fire_status nn_fail(fire_nn *nn, fire_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (nn) nn->err = buf;
  return s;
}
#define NN_HIP(nn, expr)                                                            \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return nn_fail((nn), e_ == hipErrorOutOfMemory ? FIRE_E_OOM : FIRE_E_DEVICE, \
                     "%s: %s", #expr, hipGetErrorString(e_));                       \
  } while (0)

template <class T>
hipError_t nn_alloc(fire_nn *nn, T **p, int64_t count) {
  hipError_t e = hipMalloc((void **)p, sizeof(T) * (size_t)(count > 0 ? count : 1));
  if (e == hipSuccess) nn->allocs.push_back(*p);
  return e;
}

// dynamic LDS of a decoder convolution staging c planes of r x r bf16
size_t conv_lds(int c, int r) { return sizeof(uint16_t) * (size_t)c * r * r; }

hipError_t refresh_bf16(fire_nn *nn, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(nn->L.total)), dim3(256), 0, s, nn->w, nn->wb,
                     nn->L.total);
  return hipGetLastError();
}

// Forward pass; the decoder (dense layer and upsampling convolutions) runs
// only when `want_map` (the fitness head does not depend on it).
hipError_t forward(fire_nn *nn, const float *x, int B, hipStream_t s, bool want_map) {
  const Layout &L = nn->L;
  hipError_t e;
  hipLaunchKernelGGL(prep_input_kernel, dim3(blocks_for((int64_t)B * 16)), dim3(256), 0, s, x, B,
                     1.0f / (float)nn->cfg.lattice_w, 1.0f / (float)nn->cfg.lattice_h, nn->xb);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const uint16_t *wb = nn->wb;
  const float *w = nn->w;
  if ((e = gemm(B, kH, kIn, nn->xb, kIn, 1, wb + L.W1.off, kH, 1, nn->h1, kH, w + L.c1.off, 1, 0,
                nn->h1b, s)) != hipSuccess) return e;
  if ((e = gemm(B, kH, kH, nn->h1b, kH, 1, wb + L.W2.off, kH, 1, nn->h2, kH, w + L.c2.off, 1, 0,
                nn->h2b, s)) != hipSuccess) return e;
  if ((e = gemm(B, kH, kH, nn->h2b, kH, 1, wb + L.W3.off, kH, 1, nn->h3, kH, w + L.c3.off, 1, 0,
                nn->h3b, s)) != hipSuccess) return e;
  if ((e = gemm(B, 1, kH, nn->h3b, kH, 1, wb + L.Wf.off, 1, 1, nn->t, 1, w + L.cf.off, 0, 0,
                nullptr, s)) != hipSuccess) return e;
  if (!want_map) return hipSuccess;
  if ((e = gemm(B, kDec, kH, nn->h3b, kH, 1, wb + L.Wd.off, kDec, 1, nn->d0, kDec, w + L.cd.off,
                1, 0, nn->d0b, s)) != hipSuccess) return e;
  // decoder: d0b (bf16 of d0, from the dense layer) -> d1 -> d2 -> z
  hipLaunchKernelGGL((upconv_mfma_kernel<true>), dim3(B), dim3(256), conv_lds(kD0C, 16), s,
                     nn->d0b, wb + L.K1.off, w + L.k1.off, 16, kD0C, 1, nullptr, nn->d1, nn->d1b);
  hipLaunchKernelGGL((upconv_mfma_kernel<true>), dim3(B), dim3(256), conv_lds(kD0C, 32), s,
                     nn->d1b, wb + L.K2.off, w + L.k2.off, 32, kD0C, 1, nullptr, nn->d2, nn->d2b);
  hipLaunchKernelGGL((upconv_mfma_kernel<true>), dim3(B), dim3(256), conv_lds(kD0C, 64), s,
                     nn->d2b, wb + L.K3.off, w + L.k3.off, 64, 1, 0, nullptr, nn->z, nullptr);
  return hipGetLastError();
}

// Kernel and bias gradients of one decoder layer: error g_b [B][Co][2S][2S]
// and layer input in_b [B][8][S][S] (both bf16).
hipError_t conv_weight_grad(fire_nn *nn, const uint16_t *g_b, const uint16_t *in_b, int B, int Co,
                            int S, float *dK, float *dkb, hipStream_t s) {
  const int parts = B < 512 ? B : 512;
  const int O = 2 * S;
  const size_t lds = sizeof(uint16_t) * ((size_t)(Co * O * O + 7) / 8 * 8 + (size_t)kD0C * S * S);
  hipLaunchKernelGGL(upconv_wgrad_mfma_kernel, dim3(parts), dim3(256), lds, s, g_b, in_b, B, S, Co,
                     nn->wpart);
  hipLaunchKernelGGL(wgrad_finish_kernel, dim3(Co * (kConvK + 1)), dim3(256), 0, s, nn->wpart,
                     parts, Co, dK, dkb);
  return hipGetLastError();
}

// loss and gradients into nn->g (forward must have run on the same x)
hipError_t backward(fire_nn *nn, const float *y_t, const uint8_t *y_map, int B, hipStream_t s) {
  const Layout &L = nn->L;
  hipError_t e;
  float *g = nn->g;
  const uint16_t *wb = nn->wb;
  hipLaunchKernelGGL(loss_fit_kernel, dim3(1), dim3(256), 0, s, nn->t, y_t, B, nn->gt, nn->dtb,
                     nn->loss);
  const int64_t nz = (int64_t)B * kP;
  const bool use_map = y_map != nullptr && nn->cfg.w_map > 0.0f;
  if (use_map) {
    const int nb = 1024;
    hipLaunchKernelGGL(loss_map_kernel, dim3(nb), dim3(256), 0, s, nn->z, y_map, nz,
                       nn->cfg.w_map, nn->gz, nn->partial);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, nn->partial, nb,
                       1.0f / (float)nz, nn->loss + 1);
    // decoder backward: each layer's error enters its two MFMA products as
    // bf16; the data gradient comes back summed over the 2x2 upsampling
    // blocks and masked by the layer input's ReLU
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(nz)), dim3(256), 0, s, nn->gz, nn->gzb, nz);
    // last layer (one output channel): kernel, bias and data gradients from
    // the same 2x2 box sums of the error
    {
      const int64_t blocks = ((int64_t)B * 64 * 32 + 255) / 256;
      const int parts = (int)(blocks < kWgradParts ? blocks : kWgradParts);
      hipLaunchKernelGGL(upconv_grads_co1_kernel, dim3(parts), dim3(256), 0, s, nn->gzb,
                         nn->d2b, B, 64, nn->wpart, wb + L.K3.off, nn->d2, nn->gd2, nn->gd2b);
      hipLaunchKernelGGL(wgrad_finish_kernel, dim3(kConvK + 1), dim3(256), 0, s, nn->wpart, parts,
                         1, g + L.K3.off, g + L.k3.off);
    }
    if ((e = conv_weight_grad(nn, nn->gd2b, nn->d1b, B, kD0C, 32, g + L.K2.off, g + L.k2.off, s)) != hipSuccess) return e;
    hipLaunchKernelGGL((upconv_mfma_kernel<false>), dim3(B), dim3(256), conv_lds(kD0C, 64), s,
                       nn->gd2b, wb + L.K2.off, nullptr, 32, kD0C, 0, nn->d1, nn->gd1, nn->gd1b);
    if ((e = conv_weight_grad(nn, nn->gd1b, nn->d0b, B, kD0C, 16, g + L.K1.off, g + L.k1.off, s)) != hipSuccess) return e;
    // the last data gradient's bf16 copy replaces d0b, which the dense
    // layer's gradient products read next
    hipLaunchKernelGGL((upconv_mfma_kernel<false>), dim3(B), dim3(256), conv_lds(kD0C, 32), s,
                       nn->gd1b, wb + L.K1.off, nullptr, 16, kD0C, 0, nn->d0, nn->gd0, nn->d0b);
    // dense decoder layer: gd0 already carries the ReLU mask of d0
    if ((e = gemm(kH, kDec, B, nn->h3b, 1, kH, nn->d0b, kDec, 1, g + L.Wd.off, kDec, nullptr, 0,
                  0, nullptr, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(colsum_kernel, dim3(colsum_blocks(kDec)), dim3(256), 0, s, nn->gd0, B, kDec,
                       g + L.cd.off);
  } else {
    hipLaunchKernelGGL(fill_f32_kernel, dim3(1), dim3(64), 0, s, nn->loss + 1, 0.0f, (int64_t)1);
    const int64_t o = L.Wd.off, n = L.k3.off + L.k3.n - L.Wd.off;
    hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks_for(n)), dim3(256), 0, s, g + o, 0.0f, n);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // fitness head
  if ((e = gemm(kH, 1, B, nn->h3b, 1, kH, nn->dtb, 1, 1, g + L.Wf.off, 1, nullptr, 0, 0, nullptr,
                s)) != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(256), 0, s, nn->gt, B, 1, g + L.cf.off);
  // dh3 = dt Wf^T (+ dd0 Wd^T)
  if ((e = gemm(B, kH, 1, nn->dtb, 1, 1, wb + L.Wf.off, 1, 1, nn->gh, kH, nullptr, 0, 0, nullptr,
                s)) != hipSuccess) return e;
  if (use_map)
    if ((e = gemm(B, kH, kDec, nn->d0b, kDec, 1, wb + L.Wd.off, 1, kDec, nn->gh, kH, nullptr, 0, 1,
                  nullptr, s)) != hipSuccess) return e;
  // through the three hidden layers
  struct Lay { const uint16_t *in_b; const float *act; const Seg *W; const Seg *c; int kin; };
  const Lay lays[3] = {{nn->h2b, nn->h3, &L.W3, &L.c3, kH},
                       {nn->h1b, nn->h2, &L.W2, &L.c2, kH},
                       {nn->xb, nn->h1, &L.W1, &L.c1, kIn}};
  for (int li = 0; li < 3; ++li) {
    const Lay &ly = lays[li];
    hipLaunchKernelGGL(relu_bwd_kernel, dim3(blocks_for((int64_t)B * kH)), dim3(256), 0, s, nn->gh,
                       ly.act, nn->ghb, (int64_t)B * kH);
    if ((e = gemm(ly.kin, kH, B, ly.in_b, 1, ly.kin, nn->ghb, kH, 1, g + ly.W->off, kH, nullptr, 0,
                  0, nullptr, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(colsum_kernel, dim3(colsum_blocks(kH)), dim3(256), 0, s, nn->gh, B, kH,
                       g + ly.c->off);
    if (li < 2)
      if ((e = gemm(B, kH, kH, nn->ghb, kH, 1, wb + ly.W->off, 1, kH, nn->gh, kH, nullptr, 0, 0,
                    nullptr, s)) != hipSuccess) return e;
  }
  return hipGetLastError();
}
}  // namespace

extern "C" {

fire_status fire_nn_create(int device, const fire_nn_cfg *cfg, uint64_t seed, fire_nn **out) {
  if (!out || !cfg) return FIRE_E_INVALID;
  *out = nullptr;
  if (cfg->max_batch < 1 || cfg->max_batch > (1 << 16) || cfg->lattice_w < 1 || cfg->lattice_h < 1 ||
      !(cfg->w_map >= 0.0f) || !(cfg->adam_b1 >= 0.0f && cfg->adam_b1 < 1.0f) ||
      !(cfg->adam_b2 >= 0.0f && cfg->adam_b2 < 1.0f) || !(cfg->adam_eps > 0.0f))
    return FIRE_E_INVALID;
  fire_nn *nn = new (std::nothrow) fire_nn();
  if (!nn) return FIRE_E_OOM;
  nn->device = device;
  nn->cfg = *cfg;
  const int64_t Bm = cfg->max_batch, T = nn->L.total;
  auto fail_out = [&](hipError_t e) {
    fire_nn_destroy(nn);
    return e == hipErrorOutOfMemory ? FIRE_E_OOM : FIRE_E_DEVICE;
  };
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->w, T);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->m, T);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->v, T);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->g, T);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->wb, T);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->xb, Bm * kIn);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->h1b, Bm * kH);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->h2b, Bm * kH);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->h3b, Bm * kH);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->d0b, Bm * kDec);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->dtb, Bm);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->ghb, Bm * kH);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->h1, Bm * kH);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->h2, Bm * kH);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->h3, Bm * kH);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->t, Bm);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->d0, Bm * kDec);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->d1, Bm * kD0C * 32 * 32);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->d2, Bm * kD0C * 64 * 64);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->z, Bm * kP);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->gt, Bm);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->gd0, Bm * kDec);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->gd1, Bm * kD0C * 32 * 32);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->gd2, Bm * kD0C * 64 * 64);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->gz, Bm * kP);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->gh, Bm * kH);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->partial, (int64_t)1024);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->wpart, (int64_t)kWgradParts * kWgradRows * kWgradCols);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->d1b, Bm * kD0C * 32 * 32);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->d2b, Bm * kD0C * 64 * 64);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->gzb, Bm * kP);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->gd1b, Bm * kD0C * 32 * 32);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->gd2b, Bm * kD0C * 64 * 64);
  // the decoder kernels stage up to 96 KiB of planes in LDS
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&upconv_wgrad_mfma_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&upconv_mfma_kernel<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&upconv_mfma_kernel<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
  if (e == hipSuccess) e = nn_alloc(nn, &nn->loss, 2);
  if (e != hipSuccess) return fail_out(e);
  // initial parameters
  const Layout &L = nn->L;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks_for(T)), dim3(256), 0, nullptr, nn->w, 0.0f, T);
  hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks_for(T)), dim3(256), 0, nullptr, nn->m, 0.0f, T);
  hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks_for(T)), dim3(256), 0, nullptr, nn->v, 0.0f, T);
  struct Init { const Seg *s; float fan_in, fan_out; int rows_used; };
  const Init inits[] = {{&L.W1, (float)FIRE_NN_IN, (float)kH, FIRE_NN_IN}, {&L.W2, kH, kH, 0},
                        {&L.W3, kH, kH, 0}, {&L.Wf, kH, 1, 0}, {&L.Wd, kH, kDec, 0},
                        {&L.K1, kD0C * 9.0f, kD0C * 9.0f, 0}, {&L.K2, kD0C * 9.0f, kD0C * 9.0f, 0},
                        {&L.K3, kD0C * 9.0f, 9.0f, 0}};
  uint32_t tensor = 1;
  for (const Init &in : inits) {
    const float limit = sqrtf(6.0f / (in.fan_in + in.fan_out));
    hipLaunchKernelGGL(init_uniform_kernel, dim3(blocks_for(in.s->n)), dim3(256), 0, nullptr,
                       nn->w + in.s->off, in.s->n, limit, tensor++, k0, k1, in.rows_used, in.s->cols);
  }
  e = refresh_bf16(nn, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return fail_out(e);
  *out = nn;
  return FIRE_OK;
}

void fire_nn_destroy(fire_nn *nn) {
  if (!nn) return;
  (void)hipSetDevice(nn->device);
  (void)hipDeviceSynchronize();
  for (void *p : nn->allocs) (void)hipFree(p);
  delete nn;
}

const char *fire_nn_last_error(const fire_nn *nn) { return nn ? nn->err.c_str() : "null handle"; }

int64_t fire_nn_num_params(const fire_nn *nn) { return nn ? nn->L.total : 0; }

fire_status fire_nn_get_params(fire_nn *nn, float *out, void *stream) {
  if (!nn) return FIRE_E_INVALID;
  if (!out) return nn_fail(nn, FIRE_E_INVALID, "null output");
  NN_HIP(nn, hipSetDevice(nn->device));
  NN_HIP(nn, hipMemcpyAsync(out, nn->w, sizeof(float) * nn->L.total, hipMemcpyDeviceToDevice,
                            (hipStream_t)stream));
  return FIRE_OK;
}

fire_status fire_nn_set_params(fire_nn *nn, const float *in, void *stream) {
  if (!nn) return FIRE_E_INVALID;
  if (!in) return nn_fail(nn, FIRE_E_INVALID, "null input");
  NN_HIP(nn, hipSetDevice(nn->device));
  NN_HIP(nn, hipMemcpyAsync(nn->w, in, sizeof(float) * nn->L.total, hipMemcpyDeviceToDevice,
                            (hipStream_t)stream));
  NN_HIP(nn, refresh_bf16(nn, (hipStream_t)stream));
  return FIRE_OK;
}

fire_status fire_nn_forward(fire_nn *nn, const float *x, int32_t B, float *out_t, float *out_map,
                            void *stream) {
  if (!nn) return FIRE_E_INVALID;
  if (!x || !out_t || B < 1 || B > nn->cfg.max_batch)
    return nn_fail(nn, FIRE_E_INVALID, "bad batch (1..%d) or null pointer", nn->cfg.max_batch);
  NN_HIP(nn, hipSetDevice(nn->device));
  hipStream_t s = (hipStream_t)stream;
  NN_HIP(nn, forward(nn, x, B, s, out_map != nullptr));
  NN_HIP(nn, hipMemcpyAsync(out_t, nn->t, sizeof(float) * B, hipMemcpyDeviceToDevice, s));
  if (out_map) {
    hipLaunchKernelGGL(sigmoid_kernel, dim3(blocks_for((int64_t)B * kP)), dim3(256), 0, s, nn->z,
                       out_map, (int64_t)B * kP);
    NN_HIP(nn, hipGetLastError());
  }
  return FIRE_OK;
}

fire_status fire_nn_gradients(fire_nn *nn, const float *x, const float *y_t, const uint8_t *y_map,
                              int32_t B, float *out_loss, float *out_grads, void *stream) {
  if (!nn) return FIRE_E_INVALID;
  if (!x || !y_t || !out_loss || B < 1 || B > nn->cfg.max_batch)
    return nn_fail(nn, FIRE_E_INVALID, "bad batch (1..%d) or null pointer", nn->cfg.max_batch);
  NN_HIP(nn, hipSetDevice(nn->device));
  hipStream_t s = (hipStream_t)stream;
  NN_HIP(nn, forward(nn, x, B, s, y_map != nullptr && nn->cfg.w_map > 0.0f));
  NN_HIP(nn, backward(nn, y_t, y_map, B, s));
  NN_HIP(nn, hipMemcpyAsync(out_loss, nn->loss, 2 * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (out_grads)
    NN_HIP(nn, hipMemcpyAsync(out_grads, nn->g, sizeof(float) * nn->L.total,
                              hipMemcpyDeviceToDevice, s));
  return FIRE_OK;
}

fire_status fire_nn_train_step(fire_nn *nn, const float *x, const float *y_t, const uint8_t *y_map,
                               int32_t B, float lr, int32_t step, float *out_loss, void *stream) {
  if (!nn) return FIRE_E_INVALID;
  if (!x || !y_t || B < 1 || B > nn->cfg.max_batch || step < 1 || !(lr > 0.0f))
    return nn_fail(nn, FIRE_E_INVALID, "bad batch, step or learning rate");
  NN_HIP(nn, hipSetDevice(nn->device));
  hipStream_t s = (hipStream_t)stream;
  NN_HIP(nn, forward(nn, x, B, s, y_map != nullptr && nn->cfg.w_map > 0.0f));
  NN_HIP(nn, backward(nn, y_t, y_map, B, s));
  const float c1 = 1.0f - powf(nn->cfg.adam_b1, (float)step);
  const float c2 = 1.0f - powf(nn->cfg.adam_b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(nn->L.total)), dim3(256), 0, s, nn->w, nn->wb,
                     nn->m, nn->v, nn->g, nn->L.total, lr, nn->cfg.adam_b1, nn->cfg.adam_b2,
                     nn->cfg.adam_eps, c1, c2);
  NN_HIP(nn, hipGetLastError());
  if (out_loss)
    NN_HIP(nn, hipMemcpyAsync(out_loss, nn->loss, 2 * sizeof(float), hipMemcpyDeviceToDevice, s));
  return FIRE_OK;
}

fire_status fire_gemm_bf16(int M, int N, int K, const uint16_t *A, int64_t sam, int64_t sak,
                           const uint16_t *Bm, int64_t sbk, int64_t sbn, float *C, int64_t ldc,
                           const float *bias, int relu, int accumulate, uint16_t *Cb,
                           void *stream) {
  if (M < 1 || N < 1 || K < 1 || !A || !Bm || !C || ldc < N) return FIRE_E_INVALID;
  if (gemm(M, N, K, A, sam, sak, Bm, sbk, sbn, C, ldc, bias, relu, accumulate, Cb,
           (hipStream_t)stream) != hipSuccess)
    return FIRE_E_DEVICE;
  return FIRE_OK;
}

fire_status fire_pool_maps(const uint32_t *maps, int32_t n, int32_t W, int32_t H,
                           int64_t map_words, int32_t out_w, int32_t out_h, uint8_t *out,
                           void *stream) {
  if (!maps || !out || n < 0 || W < 1 || H < 1 || out_w < 1 || out_h < 1 || out_w > W ||
      out_h > H || map_words < (int64_t)H * ((W + 31) / 32))
    return FIRE_E_INVALID;
  if (n == 0) return FIRE_OK;
  const int64_t total = (int64_t)n * out_w * out_h;
  hipLaunchKernelGGL(pool_maps_kernel, dim3(blocks_for(total)), dim3(256), 0, (hipStream_t)stream,
                     maps, n, W, H, map_words, out_w, out_h, out);
  return hipGetLastError() == hipSuccess ? FIRE_OK : FIRE_E_DEVICE;
}

fire_status fire_colsum_f32(const float *d, int32_t M, int32_t N, float *out, void *stream) {
  if (!d || !out || M < 1 || N < 1) return FIRE_E_INVALID;
  hipLaunchKernelGGL(colsum_kernel, dim3(colsum_blocks(N)), dim3(256), 0, (hipStream_t)stream, d,
                     M, N, out);
  return hipGetLastError() == hipSuccess ? FIRE_OK : FIRE_E_DEVICE;
}

fire_status fire_nn_select(const double *cand, const float *score, int32_t n, int32_t G,
                           int32_t keep, int32_t k, double *out, int32_t *out_idx, void *stream) {
  if (!cand || !score || !out || n < 1 || n > 4096 || G < 1 || k < 1 || k > n || keep < 0 ||
      keep > k)
    return FIRE_E_INVALID;
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, cand, score, n,
                     G, keep, k, out, out_idx);
  return hipGetLastError() == hipSuccess ? FIRE_OK : FIRE_E_DEVICE;
}

fire_status fire_nn_rows_from_results(const double *params, int32_t reps, const float *ign,
                                      float ign_x, float ign_y, const fire_result *results,
                                      int32_t n, float *out_x, float *out_y, double *out_fit,
                                      void *stream) {
  if (n < 0 || !results || reps < 1 || (out_x && !params)) return FIRE_E_INVALID;
  if (n == 0) return FIRE_OK;
  hipLaunchKernelGGL(rows_from_results_kernel, dim3(blocks_for(n)), dim3(256), 0,
                     (hipStream_t)stream, params, reps, ign, ign_x, ign_y, results, n, out_x,
                     out_y, out_fit);
  return hipGetLastError() == hipSuccess ? FIRE_OK : FIRE_E_DEVICE;
}

fire_status fire_gather_rows(const void *src, int64_t row_bytes, const int64_t *rows, int32_t n,
                             void *dst, void *stream) {
  if (n < 0 || row_bytes < 4 || row_bytes % 4 != 0 || (n > 0 && (!src || !rows || !dst)))
    return FIRE_E_INVALID;
  if (n == 0) return FIRE_OK;
  const int vec = row_bytes % 16 == 0 && (uintptr_t)src % 16 == 0 && (uintptr_t)dst % 16 == 0;
  const int64_t words = row_bytes / 4;
  hipLaunchKernelGGL(gather_rows_kernel,
                     dim3(blocks_for((int64_t)n * (vec ? words / 4 : words))), dim3(256), 0,
                     (hipStream_t)stream, (const uint32_t *)src, words, rows, n, (uint32_t *)dst,
                     vec);
  return hipGetLastError() == hipSuccess ? FIRE_OK : FIRE_E_DEVICE;
}

fire_status fire_nn_candidates(const double *sets, int32_t n_sets, int32_t P, int32_t E,
                               float ign_x, float ign_y, double *cand, float *x, void *stream) {
  if (!sets || !cand || !x || n_sets < 1 || P < 1 || E < 0 || E >= P) return FIRE_E_INVALID;
  const int n = P + (n_sets - 1) * (P - E);
  hipLaunchKernelGGL(candidates_kernel, dim3(blocks_for(n)), dim3(256), 0,
                     (hipStream_t)stream, sets, n_sets, P, E, ign_x, ign_y, cand, x);
  return hipGetLastError() == hipSuccess ? FIRE_OK : FIRE_E_DEVICE;
}

}  // extern "C"
