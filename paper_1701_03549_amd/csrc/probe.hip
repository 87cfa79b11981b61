// Hardware probes of the running GPU (gfx950): the ceilings the simulation
// kernels are measured against. Streaming reads from a buffer that stays in
// L2, in the last-level (MALL) cache or in HBM; the throughput of the
// Philox4x32-10 generator the simulations draw their coins from; and the
// latencies that make up one step of a simulation (workgroup barrier,
// dependent global load served by L2, dependent LDS atomic, dependent
// Philox evaluation). Each probe is timed by its caller with events on the
// launch stream (bandwidth, throughput) or times itself with the constant
// 100 MHz wall clock (latencies).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fire_probe.h"

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Philox4x32-10 (Salmon et al., SC'11), written out as in the simulation
// kernels: ten rounds of two 32x32->64 multiplies and xors.
__device__ __forceinline__ void philox_rounds(uint32_t &c0, uint32_t &c1, uint32_t &c2,
                                              uint32_t &c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p2 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p2 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p2;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Every workgroup reads `words16` 16-byte words from `buf` `passes` times
// (whole buffer per workgroup when `per_block`, else a grid-stride share).
__global__ __launch_bounds__(256) void read_kernel(const u32x4 *buf, int64_t words16, int passes,
                                                   int per_block, uint32_t *sink) {
  uint32_t acc = 0;
  const int64_t start = per_block ? threadIdx.x : blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t step = per_block ? blockDim.x : (int64_t)gridDim.x * blockDim.x;
  for (int p = 0; p < passes; ++p) {
    // the pass index enters the value so passes are not folded together
    for (int64_t i = start; i < words16; i += step) {
      const u32x4 v = buf[i];
      acc ^= (v.x + (uint32_t)p) ^ v.y ^ v.z ^ v.w;
    }
  }
  if (acc == 0x9E3779B9u) sink[blockIdx.x] = acc;  // practically never; keeps the loads
}

__global__ __launch_bounds__(256) void philox_kernel(uint32_t iters, uint32_t k0, uint32_t k1,
                                                     uint32_t *sink) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (uint32_t i = 0; i < iters; ++i) {
    uint32_t c0 = t, c1 = i, c2 = 0x1234u, c3 = 1u;
    philox_rounds(c0, c1, c2, c3, k0, k1);
    acc ^= c0 ^ c1 ^ c2 ^ c3;
  }
  if (acc == 0x9E3779B9u) sink[t] = acc;
}

// One workgroup of 256 threads. kind 0: workgroup barriers; 1: dependent
// global loads (pointer chase over `chain`, n entries); 2: dependent LDS
// atomics; 3: dependent Philox evaluations. out[0] = wall-clock ticks of
// `iters` operations (thread 0), out[1] = a value that depends on all of
// them.
__global__ __launch_bounds__(256) void latency_kernel(int kind, int iters, const uint32_t *chain,
                                                      uint32_t n, uint64_t *out) {
  __shared__ uint32_t sh[256];
  sh[threadIdx.x] = threadIdx.x;
  __syncthreads();
  uint64_t t0 = 0, t1 = 0;
  uint32_t v = 0;
  if (kind == 0) {
    t0 = wall_clock64();
    for (int i = 0; i < iters; ++i) __syncthreads();
    t1 = wall_clock64();
  } else if (threadIdx.x == 0) {
    if (kind == 1) {
      uint32_t p = 0;
      for (int i = 0; i < 64; ++i) p = chain[p];  // warm the cache
      t0 = wall_clock64();
      for (int i = 0; i < iters; ++i) p = chain[p] % n;
      t1 = wall_clock64();
      v = p;
    } else if (kind == 2) {
      uint32_t p = 0;
      t0 = wall_clock64();
      for (int i = 0; i < iters; ++i) p = atomicAdd(&sh[p & 255u], 1u) & 255u;
      t1 = wall_clock64();
      v = p;
    } else {
      uint32_t c0 = 1, c1 = 2, c2 = 3, c3 = 4;
      t0 = wall_clock64();
      for (int i = 0; i < iters; ++i) philox_rounds(c0, c1, c2, c3, 0x5EED0001u, (uint32_t)i);
      t1 = wall_clock64();
      v = c0 ^ c1 ^ c2 ^ c3;
    }
  }
  if (threadIdx.x == 0) {
    out[0] = t1 - t0;
    out[1] = v;
  }
}

}  // namespace

extern "C" {

fire_status fire_probe_read(const void *buf, int64_t bytes, int32_t passes, int32_t per_block,
                            int32_t grid, uint32_t *sink, void *stream) {
  if (!buf || !sink || bytes < 16 || (bytes % 16) != 0 || passes < 1 || grid < 1 ||
      (((uintptr_t)buf) % 16) != 0)
    return FIRE_E_INVALID;
  hipLaunchKernelGGL(read_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream,
                     (const u32x4 *)buf, bytes / 16, passes, per_block, sink);
  return hipGetLastError() == hipSuccess ? FIRE_OK : FIRE_E_DEVICE;
}

fire_status fire_probe_philox(uint32_t iters, int32_t grid, uint32_t *sink, void *stream) {
  if (!sink || grid < 1 || iters < 1) return FIRE_E_INVALID;
  hipLaunchKernelGGL(philox_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, iters,
                     0x5EED0001u, 0u, sink);
  return hipGetLastError() == hipSuccess ? FIRE_OK : FIRE_E_DEVICE;
}

fire_status fire_probe_latency(int32_t kind, int32_t iters, const uint32_t *chain, uint32_t n,
                               uint64_t *out, void *stream) {
  if (!out || kind < 0 || kind > 3 || iters < 1 || (kind == 1 && (!chain || n < 1)))
    return FIRE_E_INVALID;
  hipLaunchKernelGGL(latency_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, kind, iters,
                     chain, n, out);
  return hipGetLastError() == hipSuccess ? FIRE_OK : FIRE_E_DEVICE;
}

}  // extern "C"
