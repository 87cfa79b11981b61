// CPU stand-ins for the device features sim_kernel uses, so that the kernel's
// own source runs with one OS thread per GPU thread: __syncthreads is a
// barrier of the workgroup's threads, wave operations (ballot, readfirstlane)
// are a rendezvous of the wave's 64 threads, the lane-pair shuffle a
// rendezvous of two, atomics take one global lock, and LDS is a per-workgroup
// buffer. Memory is sequentially consistent between barriers; a watchdog in
// emu_wg.cpp reports a barrier that never completes.
#pragma once
#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

struct Dim3 { unsigned x = 0, y = 0, z = 0; };
struct uint4 { uint32_t x, y, z, w; };
inline uint4 make_uint4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) { return {a, b, c, d}; }

// A generation-counting barrier; a thread that leaves the kernel drops out.
struct Barrier {
  explicit Barrier(int n) : expected(n), count(n) {}
  void arrive_and_wait() {
    std::unique_lock<std::mutex> lk(mu);
    const long gen = generation;
    if (--count == 0) { count = expected; ++generation; cv.notify_all(); return; }
    cv.wait(lk, [&] { return generation != gen; });
  }
  void arrive_and_drop() {
    std::unique_lock<std::mutex> lk(mu);
    --expected;
    if (--count == 0) { count = expected; ++generation; cv.notify_all(); }
  }
  std::mutex mu;
  std::condition_variable cv;
  int expected, count;
  long generation = 0;
};

// Per workgroup: its barriers, the exchange slots of wave operations, and
// the per-thread record of the step-loop check.
struct WgCtx {
  Barrier *block = nullptr;
  std::vector<Barrier *> wave, pair;
  uint64_t slots[1024];
  uint32_t agree[1024][4];
};

// Thread identity and workgroup (each emulated thread sets its own).
extern thread_local Dim3 threadIdx, blockIdx;
extern Dim3 blockDim, gridDim;
extern thread_local uint32_t *g_lds;
extern thread_local WgCtx *g_wg;
extern thread_local int *g_where;   // source line of the barrier a thread waits at
extern std::atomic<long> g_progress;
extern std::mutex g_atomic_mu;

template <class T> inline T min(T a, T b) { return a < b ? a : b; }
template <class T> inline T max(T a, T b) { return a < b ? b : a; }
inline double rint(double x) { return std::nearbyint(x); }
inline uint64_t wall_clock64() { return 0; }
inline double __builtin_amdgcn_ldexp(double x, int n) { return std::ldexp(x, n); }
inline double __builtin_amdgcn_rcp(double x) { return 1.0 / x; }

inline void wg_sync(int line) {
  *g_where = line;
  g_wg->block->arrive_and_wait();
  g_progress.fetch_add(1, std::memory_order_relaxed);
  *g_where = -line;
}
#define __syncthreads() wg_sync(__LINE__)

inline void wave_sync(int line) {
  *g_where = 100000 + line;
  g_wg->wave[threadIdx.x / 64]->arrive_and_wait();
  *g_where = -(100000 + line);
}
inline uint64_t ballot_impl(bool p, int line) {
  const unsigned t = threadIdx.x, w0 = t & ~63u;
  g_wg->slots[t] = p;
  wave_sync(line);
  uint64_t m = 0;
  for (int i = 0; i < 64; ++i) if (g_wg->slots[w0 + i]) m |= 1ull << i;
  wave_sync(line);
  return m;
}
#define __ballot(p) ballot_impl((p), __LINE__)
inline uint32_t readfirstlane_impl(uint32_t v, int line) {
  const unsigned t = threadIdx.x, w0 = t & ~63u;
  g_wg->slots[t] = v;
  wave_sync(line);
  const uint32_t r = (uint32_t)g_wg->slots[w0];
  wave_sync(line);
  return r;
}
#define __builtin_amdgcn_readfirstlane(v) readfirstlane_impl((v), __LINE__)
inline int shfl_xor1_impl(int v, int mask, int line) {
  if (mask != 1) { fprintf(stderr, "emulated shuffle supports mask 1 only\n"); abort(); }
  const unsigned t = threadIdx.x;
  g_wg->slots[t] = (uint32_t)v;
  *g_where = 200000 + line;
  g_wg->pair[t / 2]->arrive_and_wait();
  const int r = (int)(uint32_t)g_wg->slots[t ^ 1u];
  g_wg->pair[t / 2]->arrive_and_wait();
  *g_where = -(200000 + line);
  return r;
}
#define __shfl_xor(v, m) shfl_xor1_impl((v), (m), __LINE__)
inline uint32_t mbcnt_lo(uint32_t m, uint32_t acc) {
  const unsigned l = threadIdx.x % 64;
  const uint32_t mask = l >= 32 ? 0xFFFFFFFFu : ((1u << l) - 1u);
  return acc + __builtin_popcount(m & mask);
}
inline uint32_t mbcnt_hi(uint32_t m, uint32_t acc) {
  const unsigned l = threadIdx.x % 64;
  const uint32_t mask = l <= 32 ? 0u : ((1u << (l - 32)) - 1u);
  return acc + __builtin_popcount(m & mask);
}
#define __builtin_amdgcn_mbcnt_lo(m, a) mbcnt_lo((m), (a))
#define __builtin_amdgcn_mbcnt_hi(m, a) mbcnt_hi((m), (a))
#define __popc(x) __builtin_popcount((uint32_t)(x))
#define __popcll(x) __builtin_popcountll((uint64_t)(x))
// __hip_atomic_load / store / fetch_or are clang builtins on the host too
#ifndef __HIP_MEMORY_SCOPE_AGENT
#define __HIP_MEMORY_SCOPE_AGENT 3
#endif
template <class T> T atomicAdd(T *p, T v) { std::lock_guard<std::mutex> g(g_atomic_mu); T o = *p; *p = o + v; return o; }
template <class T> T atomicOr(T *p, T v) { std::lock_guard<std::mutex> g(g_atomic_mu); T o = *p; *p = o | v; return o; }
inline uint32_t __float_as_uint(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }
inline float __uint_as_float(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }

// The check the generator inserts at the top of sim_kernel's step loop:
// every thread of the workgroup must see the same frontier length, abort
// flag, step and simulation there, or the threads would leave the loop at
// different steps and wait at different barriers.
inline void step_agree(uint32_t n_cur, bool aborted, uint32_t step, uint32_t sim, int line) {
  const unsigned t = threadIdx.x;
  uint32_t *mine = g_wg->agree[t];
  mine[0] = n_cur; mine[1] = aborted; mine[2] = step; mine[3] = sim;
  wg_sync(line);
  if (t == 0) {
    for (unsigned o = 1; o < blockDim.x; ++o) {
      const uint32_t *q = g_wg->agree[o];
      if (q[0] != n_cur || q[1] != (uint32_t)aborted || q[2] != step || q[3] != sim) {
        fprintf(stderr,
                "threads disagree in workgroup %u at step %u of simulation %u: thread 0 sees "
                "front %u abort %d, thread %u sees front %u abort %u step %u simulation %u\n",
                blockIdx.x, step, sim, n_cur, (int)aborted, o, q[0], q[1], q[2], q[3]);
        fflush(stderr);
        abort();
      }
    }
  }
  wg_sync(line);
}
#define EMU_STEP_AGREE(n, ab, st, sm) step_agree((n), (ab), (st), (sm), __LINE__)
