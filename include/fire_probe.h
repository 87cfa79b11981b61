/*
 * fire_probe.h -- hardware probes of the running GPU (MI355X / gfx950): the
 * ceilings the simulation kernels of fire.h are measured against. Not part
 * of the paper's method; they turn the paper's observation that its kernels
 * are memory-bound (performance-analysis section) into measured numbers on
 * this hardware: which ceiling a step of a simulation actually meets.
 *
 * All pointers are device pointers; `stream` is a hipStream_t. Each call
 * launches one kernel and returns; the caller times bandwidth and
 * throughput probes with events on `stream`. Errors are returned
 * (FIRE_E_INVALID for bad arguments, checked before any device work).
 */
#ifndef FIRE_PROBE_H_
#define FIRE_PROBE_H_

#include <stdint.h>

#include "fire.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Streaming read of `bytes` (a multiple of 16, 16-byte aligned buffer)
 * `passes` times by `grid` workgroups of 256 threads, 16 bytes per load,
 * coalesced. per_block = 1: every workgroup reads the whole buffer (a
 * buffer of a few MiB then stays in each XCD's L2); 0: the workgroups
 * share the buffer in grid stride (a buffer larger than L2 and smaller
 * than the last-level cache is then served from it after the first pass;
 * one pass over a much larger buffer measures HBM). Bytes read =
 * bytes * passes * (per_block ? grid : 1). sink [grid] receives at most a
 * checksum word. */
fire_status fire_probe_read(const void *buf, int64_t bytes, int32_t passes, int32_t per_block,
                            int32_t grid, uint32_t *sink, void *stream);

/* Philox4x32-10 throughput: grid * 256 threads each evaluate `iters`
 * independent calls (counter (thread, i, 0x1234, 1)); calls =
 * grid * 256 * iters. sink [grid * 256]. */
fire_status fire_probe_philox(uint32_t iters, int32_t grid, uint32_t *sink, void *stream);

/* Latency of `iters` dependent operations in one workgroup of 256 threads,
 * timed in the kernel with the 100 MHz wall clock: kind 0 workgroup
 * barriers (4 wavefronts); 1 global loads, each address taken from the
 * previous load (chain [n] holds the next index, a cycle; a chain of a few
 * hundred KiB is served by L2); 2 LDS atomic adds whose addresses depend
 * on the previous result; 3 Philox4x32-10 evaluations, each on the
 * previous output. out [2]: wall-clock ticks, a checksum. */
fire_status fire_probe_latency(int32_t kind, int32_t iters, const uint32_t *chain, uint32_t n,
                               uint64_t *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FIRE_PROBE_H_ */
