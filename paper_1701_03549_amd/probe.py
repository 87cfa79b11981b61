"""Hardware ceilings of the running GPU, measured with the probes of
include/fire_probe.h (argument marshalling and timing only).

measure() returns streaming-read bandwidth from L2, from the last-level
(MALL) cache and from HBM, Philox4x32-10 throughput, and the latencies that
make up one simulation step (workgroup barrier, dependent global load
served by L2, dependent LDS atomic, dependent Philox evaluation).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import fire

EXPORTS = ["fire_probe_read", "fire_probe_philox", "fire_probe_latency"]
_done = False


def _lib():
    global _done
    lib = fire.load_library()
    if not _done:
        vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        sig = {"fire_probe_read": (i32, [vp, i64, i32, i32, i32, vp, vp]),
               "fire_probe_philox": (i32, [u32, i32, vp, vp]),
               "fire_probe_latency": (i32, [i32, i32, vp, u32, vp, vp])}
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype, f.argtypes = res, args
        _done = True
    return lib


def _time(fn, reps):
    """Median milliseconds of fn() over reps launches (events on the current stream)."""
    s = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn()
        b.record(s)
        b.synchronize()
        ms.append(a.elapsed_time(b))
    return float(np.median(ms))


def read_bandwidth(nbytes: int, passes: int, per_block: bool, grid: int, reps: int = 5) -> float:
    """GB/s of streaming 16-byte reads (see fire_probe_read)."""
    lib = _lib()
    buf = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    sink = torch.zeros(grid, dtype=torch.int32, device="cuda")
    st = int(torch.cuda.current_stream().cuda_stream)

    def run():
        r = lib.fire_probe_read(buf.data_ptr(), nbytes, passes, int(per_block), grid,
                                sink.data_ptr(), st)
        if r != 0:
            raise fire.FireError(r, "fire_probe_read failed")
    ms = _time(run, reps)
    total = nbytes * passes * (grid if per_block else 1)
    del buf
    return total / (ms * 1e-3) / 1e9


def philox_rate(grid: int, iters: int = 256, reps: int = 5) -> float:
    """Philox4x32-10 calls per second over the whole GPU."""
    lib = _lib()
    sink = torch.zeros(grid * 256, dtype=torch.int32, device="cuda")
    st = int(torch.cuda.current_stream().cuda_stream)

    def run():
        r = lib.fire_probe_philox(iters, grid, sink.data_ptr(), st)
        if r != 0:
            raise fire.FireError(r, "fire_probe_philox failed")
    ms = _time(run, reps)
    return grid * 256 * iters / (ms * 1e-3)


def latency_ns(kind: int, iters: int = 4096, chain_bytes: int = 1 << 20) -> float:
    """Nanoseconds per dependent operation (fire_probe_latency kinds 0..3)."""
    lib = _lib()
    n = chain_bytes // 4
    chain = None
    if kind == 1:
        # a random cycle over n entries, 64 bytes apart on average
        perm = np.random.default_rng(1).permutation(n).astype(np.uint32)
        nxt = np.empty(n, dtype=np.uint32)
        nxt[perm] = np.roll(perm, -1)
        chain = torch.from_numpy(nxt.view(np.int32)).cuda()
    out = torch.zeros(2, dtype=torch.int64, device="cuda")
    st = int(torch.cuda.current_stream().cuda_stream)
    r = lib.fire_probe_latency(kind, iters, chain.data_ptr() if chain is not None else None, n,
                               out.data_ptr(), st)
    if r != 0:
        raise fire.FireError(r, "fire_probe_latency failed")
    ticks = int(out[0].item())
    return ticks * 10.0 / iters  # the wall clock runs at 100 MHz: 10 ns per tick


def measure(num_cu: int | None = None) -> dict:
    """All ceilings, in a dict of plain numbers."""
    props = torch.cuda.get_device_properties(0)
    cu = num_cu or props.multi_processor_count
    return {
        "l2_read_gbs": read_bandwidth(1 << 20, 64, True, 4 * cu),
        "mall_read_gbs": read_bandwidth(128 << 20, 8, False, 8 * cu),
        "hbm_read_gbs": read_bandwidth(4 << 30, 1, False, 8 * cu, reps=3),
        "philox_calls_per_s": philox_rate(8 * cu),
        "barrier_ns": latency_ns(0),
        "l2_load_ns": latency_ns(1),
        "lds_atomic_ns": latency_ns(2),
        "philox_ns": latency_ns(3, iters=1024),
        "compute_units": cu,
    }
