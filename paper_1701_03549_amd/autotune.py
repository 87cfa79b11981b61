"""Schedule autotuner for the simulation kernel.

For a representative batch on one landscape size class it times every
candidate schedule (threads per workgroup, workgroups per compute unit,
LDS queue capacity, threshold table vs per-trial evaluation) with HIP
events on the launch stream, checks that every schedule returns bit-identical
results (they must: results do not depend on the schedule), and keeps the
fastest. Choices are cached per GPU architecture, size class and kind of
batch (at most 8 parameter vectors, or more) in a JSON file committed beside
this module, and applied through fire_set_class_schedule.

    python -m paper_1701_03549_amd.autotune            # tune the built-in workloads
"""
from __future__ import annotations

import itertools
import json
import os
import sys

import numpy as np
import torch

from . import fire, synth

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_schedules.json")


def arch_name() -> str:
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def cells_bucket(cells: int) -> int:
    b = 0
    while (1 << b) < cells:
        b += 1
    return b


def candidates(table_ok: bool, side: int = 0):
    """Schedules to time. One simulation per workgroup: workgroup size x
    workgroups per CU x LDS queue capacity x threshold mode x LDS window
    (none, or a quarter, half and three quarters of the lattice side, when
    that is at least 64 cells). The wavefront-per-simulation kernel is
    left out: on the calibration batch it was a third slower than the
    workgroup kernel, and it stays off the built-in paths."""
    windows = [0] + sorted({w for w in (side // 4, side // 2, 3 * side // 4)
                            if w >= 64 and w % 32 == 0 and w < side})
    tables = (0, 1) if table_ok else (0,)
    for threads, wg, qcap, win in itertools.product((128, 256, 512, 1024), (1, 2, 4, 5, 8),
                                                    (1024, 4096), windows):
        if threads > 512 and win > 0:
            continue  # the library runs 1024-thread schedules without a window
        for table in tables:
            yield {"threads": threads, "queue_cap": qcap, "table_mode": table, "wg_per_cu": wg,
                   "window": win, "wave": 0}


def time_schedule(g: fire.FireGPU, sched, d_beta, d_sims, n, seed, out, reps=3):
    """Median milliseconds of `reps` launches (HIP events on the launch
    stream) under `sched`, or under the built-in plan when it is None."""
    if sched is None:
        g.set_schedule(reset=True)
    else:
        g.set_schedule(**sched)
    stream = torch.cuda.current_stream()
    g.run_dev(d_beta, d_sims, n, seed, out, stream=stream)  # warm-up (allocations)
    g.sync()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        g.run_dev(d_beta, d_sims, n, seed, out, stream=stream)
        b.record(stream)
    g.sync()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def tune(g: fire.FireGPU, lid: int, sims: np.ndarray, betas: np.ndarray, seed: int,
         log=None):
    """Tune one size class (all sims on landscape `lid`). Returns (best, table)."""
    n = len(sims)
    d_sims = torch.from_numpy(np.ascontiguousarray(sims).view(np.uint8).copy()).to(g.device)
    d_beta = torch.from_numpy(np.ascontiguousarray(betas, dtype=np.float64)).to(g.device)
    out = torch.empty((n, 24), dtype=torch.uint8, device=g.device)
    ref = None
    rows = []
    side = max(g.dims[lid])
    W, H = g.dims[lid]
    # the built-in plan first (its window size is not among the grid's)
    g.set_schedule(reset=True)
    builtin = g.get_schedule(W * H, len(betas), n)
    ms = time_schedule(g, None, d_beta, d_sims, n, seed, out)
    ref = out.clone()
    rows.append((ms, dict(builtin)))
    if log:
        log(f"{ms:8.3f} ms  built-in {builtin}")
    for sched in candidates(table_ok=len(betas) <= 8, side=side):
        if log:
            log(f"timing {sched}")
        try:
            ms = time_schedule(g, sched, d_beta, d_sims, n, seed, out)
        except fire.FireError as e:  # LDS budget exceeded for this shape
            if log:
                log(f"skip {sched}: {e}")
            continue
        if ref is None:
            ref = out.clone()
        elif not torch.equal(out, ref):
            raise RuntimeError(f"schedule {sched} changed the results")
        rows.append((ms, sched))
        if log:
            log(f"{ms:8.3f} ms  {sched}")
    g.set_schedule(reset=True)
    rows.sort(key=lambda r: r[0])
    return rows[0][1], rows


def load_cache(path: str = CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


KINDS = {"replicate": False, "many": True}


def apply_cache(g: fire.FireGPU, path: str = CACHE) -> int:
    """Install the cached schedules of this architecture (per size class and
    batch kind: at most 8 parameter vectors, or more); returns how many."""
    entries = load_cache(path).get(arch_name(), {})
    n = 0
    for bucket, kinds in entries.items():
        for kind, e in kinds.items():
            g.set_class_schedule(1 << int(bucket), e["schedule"], many_params=KINDS[kind])
            n += 1
    return n


def workloads():
    """Representative batches per size class: replicate batches at a
    contained parameter vector and random parameter vectors from the
    search box, on the synthetic landscapes of the benchmark configs."""
    rng = np.random.default_rng(7)
    beta_star = np.array([[-3.0, -0.5, 6.0, 1.0, 2.0]])
    for W, H, seed in ((128, 128, 101), (256, 256, 102), (512, 512, 102), (1024, 768, 104),
                       (1024, 1024, 103)):
        yield (W, H, seed, beta_star, 1280)
        yield (W, H, seed, rng.uniform(-30, 30, size=(500, 5)), 500)


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=CACHE, help="cache file to update")
    ap.add_argument("--only", default=None, help="tune only this lattice, e.g. 512x512")
    args = ap.parse_args()
    log = lambda m: print(f"[autotune] {m}", flush=True)  # noqa: E731
    g = fire.FireGPU(0)
    cache = load_cache(args.out)
    arch = arch_name()
    mine = cache.setdefault(arch, {})
    for W, H, seed, betas, n in workloads():
        if args.only and args.only != f"{W}x{H}":
            continue
        ls = synth.make_landscape(W, H, seed)
        lid = g.load_landscape(ls)
        c = synth.ignition_site(ls)
        sims = fire.make_sims(n, lid, -1, c, param_index=np.arange(n) % len(betas))
        kind = "many" if len(betas) > 8 else "replicate"
        log(f"{W}x{H}, {len(betas)} parameter vector(s), {n} simulations ({kind})")
        best, rows = tune(g, lid, sims, betas, 0x5EED0001, log=log)
        b = str(cells_bucket(W * H))
        mine.setdefault(b, {})[kind] = {"schedule": best, "ms": rows[0][0],
                                        "lattice": [W, H], "sims": n,
                                        "runner_up": rows[1][1] if len(rows) > 1 else None,
                                        "runner_up_ms": rows[1][0] if len(rows) > 1 else None}
        g.free_landscape(lid)
        with open(args.out, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    log(f"wrote {args.out}")
    g.close()


if __name__ == "__main__":
    sys.exit(main())
