"""Schedule autotuner for the simulation kernel.

For a representative batch on one landscape size class it times every
candidate schedule (threads per workgroup, workgroups per compute unit,
LDS queue capacity, threshold table vs per-trial evaluation) with HIP
events on the launch stream, checks that every schedule returns bit-identical
results (they must: results do not depend on the schedule), and keeps the
fastest. Choices are cached per GPU architecture, size class and kind of
batch (replicate, GA population, scattered) in a JSON file committed beside
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
    rows.append((ms, dict(builtin, builtin=True)))
    if log:
        log(f"{ms:8.3f} ms  built-in {builtin}")
    table_ok = len(betas) <= 8 or n >= 8 * len(betas)
    for sched in candidates(table_ok=table_ok, side=side):
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


def apply_cache(g: fire.FireGPU, path: str = CACHE) -> int:
    """Install the cached schedules of this architecture (per size class and
    batch kind: replicate, population, scattered); returns how many."""
    entries = load_cache(path).get(arch_name(), {})
    n = 0
    for bucket, kinds in entries.items():
        for kind, e in kinds.items():
            if kind not in fire.FireGPU.BATCH_KINDS:
                continue
            g.set_class_schedule(1 << int(bucket), e["schedule"], kind=kind)
            n += 1
    return n


def workloads():
    """The batches the library runs, per size class and kind: replicate
    batches at the calibration vector (the scan workload's 256 candidate
    ignitions x 32 replicates at 1024x1024), GA populations (64 vectors from
    Table 1's Gaussian prior x 20 replicates) and scattered batches (one
    simulation per vector drawn uniformly from the search box, as Monte
    Carlo fits and the uneven batch have). Yields (kind, landscape, label,
    parameter rows, descriptors-builder)."""
    from . import scan
    rng = np.random.default_rng(7)
    beta_star = np.array([[-3.0, -0.5, 6.0, 1.0, 2.0]])
    for W, H, seed in ((128, 128, 101), (256, 256, 102), (512, 512, 102)):
        ls = synth.make_landscape(W, H, seed)
        c = synth.ignition_site(ls)
        yield ("replicate", ls, f"{W}x{H}", beta_star,
               lambda lid, c=c: fire.make_sims(1280, lid, -1, c))
        pop = np.clip(rng.normal(0.0, 5.0, size=(64, 5)), -30, 30)
        yield ("population", ls, f"{W}x{H}", pop,
               lambda lid, c=c: fire.make_sims(1280, lid, -1, c,
                                               param_index=np.repeat(np.arange(64), 20)))
        box = rng.uniform(-30.0, 30.0, size=(2000, 5))
        yield ("scattered", ls, f"{W}x{H}", box,
               lambda lid, c=c: fire.make_sims(2000, lid, -1, c, param_index=np.arange(2000)))
    ls = synth.make_landscape(1024, 768, 104)
    c = synth.ignition_site(ls)
    box = rng.uniform(-30.0, 30.0, size=(500, 5))
    yield ("scattered", ls, "1024x768", box,
           lambda lid, c=c: fire.make_sims(500, lid, -1, c, param_index=np.arange(500)))
    ls = synth.scan_landscape()
    c = synth.scan_ignition(ls)
    cands = scan.candidate_grid(c, *synth.SCAN_SIZE, spacing=4, half=8)
    yield ("replicate", ls, "1024x1024 scan", np.array([synth.SCAN_BETA]),
           lambda lid, cands=cands: scan.scan_sims(lid, -1, cands, 32))


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=CACHE, help="cache file to update")
    ap.add_argument("--only", default=None, help="tune only workloads whose label starts so")
    args = ap.parse_args()
    log = lambda m: print(f"[autotune] {m}", flush=True)  # noqa: E731
    g = fire.FireGPU(0)
    cache = load_cache(args.out)
    arch = arch_name()
    mine = cache.setdefault(arch, {})
    for kind, ls, label, betas, make in workloads():
        if args.only and not label.startswith(args.only):
            continue
        H, W = np.asarray(ls["veg"]).shape
        lid = g.load_landscape(ls)
        sims = make(lid)
        log(f"{label}, {kind}: {len(betas)} parameter vector(s), {len(sims)} simulations")
        best, rows = tune(g, lid, sims, betas, 0x5EED0001, log=log)
        b = str(cells_bucket(W * H))
        builtin_ms = next(ms for ms, s in rows if s.get("builtin"))
        if best.get("builtin"):
            # the built-in plan won: no class entry (it adapts to the batch)
            mine.setdefault(b, {}).pop(kind, None)
            log(f"{label}, {kind}: built-in plan kept ({builtin_ms:.3f} ms)")
            g.free_landscape(lid)
            continue
        mine.setdefault(b, {})[kind] = {"schedule": best, "ms": rows[0][0], "lattice": [W, H],
                                        "workload": label, "sims": len(sims),
                                        "builtin_ms": builtin_ms,
                                        "runner_up": rows[1][1] if len(rows) > 1 else None,
                                        "runner_up_ms": rows[1][0] if len(rows) > 1 else None}
        g.free_landscape(lid)
        with open(args.out, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    log(f"wrote {args.out}")
    g.close()


if __name__ == "__main__":
    sys.exit(main())
