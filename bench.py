"""Benchmark: fire simulations/s and neighbour-trials/s at 512x512 on one GPU.

One step = one pass of the simulation hot path over the calibration batch:
the Eq. 1 threshold table of the calibration vector, then 1280 seeded
replicate simulations (ignition at the centre, run to extinction) on a
512x512 synthetic landscape with the Eq. 2 fitness against a reference map
fused in. Inputs (landscape, reference map, descriptors, parameters) are
resident on the device before timing starts.

Also reported: the simulation kernel's achieved algorithmic bandwidth against
the HBM peak, the CPU oracle timed on the host cores on the same batch, and
(unless --no-ga) the wall time of a whole GA calibration (64 individuals x 20
replicates x 50 generations) as a captured-graph batched run versus plain
one-simulation-per-launch evaluation with a host synchronisation after each.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fire simulations/sec + neighbour-trials/sec at 512², GA wall-time batched vs plain"
HBM_PEAK_GBS = 8000.0
BETA_STAR = (-3.0, -0.5, 6.0, 1.0, 2.0)
SIM_SEED = 0x5EED0001
TARGET_SEED = 0x7A26E7
GA_SEED = 0x6A00001
W = H = 512
LANDSCAPE_SEED = 102
N_SIMS = 1280
PROFILE_PMC = os.path.join(ROOT, "profiles", "sim_kernel_512x512_1280_pmc.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1701_03549_amd", "csrc", "fire_kernels.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_sha() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def apply_tuned(g) -> int:
    """Install the autotuner's cached schedules for this GPU architecture
    (per size class and batch kind); returns how many."""
    from paper_1701_03549_amd import autotune
    return autotune.apply_cache(g)


def reference_fire(g, ls, lid, centre):
    """Reference map: the first replicate under the reference seed whose burnt
    fraction lies in [1%, 15%] and that does not touch the lattice border,
    simulated by the library at the calibration vector."""
    from paper_1701_03549_amd import fire
    n = 256
    sims = fire.make_sims(n, lid, -1, centre)
    res, maps = g.run(np.array([BETA_STAR]), sims, TARGET_SEED, want_maps=True)
    g.sync()
    r = fire.results_to_numpy(res)
    m = maps.cpu().numpy().view(np.uint32).reshape(n, H, -1)
    for k in range(n):
        frac = r["burnt"][k] / (W * H)
        mk = m[k]
        border = mk[0].any() or mk[-1].any() or (mk[:, 0] & 1).any() or ((mk[:, -1] >> 31) & 1).any()
        if 0.01 <= frac <= 0.15 and not border:
            return mk.copy(), k
    raise RuntimeError("no contained reference fire among the first 256 replicates")


def _oracle_pass(ls, beta, centre, n, ref, threads):
    """One pass of the oracle over a replicate batch: thresholds, n
    simulations, Eq. 2 (when ref is given). Returns (sims, trials)."""
    import oracle
    sims = [dict(param=0, ign=centre, sim_index=i) for i in range(n)]
    T = oracle.thresholds(ls, beta)
    out = oracle.run_batch(ls["veg"], [T], sims, SIM_SEED, ref_bits=ref, threads=threads)
    return len(out), sum(o["trials"] for o in out)


def _time_oracle(ls, beta, centre, n, ref, threads, budget_s):
    t0 = time.perf_counter()
    done = trials = passes = 0
    while True:
        d, t = _oracle_pass(ls, beta, centre, n, ref, threads)
        done += d
        trials += t
        passes += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return done / dt, trials / dt, passes, dt


def cpu_baseline(ls, centre, ref, budget_s=8.0):
    """The oracle (plain C, binary64), on the host's cores and on one core,
    on the calibration batch (1280 replicates at 512x512) and on the plain
    64x64 workload (200 replicates at beta = 0)."""
    from paper_1701_03549_amd import synth
    nproc = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = nproc
    # the process's CPU share: a GPU run gets at most 16 host threads
    threads = max(1, min(16, avail))
    v, tr, passes, dt = _time_oracle(ls, BETA_STAR, centre, N_SIMS, ref, threads, budget_s)
    v1, tr1, passes1, dt1 = _time_oracle(ls, BETA_STAR, centre, N_SIMS, ref, 1, budget_s / 2)
    ls64 = synth.make_landscape(64, 64, 101)
    c64 = synth.nearest_burnable(ls64["veg"], 32, 32)
    beta0 = (0.0, 0.0, 0.0, 0.0, 0.0)
    w, wtr, wp, wdt = _time_oracle(ls64, beta0, c64, 200, None, threads, budget_s / 4)
    w1, w1tr, w1p, w1dt = _time_oracle(ls64, beta0, c64, 200, None, 1, budget_s / 4)
    return {"value": v, "unit": "sims/s", "cores": threads, "kind": "oracle",
            "trials_per_s": tr, "host_nproc": nproc, "host_cpus_available": avail,
            "sample": f"{passes} pass(es) over the full calibration batch ({N_SIMS} replicates at "
                      f"512x512, thresholds + simulation + Eq. 2) on {threads} threads, {dt:.1f} s",
            "one_core": {"value": v1, "trials_per_s": tr1,
                         "sample": f"{passes1} pass(es) of the same batch on 1 thread, {dt1:.1f} s"},
            "plain_64": {"workload": "64x64, seed 101, beta = 0, 200 replicates to extinction",
                         "value": w, "trials_per_s": wtr, "cores": threads,
                         "one_core_value": w1, "one_core_trials_per_s": w1tr,
                         "sample": f"{wp} and {w1p} passes, {wdt:.1f} s and {w1dt:.1f} s"}}


def pmc_profile():
    """The committed counter summary of the simulation kernel, or None once
    the kernel source differs from the one the counters were taken on."""
    if not os.path.exists(PROFILE_PMC):
        return None
    with open(PROFILE_PMC) as f:
        p = json.load(f)
    if p.get("kernel_source_sha") != kernel_sha():
        return None
    return p


def run_ga(g, lid, tid, centre, plain: bool):
    """Batched (graph-captured) GA and, optionally, the plain per-simulation
    GA; returns wall times and a bit-identity check of the two histories."""
    import torch
    from paper_1701_03549_amd import ga
    rng = np.random.default_rng(2024)
    pop0 = np.clip(rng.normal(0.0, 5.0, size=(64, 5)), -30.0, 30.0)  # Table 1 Gaussian prior
    out = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hb = ga.run_batched(g, lid, tid, centre, pop0, R=20, generations=50, sim_seed=SIM_SEED,
                        ga_seed=GA_SEED)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    out["batched_s"] = tb
    out["batched_sims_per_s"] = 64 * 20 * 50 / tb
    log(f"batched GA: {tb:.2f} s")
    est = ga.recovered(g, hb, cutoff=0.3)
    out["recovered"] = est
    if plain:
        t0 = time.perf_counter()
        hp = ga.run_plain(g, lid, tid, centre, pop0, R=20, generations=50, sim_seed=SIM_SEED,
                          ga_seed=GA_SEED,
                          progress=lambda k: log(f"plain GA generation {k} done") if k % 5 == 0
                          else None)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        out["plain_s"] = tp
        out["plain_sims_per_s"] = 64 * 20 * 50 / tp
        out["speedup"] = tp / tb
        out["identical_trajectory"] = bool(torch.equal(hb[0], hp[0]) and torch.equal(hb[1], hp[1]))
    return out


def run_mc(g, lid, tid, centre, ga_sims_per_s):
    """Brute-force Monte Carlo fit (Appendix C): as many simulations as the
    GA's (64 x 20 x 50), parameters uniform over the search box, one
    persistent launch; throughput against the GA's and the spread of work
    per simulation (trials) that drives it."""
    import torch
    from paper_1701_03549_amd import mc
    n = 64 * 20 * 50
    mc.run_mc(g, lid, tid, centre, 4096, seed=7, sim_seed=SIM_SEED)  # warm-up
    torch.cuda.synchronize()
    out = mc.run_mc(g, lid, tid, centre, n, seed=2025, sim_seed=SIM_SEED, cutoff=0.3, chunk=n)
    tr = out["trials"].double()
    res = {"sims": n, "wall_s": out["wall_s"], "sims_per_s": n / out["wall_s"],
           "trials_per_s": float(tr.sum().item()) / out["wall_s"],
           "trials_per_sim_mean": float(tr.mean().item()),
           "trials_per_sim_cv": float((tr.std() / tr.mean()).item()),
           "ga_over_mc_sims_per_s": (ga_sims_per_s / (n / out["wall_s"])) if ga_sims_per_s else None,
           "best_fitness": out["best_fitness"], "n_accepted": out["n_accepted"],
           "accepted_mean": out["accepted_mean"]}
    log(f"MC: {n} sims in {out['wall_s']:.3f} s, best fitness {out['best_fitness']:.3f}")
    return res


def run_ignition_ga(g, lid, tid, centre, ref_bits):
    """The 7-parameter GA (ignition estimated): 64 individuals x 20
    replicates x 50 generations, betas from Table 1's Gaussian prior,
    ignitions uniform over the reference burnt cells; accepted ensemble at
    the variable-ignition cutoff 1.5."""
    import torch
    from paper_1701_03549_amd import ga
    W, H = g.dims[lid]
    pop0 = ga.initial_population_ignition(ref_bits, W, H, 64, seed=2024)
    ga.run_ignition(g, lid, tid, pop0, R=20, generations=2, sim_seed=SIM_SEED, ga_seed=GA_SEED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = ga.run_ignition(g, lid, tid, pop0, R=20, generations=50, sim_seed=SIM_SEED,
                           ga_seed=GA_SEED)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rec = ga.recovered(g, hist, cutoff=1.5)
    m = rec["accepted_mean"]
    err = float(np.hypot(m[5] - centre[0], m[6] - centre[1]))
    bp = rec["best_params"]
    log(f"7-gene GA: {dt:.2f} s, ignition error {err:.1f} cells")
    return {"wall_s": dt, "sims_per_s": 64 * 20 * 50 / dt, "recovered": rec,
            "true_ignition": list(map(int, centre)),
            "accepted_ignition_error_cells": err,
            "best_ignition_error_cells": float(np.hypot(bp[5] - centre[0], bp[6] - centre[1]))}


def run_dense(g, lid, tid, centre, frontier_sims_per_s):
    """The per-cell ablation path (fire_run_dense: one launch per step over
    the whole lattice, host-polled, one simulation after another, as the
    paper runs them) on 32 replicates of the calibration batch."""
    import torch
    from paper_1701_03549_amd import fire
    n = 32
    sims = fire.make_sims(n, lid, tid, centre)
    g.run_dense(np.array([BETA_STAR]), sims[:2], SIM_SEED)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, _ = g.run_dense(np.array([BETA_STAR]), sims, SIM_SEED)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = fire.results_to_numpy(res)
    steps = int(r["steps"].sum())
    log(f"per-cell path: {n} sims in {dt:.3f} s ({dt / steps * 1e6:.1f} us per step)")
    return {"sims": n, "wall_s": dt, "sims_per_s": n / dt, "steps": steps,
            "us_per_step": dt / steps * 1e6, "mean_burnt": float(r["burnt"].mean()),
            "frontier_over_dense": frontier_sims_per_s / (n / dt),
            "state_bytes_per_step": 2 * W * H}


def run_turn_off(g, lid, tid, centre, d_sims, reps=10):
    """The calibration batch (1280 replicates at 512x512) with turn-off times
    of 2 steps for forest and 3 for the other vegetation (the turn-off-time
    kernel), against the same batch with one-step burns."""
    import torch
    from paper_1701_03549_amd import fire
    d_beta = torch.tensor([BETA_STAR], dtype=torch.float64, device="cuda")
    out = torch.empty((N_SIMS, 24), dtype=torch.uint8, device="cuda")
    bs = np.full(256, 3, dtype=np.uint8)
    bs[1] = 2
    g.set_burn_steps(lid, bs)
    try:
        g.run_dev(d_beta, d_sims, N_SIMS, SIM_SEED, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g.run_dev(d_beta, d_sims, N_SIMS, SIM_SEED, out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
    finally:
        g.set_burn_steps(lid, None)
    r = fire.results_to_numpy(out)
    trials = int(r["trials"].sum())
    log(f"turn-off times: {dt * 1e3:.2f} ms per batch, mean burnt {r['burnt'].mean():.0f}")
    return {"burn_steps": {"forest": 2, "other": 3}, "ms_per_batch": dt * 1e3,
            "sims_per_s": N_SIMS / dt, "trials_per_s": trials / dt,
            "mean_burnt": float(r["burnt"].mean()), "mean_steps": float(r["steps"].mean()),
            "mean_fitness": float(np.nanmean(r["fitness"]))}


def run_scan(log_fn):
    """Ignition-point scan on the 1024x1024 scan landscape (seed 103, smooth
    wind) at the scan parameter vector: 256 candidate cells on a 4-cell grid
    around the true ignition x 32 replicates, Eq. 2 against a contained
    reference fire (2-20% of the lattice, off the border), device reduction."""
    import torch
    from paper_1701_03549_amd import fire, scan, synth
    g = fire.FireGPU(0)
    apply_tuned(g)
    ls = synth.scan_landscape()
    W, H = synth.SCAN_SIZE
    beta = synth.SCAN_BETA
    c = synth.scan_ignition(ls)
    lid = g.load_landscape(ls)
    res, maps = g.run(np.array([beta]), fire.make_sims(64, lid, -1, c), TARGET_SEED,
                      want_maps=True)
    g.sync()
    r = fire.results_to_numpy(res)
    m = maps.cpu().numpy().view(np.uint32).reshape(64, H, -1)
    k = next(i for i in range(64)
             if 0.02 <= r["burnt"][i] / (W * H) <= 0.20 and not (
                 m[i, 0].any() or m[i, -1].any() or (m[i, :, 0] & 1).any()
                 or ((m[i, :, -1] >> ((W - 1) % 32)) & 1).any()))
    tid = g.load_target(lid, m[k])
    cands = scan.candidate_grid(c, W, H, spacing=4, half=8)
    scan.run_scan(g, lid, tid, beta, cands, R=32, seed=SIM_SEED, cutoff=0.3)  # warm-up
    g.sync()
    times = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = scan.run_scan(g, lid, tid, beta, cands, R=32, seed=SIM_SEED, cutoff=0.3)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    mean = out["mean"].cpu().numpy()
    true_k = int(np.argmin(np.abs(cands - np.array(c)).sum(axis=1)))
    rank = int((mean < mean[true_k]).sum())
    dt = float(np.median(times))
    # surrogate screening of the candidates: a network trained on runs with
    # ignitions uniform over the candidate box keeps 64 of the 256, which
    # are then scanned exactly (with the coins of the full scan)
    from paper_1701_03549_amd import nn, surrogate
    x0, y0 = int(cands[:, 0].min()), int(cands[:, 1].min())
    box = (x0, y0, int(cands[:, 0].max()) - x0 + 1, int(cands[:, 1].max()) - y0 + 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, y = surrogate.make_ignition_dataset(g, lid, tid, beta, box, 4096, seed=3, sim_seed=0xDA7A)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net = nn.Surrogate(max_batch=512, lattice=box[2:], w_map=0.0, seed=1)
    t0 = time.perf_counter()
    surrogate.train(net, X, y, None, epochs=8, batch=512, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    t0 = time.perf_counter()
    kept, so = surrogate.screened_scan(g, net, lid, tid, beta, cands, box, 64, R=32,
                                       seed=SIM_SEED, cutoff=0.3)
    torch.cuda.synchronize()
    t_screen = time.perf_counter() - t0
    top = set(np.argsort(mean, kind="stable")[:64].tolist())
    screening = {"training_runs": 4096, "data_s": t_data, "train_s": t_train,
                 "kept": 64, "screened_scan_ms": t_screen * 1e3,
                 "best_kept": bool(int(np.argmin(mean)) in set(kept.tolist())),
                 "top64_overlap": len(top & set(kept.tolist())),
                 "rows_equal_full_scan": bool(torch.equal(so["deltas"], out["deltas"][kept]))}
    net.close()
    g.close()
    log_fn(f"scan: {len(cands)} x 32 simulations in {dt * 1e3:.2f} ms; true ignition ranks {rank}; "
           f"screening {screening}")
    return {"lattice": [W, H], "beta": list(beta), "candidates": len(cands), "replicates": 32,
            "wall_ms": dt * 1e3, "sims_per_s": len(cands) * 32 / dt,
            "true_candidate_rank": rank, "reference_cells": int(r["burnt"][k]),
            "reference_replicate": k, "screening": screening}


def run_uneven(log_fn):
    """2000 simulations over four landscapes of different sizes with
    parameter vectors drawn uniformly from the search box, as one fire_run
    (grouped by landscape into concurrent persistent launches) and as one
    persistent launch sized for the largest lattice (fire_run_dev)."""
    import torch
    from paper_1701_03549_amd import fire, synth
    g = fire.FireGPU(0)
    apply_tuned(g)
    sizes = [(128, 128, 101), (256, 256, 102), (512, 512, 103), (1024, 768, 104)]
    lids, sims = [], []
    rng = np.random.default_rng(404)
    betas = rng.uniform(-30.0, 30.0, size=(2000, 5))
    for k, (W, H, sd) in enumerate(sizes):
        ls = synth.make_landscape(W, H, sd)
        lid = g.load_landscape(ls)
        lids.append(lid)
        sims.append(fire.make_sims(500, lid, -1, synth.ignition_site(ls),
                                   param_index=np.arange(500 * k, 500 * (k + 1)),
                                   sim_index=np.arange(500 * k, 500 * (k + 1), dtype=np.uint32)))
    sims = np.concatenate(sims)
    res, _ = g.run(betas, sims, SIM_SEED)  # warm-up
    g.sync()
    d_sims = torch.from_numpy(sims.view(np.uint8).copy()).cuda()
    d_beta = torch.from_numpy(betas).cuda()
    out = torch.empty((2000, 24), dtype=torch.uint8, device="cuda")
    g.run_dev(d_beta, d_sims, 2000, SIM_SEED, out)
    g.sync()
    tg, ts = [], []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, _ = g.run(betas, sims, SIM_SEED)
        torch.cuda.synchronize()
        tg.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        g.run_dev(d_beta, d_sims, 2000, SIM_SEED, out)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    same = bool(torch.equal(res, out))
    # the single launch captured as a graph, as a GA generation launches it
    out_g = torch.empty_like(out)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g.run_dev(d_beta, d_sims, 2000, SIM_SEED, out_g, stream=torch.cuda.current_stream())
    tr = []
    for _ in range(3):
        out_g.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        graph.replay()
        torch.cuda.synchronize()
        tr.append(time.perf_counter() - t0)
    same_graph = bool(torch.equal(out_g, out))
    del graph
    # the same capture over descriptors uploaded longest-expected-first
    # (fire_order_sims, the order fire_run starts such a batch in)
    order = g.order_sims(betas, sims)
    d_sims_o = torch.from_numpy(sims[order].view(np.uint8).copy()).cuda()
    out_o = torch.empty_like(out)
    g.run_dev(d_beta, d_sims_o, 2000, SIM_SEED, out_o)
    g.sync()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g.run_dev(d_beta, d_sims_o, 2000, SIM_SEED, out_o, stream=torch.cuda.current_stream())
    tro = []
    for _ in range(3):
        out_o.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        graph.replay()
        torch.cuda.synchronize()
        tro.append(time.perf_counter() - t0)
    idx = torch.from_numpy(order.astype(np.int64)).cuda()
    same_ordered = bool(torch.equal(out_o, out[idx]))
    del graph
    # load balance of each form, from the per-simulation device clocks
    from paper_1701_03549_amd.timing import load_balance
    clocks = torch.zeros((2000, 2), dtype=torch.int64, device="cuda")
    g.set_sim_timing(clocks)
    g.run_dev(d_beta, d_sims, 2000, SIM_SEED, out)
    g.sync()
    lb_single = load_balance(clocks.cpu().numpy())
    clocks.zero_()
    g.run(betas, sims, SIM_SEED)
    g.sync()
    lb_grouped = load_balance(clocks.cpu().numpy())
    g.set_sim_timing(None)
    r = fire.results_to_numpy(res)
    trials = int(r["trials"].sum())
    g.close()
    dt_g, dt_s, dt_r = float(np.median(tg)), float(np.median(ts)), float(np.median(tr))
    dt_ro = float(np.median(tro))
    log_fn(f"uneven: grouped {dt_g * 1e3:.1f} ms, single launch {dt_s * 1e3:.1f} ms, graph replay "
           f"{dt_r * 1e3:.1f} ms, ordered graph replay {dt_ro * 1e3:.1f} ms; load balance single "
           f"{lb_single}, grouped {lb_grouped}")
    return {"sims": 2000, "lattices": [[w, h] for w, h, _ in sizes],
            "grouped_ms": dt_g * 1e3, "single_launch_ms": dt_s * 1e3, "graph_replay_ms": dt_r * 1e3,
            "ordered_graph_replay_ms": dt_ro * 1e3, "ordered_graph_identical": same_ordered,
            "grouped_sims_per_s": 2000 / dt_g, "grouped_trials_per_s": trials / dt_g,
            "identical_results": same, "graph_identical": same_graph,
            "load_balance_single": lb_single, "load_balance_grouped": lb_grouped,
            "mean_burnt": float(r["burnt"].mean())}


def run_surrogate(log_fn):
    """Learned surrogate on the 256x256 landscape (seed 105): simulator-made
    training data, MFMA training, and the GA with and without screening."""
    import torch
    from paper_1701_03549_amd import fire, nn, surrogate, synth
    g = fire.FireGPU(0)
    W = H = 256
    ls = synth.make_landscape(W, H, 105)
    c = synth.ignition_site(ls)
    lid = g.load_landscape(ls)
    res, maps = g.run(np.array([BETA_STAR]), fire.make_sims(64, lid, -1, c), TARGET_SEED,
                      want_maps=True)
    g.sync()
    r = fire.results_to_numpy(res)
    k = int(np.argmax(r["burnt"] >= 0.001 * W * H))
    tid = g.load_target(lid, maps.cpu().numpy().view(np.uint32)[k].reshape(H, -1))
    n_data, epochs, batch = 100000, 4, 512
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, y_t, y_map = surrogate.make_dataset(g, lid, tid, n_data, seed=5, sim_seed=0xDA7A,
                                           prior_sd=5.0, ign=c)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net = nn.Surrogate(max_batch=batch, lattice=(W, H), w_map=1.0, seed=1)
    n_train = n_data - n_data // 10
    t0 = time.perf_counter()
    surrogate.train(net, X[n_data // 10:], y_t[n_data // 10:], y_map[n_data // 10:],
                    epochs=epochs, batch=batch)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    steps = epochs * (n_train // batch)
    # MFMA work per sample: forward GEMMs (16x256, 2 x 256x256, 256x1, 256x2048) and
    # twice that in the backward pass
    gemm_flop = 3 * 2 * (16 * 256 + 2 * 256 * 256 + 256 + 256 * 2048)
    pv = net.predict(X[:n_data // 10]).cpu().numpy()
    rho = surrogate.spearman(pv, y_t[:n_data // 10].cpu().numpy())
    trained = net.get_params()
    log_fn(f"surrogate: data {t_data:.2f} s, training {t_train:.2f} s, held-out Spearman {rho:.3f}")
    from paper_1701_03549_amd import ga
    rows = []
    for s_ in range(5):
        pop0 = np.clip(np.random.default_rng(100 + s_).normal(0, 5, size=(64, 5)), -30, 30)
        kw = dict(R=20, sim_seed=SIM_SEED + s_, ga_seed=GA_SEED + s_)
        # plain: the library's graph-captured GA, 30 generations
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, fp = ga.run_batched(g, lid, tid, c, pop0, generations=30, **kw)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        plain = surrogate.best_mean_fitness(fp)
        # screened: the whole 30-generation run captured as one graph, a
        # fresh optimiser on the trained parameters
        ns = net.clone()
        _, fs, tm = surrogate.run_ga(g, lid, tid, c, pop0, generations=30, net=ns, seed=s_,
                                     graph=True, **kw)
        ns.close()
        screened = surrogate.best_mean_fitness(fs)
        # the plain GA at equal accuracy: the shortest run (30 ... 480
        # generations) whose best mean fitness reaches the screened run's
        match = None
        for G in (30, 60, 120, 240, 480):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, fg = ga.run_batched(g, lid, tid, c, pop0, generations=G, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if surrogate.best_mean_fitness(fg) <= screened:
                match = {"generations": G, "wall_s": dt, "sims": 64 * 20 * G}
                break
        rows.append({"plain_best_mean_fitness": plain, "plain_wall_s": t_plain,
                     "screened_best_mean_fitness": screened,
                     "screened_wall_s": tm["capture_s"] + tm["replay_s"],
                     "screened_replay_s": tm["replay_s"], "plain_to_equal_accuracy": match})
        log_fn(f"surrogate GA seed {s_}: {rows[-1]}")
    net.close()
    g.close()
    return {"lattice": [W, H], "training_runs": n_data, "data_s": t_data,
            "train_s": t_train, "train_samples_per_s": steps * batch / t_train,
            "gemm_tflops": steps * batch * gemm_flop / t_train / 1e12,
            "gemm_peak_tflops": 2500.0, "heldout_spearman": rho,
            "ga_seeds": 5, "ga_sims_per_run": 64 * 20 * 30, "runs": rows,
            "plain_best_mean_fitness": [r["plain_best_mean_fitness"] for r in rows],
            "screened_best_mean_fitness": [r["screened_best_mean_fitness"] for r in rows],
            "plain_wall_s": float(np.mean([r["plain_wall_s"] for r in rows])),
            "screened_wall_s": float(np.mean([r["screened_wall_s"] for r in rows])),
            "note": "screened wall time excludes the one-off training data ("
                    f"{t_data:.2f} s) and training ({t_train:.2f} s) on this landscape"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-ga", action="store_true", help="skip the GA wall-time comparison")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain GA run")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate section")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the ignition-scan and uneven-batch sections")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain elementwise copy of 256 MiB (read) + 256 MiB (write) "
                         "three times, to scale the profiler's HBM byte counters")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the benchmark measures one GPU only; simulations are independent, so N "
              "GPUs would each run their own share of the batch (see the sharding design). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1701_03549_amd import fire, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    g = fire.FireGPU(0)
    n_tuned = apply_tuned(g)
    ls = synth.make_landscape(W, H, LANDSCAPE_SEED)
    centre = synth.ignition_site(ls)
    lid = g.load_landscape(ls)
    ref, ref_k = reference_fire(g, ls, lid, centre)
    tid = g.load_target(lid, ref)
    log(f"reference fire: replicate {ref_k}, {int(np.unpackbits(ref.view(np.uint8)).sum())} cells")

    sims = fire.make_sims(N_SIMS, lid, tid, centre)
    d_sims = torch.from_numpy(sims.view(np.uint8).copy()).cuda()
    d_beta = torch.tensor([BETA_STAR], dtype=torch.float64, device="cuda")
    out = torch.empty((N_SIMS, 24), dtype=torch.uint8, device="cuda")
    table = torch.empty((H, W, 8), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def step(ev=None):
        g.thresholds_dev(lid, d_beta, out=table, stream=stream)
        if ev is not None:
            ev[0].record(stream)
        g.run_dev(d_beta, d_sims, N_SIMS, SIM_SEED, out, override=table, stream=stream)
        if ev is not None:
            ev[1].record(stream)

    if args.calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        log("copy calibration: 3 x torch.neg over 268435456 B in, 268435456 B out")
        del a, b
    for _ in range(args.warmup):
        step()
    g.sync()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g.sync()
    sim_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    # the plan the timed launches used (built-in choice after the warm-up)
    sched = g.get_schedule(W * H, 1, N_SIMS)
    r = fire.results_to_numpy(out)
    trials = int(r["trials"].sum())
    burnt = int(r["burnt"].sum())
    ms_per_step = dt / args.steps * 1e3
    sims_per_s = N_SIMS * args.steps / dt
    trials_per_s = trials * args.steps / dt
    alg_bytes = 4 * trials + 8 * burnt + 24 * N_SIMS
    achieved = alg_bytes / (sim_ms * 1e-3) / 1e9
    log(f"{ms_per_step:.3f} ms/step, sim kernel {sim_ms:.3f} ms, {sims_per_s:.0f} sims/s, "
        f"{trials_per_s:.3e} trials/s, mean burnt {burnt / N_SIMS:.1f}, mean trials "
        f"{trials / N_SIMS:.1f}")

    prof = pmc_profile()
    wave = bool(sched.get("wave"))
    kname = "simw_kernel" if wave else "sim_kernel"
    log("probing the hardware ceilings ...")
    from paper_1701_03549_amd import probe
    ceil = probe.measure()
    # the ceilings this launch meets, each as the fraction of the measured
    # kernel time it explains
    sim_s = sim_ms * 1e-3
    units = 2 * burnt  # Philox evaluations the simulations need (2 per burning cell)
    # one step's dependent chain: queue entry (LDS), then the threshold load
    # (L2) alongside the Philox evaluation, then the bit atomics and the
    # append (LDS); plus a workgroup barrier per phase for sim_kernel
    lds = ceil["lds_atomic_ns"]
    step_ns = lds + max(ceil["l2_load_ns"], ceil["philox_ns"]) + 2 * lds
    if not wave:
        step_ns += 2 * ceil["barrier_ns"]
    max_steps = int(r["steps"].max())
    fractions = {
        "hbm": alg_bytes / sim_s / 1e9 / HBM_PEAK_GBS,
        "l2": alg_bytes / sim_s / 1e9 / ceil["l2_read_gbs"],
        "alu": units / sim_s / ceil["philox_calls_per_s"],
        "latency": max_steps * step_ns * 1e-9 / sim_s,
    }
    binding = max(fractions, key=fractions.get)
    log(f"ceilings: {ceil}; fractions {fractions} -> {binding}")
    result = {
        "metric": METRIC, "value": sims_per_s, "unit": "sims/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "calibration batch: 512x512 synthetic landscape (seed 102), "
                               "1280 replicates at the calibration vector, ignition on the "
                               "NW-facing slope nearest the centre, run to extinction, Eq. 2 "
                               "vs a contained reference fire",
                   "lattice": [W, H], "sims_per_step": N_SIMS, "beta": list(BETA_STAR),
                   "ignition": list(centre), "schedule": sched, "threshold_mode": "table",
                   "tuned_schedules": n_tuned},
        "trials_per_s": trials_per_s,
        "mean_burnt": burnt / N_SIMS, "mean_trials": trials / N_SIMS,
        "roofline": {
            "bound": binding,
            **({"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s"} if binding == "hbm" else
               {"achieved": alg_bytes / sim_s / 1e9, "peak": ceil["l2_read_gbs"], "unit": "GB/s"}
               if binding == "l2" else
               {"achieved": units / sim_s / 1e9, "peak": ceil["philox_calls_per_s"] / 1e9,
                "unit": "G Philox calls/s"} if binding == "alu" else
               {"achieved": max_steps * step_ns * 1e-6, "peak": sim_ms, "unit": "ms (chain of "
                "dependent steps vs kernel time)"}),
            "frac": fractions[binding],
            "traffic": prof.get("hbm_bytes_per_launch") if prof else None,
            "fractions": fractions,
            "hbm": {"achieved_gbs": achieved, "peak_gbs": HBM_PEAK_GBS,
                    "measured_read_gbs": ceil["hbm_read_gbs"]},
            "l2": {"peak_gbs": ceil["l2_read_gbs"], "mall_gbs": ceil["mall_read_gbs"]},
            "alu": {"philox_calls_per_launch": units, "trials_per_call": trials / units,
                    "peak_calls_per_s": ceil["philox_calls_per_s"],
                    "lane_slots_per_call": 256 * 2.4e9 * 64 / ceil["philox_calls_per_s"]},
            "latency": {"max_steps": max_steps, "step_floor_ns": step_ns,
                        "components_ns": {k: ceil[k] for k in ("barrier_ns", "l2_load_ns",
                                                               "lds_atomic_ns", "philox_ns")}},
            "issue": ({k: prof["sq"][k] for k in ("valu_busy_frac", "wave_busy_frac",
                                                "wave_wait_frac", "wave_issue_wait_frac")}
                      if prof and "sq" in prof else None),
            "kernel": kname, "kernel_ms": sim_ms,
            "algorithmic_bytes_per_launch": alg_bytes,
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        log("CPU oracle baseline (host threads, one thread; 512x512 and 64x64) ...")
        result["cpu_baseline"] = cpu_baseline(ls, centre, ref)
        cb = result["cpu_baseline"]
        log(f"oracle: {cb['value']:.0f} sims/s on {cb['cores']} threads, "
            f"{cb['one_core']['value']:.0f} on one; 64x64: {cb['plain_64']['value']:.0f}")
    if not args.no_ga:
        log("GA calibration runs ...")
        result["ga"] = run_ga(g, lid, tid, centre, plain=not args.no_plain)
        log("Monte Carlo fit ...")
        result["mc"] = run_mc(g, lid, tid, centre, result["ga"]["batched_sims_per_s"])
        log("7-gene GA ...")
        result["ignition_ga"] = run_ignition_ga(g, lid, tid, centre, ref)
    if not args.no_extra:
        log("per-cell path ...")
        result["dense"] = run_dense(g, lid, tid, centre, sims_per_s)
        log("turn-off times ...")
        result["turn_off"] = run_turn_off(g, lid, tid, centre, d_sims)
    g.close()
    if not args.no_extra:
        log("ignition scan ...")
        result["scan"] = run_scan(log)
        log("uneven batch ...")
        result["uneven"] = run_uneven(log)
    if not args.no_surrogate:
        log("surrogate ...")
        result["surrogate"] = run_surrogate(log)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
