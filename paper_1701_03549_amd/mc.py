"""Brute-force Monte Carlo fit (Appendix C) over the library.

Parameter vectors are drawn uniformly from the search box (numpy PCG64 under
`seed`: inputs, not model arithmetic), each is simulated once from the
ignition with the Eq. 2 fitness against the reference map (fire_run, one
persistent launch per chunk), and the ensemble with fitness under the cutoff
gives the best fit and the spread (fire_ensemble) — the same estimator as the
GA's, without the search.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import fire


def sample_params(n: int, seed: int, box=(-30.0, 30.0)) -> np.ndarray:
    return np.random.default_rng(seed).uniform(box[0], box[1], size=(n, 5))


def run_mc(g: fire.FireGPU, lid: int, tid: int, ign, n: int, seed: int, sim_seed: int,
           box=(-30.0, 30.0), cutoff=0.3, chunk=65536):
    """Returns dict(params, deltas (device), ensemble stats, trials, wall_s)."""
    params = sample_params(n, seed, box)
    deltas = torch.empty(n, dtype=torch.float64, device=g.device)
    trials = torch.empty(n, dtype=torch.int64, device=g.device)
    t0 = time.perf_counter()
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        sims = fire.make_sims(e - s, lid, tid, ign, param_index=np.arange(e - s),
                              sim_index=np.arange(s, e, dtype=np.uint32))
        res, _ = g.run(params[s:e], sims, sim_seed)
        v = res.view(torch.float64).reshape(-1, 3)
        deltas[s:e] = v[:, 2]
        trials[s:e] = res.view(torch.int64).reshape(-1, 3)[:, 1]
    g.sync()
    wall = time.perf_counter() - t0
    d_params = torch.from_numpy(params).to(g.device)
    ens = g.ensemble(d_params, deltas.reshape(n, 1), cutoff)
    g.sync()
    best = int(ens["best_individual"].item())
    return {"params": params, "deltas": deltas, "trials": trials, "wall_s": wall,
            "best_index": best, "best_params": params[best].tolist(),
            "best_fitness": float(deltas[best].item()),
            "n_accepted": int(ens["n_accepted"].item()),
            "accepted_mean": ens["mean"].cpu().tolist(), "accepted_sd": ens["sd"].cpu().tolist()}
