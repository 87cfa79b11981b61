"""GA calibration drivers (Appendix B) over the library's device operators.

``run_batched`` is the library's captured-graph GA (fire_ga_run): each
generation evaluates P individuals by R replicate simulations in one
persistent launch and applies the GA operators on the device.
``run_plain`` evaluates the same generations one simulation per launch with a
host synchronisation after each (the paper's execution style: simulations run
one after another) and applies the same device GA step; because every
fitness value is bit-identical, both produce the same trajectory.
"""
from __future__ import annotations

import numpy as np
import torch

from . import fire


def default_cfg(generations=50):
    return fire.FireGPU.ga_cfg(elite=2, pm0=0.2, mut_h=1.0, lo=-30.0, hi=30.0,
                               generations=generations)


def run_batched(g: fire.FireGPU, lid, tid, ign, pop0, R=20, generations=50, sim_seed=0,
                ga_seed=0, cfg=None, stream=None):
    cfg = cfg or default_cfg(generations)
    return g.ga_run(lid, tid, ign, pop0, R, cfg, sim_seed, ga_seed, stream=stream)


def run_plain(g: fire.FireGPU, lid, tid, ign, pop0, R=20, generations=50, sim_seed=0,
              ga_seed=0, cfg=None, progress=None):
    cfg = cfg or default_cfg(generations)
    pop0 = np.ascontiguousarray(pop0, dtype=np.float64)
    P = pop0.shape[0]
    dev = g.device
    stream = torch.cuda.current_stream()
    pop = torch.from_numpy(pop0.copy()).to(dev)
    hist_pop = torch.empty((generations, P, 5), dtype=torch.float64, device=dev)
    hist_fit = torch.empty((generations, P, R), dtype=torch.float64, device=dev)
    # one descriptor per simulation of every generation, on the device
    sims = fire.make_sims(generations * P * R, lid, tid, ign, param_index=0)
    d_sims = torch.from_numpy(sims.view(np.uint8).copy()).to(dev).reshape(-1, 28)
    res = torch.empty((P * R, 24), dtype=torch.uint8, device=dev)
    fit = torch.empty((P, R), dtype=torch.float64, device=dev)
    for gen in range(generations):
        hist_pop[gen].copy_(pop)
        for i in range(P):
            for r in range(R):
                k = i * R + r
                g.run_dev(pop[i], d_sims[(gen * P + i) * R + r], 1, sim_seed, res[k],
                          stream=stream)
                stream.synchronize()
        fit.copy_(res.view(torch.float64).reshape(P * R, 3)[:, 2].reshape(P, R))
        hist_fit[gen].copy_(fit)
        g.ga_step(pop, fit, cfg, gen, ga_seed, stream=stream)
        if progress is not None:
            progress(gen)
    g.sync()
    return hist_pop, hist_fit


def recovered(g: fire.FireGPU, hist, cutoff=0.3):
    """Best individual and accepted-ensemble statistics of a GA history."""
    hist_pop, hist_fit = hist
    gens, P, G = hist_pop.shape
    R = hist_fit.shape[2]
    params = hist_pop.reshape(gens * P, G).contiguous()
    deltas = hist_fit.reshape(gens * P, R).contiguous()
    e = g.ensemble(params, deltas, cutoff)
    g.sync()
    best = int(e["best_individual"].item())
    return {"best_params": params[best].cpu().tolist(),
            "best_fitness": float(deltas[best].min().item()),
            "best_mean_fitness": float(deltas[best].mean().item()),
            "n_accepted": int(e["n_accepted"].item()),
            "accepted_mean": e["mean"].cpu().tolist(), "accepted_sd": e["sd"].cpu().tolist()}
