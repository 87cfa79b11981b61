"""GA calibration drivers (Appendix B) over the library's device operators.

``run_batched`` is the library's captured-graph GA (fire_ga_run): each
generation evaluates P individuals by R replicate simulations in one
persistent launch and applies the GA operators on the device.
``run_ignition`` is the 7-parameter search of Appendix B
(fire_ga_run_ignition): each individual also carries its ignition point as
genes 5 and 6, every generation's simulations start from each individual's
cell, and the initial points are drawn from the reference fire's burnt cells
(Methods: simulations start at a random point of the reference burnt area).
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


def ignition_box(W, H, beta_box=(-30.0, 30.0), beta_h=1.0, xy_h=None):
    """Per-gene (lo, hi, h) of the 7-gene search: the betas in `beta_box`
    with width `beta_h`, the coordinates on the lattice with width `xy_h`
    cells (default max(W, H) / 32)."""
    xy_h = float(max(W, H)) / 32.0 if xy_h is None else float(xy_h)
    lo = [beta_box[0]] * 5 + [0.0, 0.0]
    hi = [beta_box[1]] * 5 + [float(W - 1), float(H - 1)]
    h = [beta_h] * 5 + [xy_h, xy_h]
    return lo, hi, h


def initial_population_ignition(ref_bits, W, H, P, seed, prior_sd=5.0, beta_box=(-30.0, 30.0)):
    """P individuals (beta[5], x, y): betas Gaussian(0, prior_sd) clamped to
    the box (uniform over it if prior_sd is None), ignition cells uniform over
    the burnt cells of the reference map (packed rows, as given to
    fire_target_load)."""
    from .synth import unpack_bits
    rng = np.random.default_rng(seed)
    if prior_sd is None:
        betas = rng.uniform(beta_box[0], beta_box[1], size=(P, 5))
    else:
        betas = np.clip(rng.normal(0.0, prior_sd, size=(P, 5)), beta_box[0], beta_box[1])
    ys, xs = np.nonzero(unpack_bits(np.asarray(ref_bits).reshape(H, -1), W))
    if xs.size == 0:
        raise ValueError("empty reference map")
    k = rng.integers(0, xs.size, size=P)
    return np.concatenate([betas, xs[k, None].astype(np.float64), ys[k, None].astype(np.float64)],
                          axis=1)


def run_ignition(g: fire.FireGPU, lid, tid, pop0, R=20, generations=50, sim_seed=0, ga_seed=0,
                 elite=2, pm0=0.2, box=None, stream=None):
    """Captured-graph GA over (beta[5], x, y). Returns device histories."""
    W, H = g.dims[lid]
    lo, hi, h = box or ignition_box(W, H)
    return g.ga_run_ignition(lid, tid, pop0, R, elite=elite, pm0=pm0, generations=generations,
                             lo=lo, hi=hi, h=h, sim_seed=sim_seed, ga_seed=ga_seed,
                             stream=stream)


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
