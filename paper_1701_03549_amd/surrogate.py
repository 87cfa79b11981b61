"""Learned-surrogate pipeline over the library (sequencing of ABI calls).

1. ``make_dataset``: runs of the simulator (fire_run) on one landscape with
   parameter vectors drawn uniformly from the GA search box and ignitions
   uniform in the central half of the lattice; each run gives the inputs
   (beta, ignition), the target log(1 + delta) of its Eq. 2 fitness against
   the reference map, and its burn map pooled to 128x128 (fire_pool_maps).
2. ``train``: Adam on the fire_nn surrogate (MFMA bf16 GEMMs).
3. ``run_ga``: the GA (Appendix B operators on the device). With a network,
   each generation draws `oversample` offspring sets from the same parents;
   half of the non-elite population is the first set as the plain GA would
   keep it, the other half the best-predicted offspring of all sets
   (fire_nn_select); every kept individual is then evaluated by exact
   simulation, which is what the GA uses, and those exact evaluations
   fine-tune the network online. Without a network it is the plain GA and
   reproduces fire_ga_run bit for bit. A whole run can be captured as one
   HIP graph and replayed.

Training data drawn from the GA's own prior (Table 1's Gaussian) at the
reference ignition ranks the GA's candidates far better than data from the
whole search box (held-out Spearman 0.95 vs 0.85 at 256x256).
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import fire, nn


def make_dataset(g: fire.FireGPU, lid: int, tid: int, n: int, seed: int, sim_seed: int,
                 box=(-30.0, 30.0), chunk=8192, maps=True, prior_sd=None, ign=None):
    """Training runs. Parameters uniform in `box`, or Gaussian(0, prior_sd)
    clamped to it (Table 1's priors); ignitions uniform in the central half,
    or all at `ign`."""
    W, H = g.dims[lid]
    rng = np.random.default_rng(seed)
    if prior_sd is None:
        betas = rng.uniform(box[0], box[1], size=(n, 5))
    else:
        betas = np.clip(rng.normal(0.0, prior_sd, size=(n, 5)), box[0], box[1])
    if ign is None:
        ign = np.stack([rng.integers(W // 4, 3 * W // 4, n), rng.integers(H // 4, 3 * H // 4, n)], 1)
    else:
        ign = np.tile(np.asarray(ign, dtype=np.int64), (n, 1))
    X = torch.empty((n, 7), dtype=torch.float32, device=g.device)
    y_t = torch.empty(n, dtype=torch.float32, device=g.device)
    y_map = torch.empty((n, nn.MAP, nn.MAP), dtype=torch.uint8, device=g.device) if maps else None
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        sims = fire.make_sims(e - s, lid, tid, ign[s:e], param_index=np.arange(e - s),
                              sim_index=np.arange(s, e, dtype=np.uint32))
        res, m = g.run(betas[s:e], sims, sim_seed, want_maps=maps)
        d_par = torch.from_numpy(np.ascontiguousarray(betas[s:e])).to(g.device)
        d_ign = torch.from_numpy(ign[s:e].astype(np.float32)).to(g.device)
        nn.rows_from_results(res, e - s, params=d_par, ign=d_ign, out_x=X[s:e], out_y=y_t[s:e])
        if maps:
            y_map[s:e] = nn.pool_maps(m, e - s, W, H, m.shape[1])
    g.sync()
    return X, y_t, y_map


def train(net: nn.Surrogate, X, y_t, y_map, epochs=4, batch=512, lr=1e-3, seed=0, log=None):
    """Adam over shuffled minibatches (a host-side permutation per epoch;
    rows gathered on the device by fire_gather_rows); returns the mean
    losses of every epoch."""
    n = X.shape[0]
    dev = X.device
    rng = np.random.default_rng(seed)
    xb = torch.empty((batch, 7), dtype=torch.float32, device=dev)
    yb = torch.empty(batch, dtype=torch.float32, device=dev)
    mb = torch.empty((batch, nn.MAP, nn.MAP), dtype=torch.uint8, device=dev) \
        if y_map is not None else None
    steps = n // batch
    losses = torch.empty((max(steps, 1), 2), dtype=torch.float32, device=dev)
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n).astype(np.int64)).to(dev)
        for k in range(steps):
            idx = perm[k * batch:(k + 1) * batch]
            nn.gather_rows(X, idx, xb)
            nn.gather_rows(y_t, idx, yb)
            if mb is not None:
                nn.gather_rows(y_map, idx, mb)
            net.train_step(xb, yb, mb, lr=lr, out_loss=losses[k])
        ep_loss = losses[:steps].cpu().numpy().mean(axis=0) if steps else np.zeros(2)
        hist.append(ep_loss)
        if log:
            log(f"epoch {ep}: fitness loss {ep_loss[0]:.4f}, map loss {ep_loss[1]:.4f}")
    return hist


def spearman(a: np.ndarray, b: np.ndarray) -> float:
    ra = np.argsort(np.argsort(a)).astype(np.float64)
    rb = np.argsort(np.argsort(b)).astype(np.float64)
    ra -= ra.mean()
    rb -= rb.mean()
    return float((ra * rb).sum() / np.sqrt((ra ** 2).sum() * (rb ** 2).sum()))


def online_indices(generations: int, P: int, R: int, steps: int, batch: int, seed: int):
    """Minibatch rows of the online Adam steps of every generation, drawn
    before the first generation runs: generation g draws `steps` batches of
    min(batch, (g + 1) P R) rows uniformly from the (g + 1) P R exact
    evaluations made so far."""
    rng = np.random.default_rng(seed)
    return [rng.integers(0, (gen + 1) * P * R, size=(steps, min(batch, (gen + 1) * P * R)))
            for gen in range(generations)]


def run_ga(g: fire.FireGPU, lid, tid, ign, pop0, R=20, generations=50, sim_seed=0, ga_seed=0,
           net: nn.Surrogate | None = None, oversample=8, cfg=None, online_steps=1,
           online_lr=5e-4, unscreened=None, seed=0, graph=False):
    """GA with optional surrogate screening. Returns (hist_pop, hist_fit,
    timings). With screening: `unscreened` offspring of the first set are
    kept as the plain GA would keep them, the rest of the population is the
    best-predicted of all `oversample` sets; with `online_steps` > 0 the
    network takes that many Adam steps per generation on minibatches of the
    exact evaluations made so far (which are free training data). One step
    per generation keeps the accuracy of eight at a third of the time.

    With `graph`, the whole run (every generation's simulations, network
    steps, GA steps and selections) is captured as one HIP graph and replayed
    once; the results are those of the eager run with the same arguments and
    a network in the same state. Eager runs time simulation and screening
    separately (a device synchronisation after each part of a generation)."""
    from .ga import default_cfg
    cfg = cfg or default_cfg(generations)
    P = pop0.shape[0]
    E = int(cfg.elite)
    dev = g.device
    screen = net is not None and oversample > 1
    pop_in = torch.from_numpy(np.ascontiguousarray(pop0, dtype=np.float64)).to(dev)
    pop = torch.empty_like(pop_in)
    hist_pop = torch.empty((generations, P, 5), dtype=torch.float64, device=dev)
    hist_fit = torch.empty((generations, P, R), dtype=torch.float64, device=dev)
    res = torch.empty((P * R, 24), dtype=torch.uint8, device=dev)
    # every generation's descriptors, on the device before the first one runs
    sims = fire.make_sims(generations * P * R, lid, tid, ign,
                          param_index=np.tile(np.repeat(np.arange(P), R), generations))
    d_sims_all = torch.from_numpy(sims.view(np.uint8).copy()).to(dev).reshape(-1, 28)
    ign_xy = (float(ign[0]), float(ign[1]))
    online = screen and online_steps > 0
    if online:
        bank_x = torch.empty((generations * P * R, 7), dtype=torch.float32, device=dev)
        bank_y = torch.empty(generations * P * R, dtype=torch.float32, device=dev)
        xb = torch.empty((net.max_batch, 7), dtype=torch.float32, device=dev)
        yb = torch.empty(net.max_batch, dtype=torch.float32, device=dev)
        idx = [torch.from_numpy(a.astype(np.int64)).to(dev)
               for a in online_indices(generations, P, R, online_steps, net.max_batch, seed)]
    if screen:
        sets = torch.empty((oversample, P, 5), dtype=torch.float64, device=dev)
        n_cand = P + (oversample - 1) * (P - E)
        cand = torch.empty((n_cand, 5), dtype=torch.float64, device=dev)
        x = torch.empty((n_cand, 7), dtype=torch.float32, device=dev)
        score = torch.empty(n_cand, dtype=torch.float32, device=dev)
    keep = E + ((P - E) // 2 if unscreened is None else unscreened)
    timing = {"simulation_s": 0.0, "screening_s": 0.0}

    def body(stream, eager):
        pop.copy_(pop_in)
        for gen in range(generations):
            d_sims = d_sims_all[gen * P * R:(gen + 1) * P * R]
            fit = hist_fit[gen]
            hist_pop[gen].copy_(pop)
            t0 = time.perf_counter()
            g.run_dev(pop, d_sims, P * R, sim_seed, res, stream=stream)
            if online:
                # the exact evaluations join the online training bank
                k0 = gen * P * R
                nn.rows_from_results(res, P * R, params=pop, reps=R, ign_xy=ign_xy,
                                     out_x=bank_x[k0:k0 + P * R], out_y=bank_y[k0:k0 + P * R],
                                     out_fit=fit, stream=stream)
            else:
                nn.rows_from_results(res, P * R, out_fit=fit, stream=stream)
            if eager:
                torch.cuda.synchronize()
                timing["simulation_s"] += time.perf_counter() - t0
            if not screen:
                g.ga_step(pop, fit, cfg, gen, ga_seed, stream=stream)
                continue
            t0 = time.perf_counter()
            if online:
                for s in range(online_steps):
                    rows = idx[gen][s]
                    nb = rows.shape[0]
                    nn.gather_rows(bank_x, rows, xb, stream=stream)
                    nn.gather_rows(bank_y, rows, yb, stream=stream)
                    net.train_step(xb[:nb], yb[:nb], None, lr=online_lr, stream=stream)
            g.ga_offspring(pop, fit, cfg, gen, ga_seed, 0x9E3779B97F4A7C15, sets, stream=stream)
            nn.candidates(sets, E, ign_xy, cand, x, stream=stream)
            net.predict(x, out=score, stream=stream)
            nn.select(cand, score, keep=keep, k=P, out=pop, stream=stream)
            if eager:
                torch.cuda.synchronize()
                timing["screening_s"] += time.perf_counter() - t0

    if not graph:
        body(torch.cuda.current_stream(), True)
        g.sync()
        return hist_pop, hist_fit, timing
    # the context's simulation buffers must not grow under capture: one
    # eager launch of a generation's batch sizes them
    g.run_dev(pop_in, d_sims_all[:P * R], P * R, sim_seed, res)
    g.sync()
    t0 = time.perf_counter()
    G = torch.cuda.CUDAGraph()
    with torch.cuda.graph(G):
        body(torch.cuda.current_stream(), False)
    timing["capture_s"] = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G.replay()
    torch.cuda.synchronize()
    timing["replay_s"] = time.perf_counter() - t0
    del G
    g.sync()
    return hist_pop, hist_fit, timing


def make_ignition_dataset(g: fire.FireGPU, lid: int, tid: int, beta, box, n: int, seed: int,
                          sim_seed: int, chunk=8192):
    """Training runs for ignition screening: parameters fixed at `beta`,
    ignition cells uniform over box = (x0, y0, w, h). Inputs are
    (beta, x - x0, y - y0), for a network whose lattice is the box (w, h);
    targets log(1 + delta) against the reference map."""
    x0, y0, bw, bh = box
    rng = np.random.default_rng(seed)
    ign = np.stack([rng.integers(x0, x0 + bw, n), rng.integers(y0, y0 + bh, n)], 1)
    X = torch.empty((n, 7), dtype=torch.float32, device=g.device)
    y_t = torch.empty(n, dtype=torch.float32, device=g.device)
    beta = np.asarray(beta, dtype=np.float64)
    d_beta = torch.from_numpy(beta.reshape(1, 5).copy()).to(g.device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        sims = fire.make_sims(e - s, lid, tid, ign[s:e], param_index=0,
                              sim_index=np.arange(s, e, dtype=np.uint32))
        res, _ = g.run(beta[None, :], sims, sim_seed)
        d_ign = torch.from_numpy((ign[s:e] - np.array([x0, y0])).astype(np.float32)).to(g.device)
        nn.rows_from_results(res, e - s, params=d_beta, reps=e - s, ign=d_ign, out_x=X[s:e],
                             out_y=y_t[s:e])
    g.sync()
    return X, y_t


def screen_ignitions(net: nn.Surrogate, beta, cands, box, keep: int) -> np.ndarray:
    """Grid positions of the `keep` candidate cells with the lowest predicted
    fitness (a network trained by make_ignition_dataset on the same box)."""
    x0, y0 = box[0], box[1]
    c = np.asarray(cands, dtype=np.float64)
    xh = np.empty((len(c), 7), dtype=np.float32)
    xh[:, :5] = np.asarray(beta, dtype=np.float64).astype(np.float32)
    xh[:, 5:] = (c - np.array([x0, y0])).astype(np.float32)
    score = net.predict(torch.from_numpy(xh).to(net.device)).cpu().numpy()
    return np.sort(np.argsort(score, kind="stable")[:keep])


def screened_scan(g: fire.FireGPU, net: nn.Surrogate, lid, tid, beta, cands, box, keep, R=32,
                  seed=0, cutoff=0.3):
    """Ignition scan of the `keep` best-predicted candidates only, each by R
    exact simulations with the coins the full scan would draw for it (its
    rows equal the full scan's rows). Returns (kept grid positions, scan)."""
    from . import scan
    kept = screen_ignitions(net, beta, cands, box, keep)
    out = scan.run_scan(g, lid, tid, beta, np.asarray(cands)[kept], R=R, seed=seed,
                        cutoff=cutoff, index=kept)
    return kept, out


def best_mean_fitness(hist_fit: torch.Tensor) -> float:
    """Lowest mean-over-replicates fitness of any evaluated individual."""
    return float(hist_fit.cpu().numpy().mean(axis=2).min())
