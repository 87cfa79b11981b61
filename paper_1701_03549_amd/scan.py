"""Ignition-point estimation by a candidate scan over the library.

The paper estimates the ignition point (Methods, propagation rules; the
ignition-point discussion of the results) by letting it vary inside the
reference burnt area. This driver evaluates a grid of candidate ignition
cells, each by R replicate simulations scored with Eq. 2 against the
reference map, and reduces them on the device (fire_scan_reduce) to a
per-candidate mean, spread, acceptance rate under the cutoff and a
normalised posterior-like map.
"""
from __future__ import annotations

import numpy as np
import torch

from . import fire


def candidate_grid(centre, W, H, spacing=4, half=8):
    """(2*half)^2 candidate cells (x0 + spacing*i, y0 + spacing*j), i, j in
    [-half, half), clamped to the lattice; the true cell is i = j = 0."""
    x0, y0 = centre
    offs = np.arange(-half, half) * spacing
    xs = np.clip(x0 + offs, 0, W - 1)
    ys = np.clip(y0 + offs, 0, H - 1)
    gy, gx = np.meshgrid(ys, xs, indexing="ij")
    return np.stack([gx.ravel(), gy.ravel()], axis=1).astype(np.int32)


def scan_sims(lid, tid, cands, R, index=None):
    """Descriptors: candidate c (grid index index[c], default c), replicate
    r -> sim_index index[c]*R + r, so a scan of a subset of the grid draws
    the same coins for a candidate as the scan of the whole grid."""
    n = len(cands) * R
    ign = np.repeat(cands, R, axis=0)
    index = np.arange(len(cands)) if index is None else np.asarray(index)
    sim_index = (np.repeat(index.astype(np.int64), R) * R + np.tile(np.arange(R), len(cands)))
    return fire.make_sims(n, lid, tid, ign, param_index=0, sim_index=sim_index.astype(np.uint32))


def run_scan(g: fire.FireGPU, lid, tid, beta, cands, R=32, seed=0, cutoff=0.3, tau=0.1,
             stream=None, index=None):
    """Evaluate every candidate; returns device tensors (deltas [C][R] and the
    reduction) plus the raw results. `index` gives the candidates' positions
    in a larger grid (their coins follow those positions)."""
    sims = scan_sims(lid, tid, cands, R, index)
    res, _ = g.run(np.asarray([beta], dtype=np.float64), sims, seed, stream=stream)
    deltas = res.view(torch.float64).reshape(-1, 3)[:, 2].reshape(len(cands), R).contiguous()
    red = g.scan_reduce(deltas, cutoff, tau=tau, stream=stream)
    red["deltas"] = deltas
    red["results"] = res
    return red
