"""Pins of the oracle's per-target form of the propagation rule (one uniform
per candidate target per step against 1 - prod(1 - p_i), the paper's
per-cell kernel), which the dense ablation kernel follows:

* p = 0 and p = 1 give the one-step model's results (ignition alone; BFS
  layers with their burnt and step counts);
* on tiny lattices the final-burn distribution matches the exact
  enumeration of the per-target rule (tests/exact_enum.py);
* with one burning neighbour the per-target threshold is that edge's;
* on a real landscape the burnt-size law matches the per-edge model's
  (two-sample tests): the two forms are equal in distribution, not bit-equal.
"""
import numpy as np
import pytest
from scipy import stats

import exact_enum
from paper_1701_03549_amd import synth
from test_oracle_simulate import OFFS, SEED, bfs_layers, mask_of

U32 = 0xFFFFFFFF


def test_p_zero_and_nonburnable(oracle_mod):
    ls = synth.make_landscape(40, 30, 7)
    T = oracle_mod.thresholds(ls, (-1000, 0, 0, 0, 0))
    ys, xs = np.nonzero(ls["veg"])
    ign = (int(xs[50]), int(ys[50]))
    r = oracle_mod.simulate_dense(ls["veg"], T, ign, 0, SEED)
    n_nb = sum(1 for dx, dy in OFFS
               if 0 <= ign[0] + dx < 40 and 0 <= ign[1] + dy < 30 and ls["veg"][ign[1] + dy, ign[0] + dx])
    assert (r["burnt"], r["steps"], r["trials"]) == (1, 1, n_nb)
    zy, zx = np.nonzero(ls["veg"] == 0)
    r = oracle_mod.simulate_dense(ls["veg"], T, (int(zx[0]), int(zy[0])), 0, SEED)
    assert (r["burnt"], r["steps"], r["trials"]) == (0, 0, 0) and not r["map"].any()
    r = oracle_mod.simulate_dense(ls["veg"], T, ign, 0, SEED, max_steps=0)
    assert (r["burnt"], r["steps"], r["trials"]) == (1, 0, 0)


def test_p_one_is_bfs(oracle_mod):
    W, H = 45, 33
    ls = synth.make_landscape(W, H, 11)
    veg = ls["veg"]
    T = oracle_mod.thresholds(ls, (1000, 0, 0, 0, 0))
    ys, xs = np.nonzero(veg)
    ign = (int(xs[len(xs) // 2]), int(ys[len(ys) // 2]))
    layers = bfs_layers(veg, ign)
    for t in (0, 1, 3, len(layers) - 1, U32):
        r = oracle_mod.simulate_dense(veg, T, ign, 3, SEED, max_steps=t)
        k = min(t, len(layers) - 1)
        ball = set().union(*layers[:k + 1])
        assert np.array_equal(synth.unpack_bits(r["map"], W), mask_of(ball, W, H)), t
        assert r["burnt"] == len(ball) and r["steps"] == min(t, len(layers))
        # trials: cells of layer i+1 plus unreachable-by-then burnable cells
        # next to layer i; with p = 1 every candidate of a step ignites, so
        # the draws are exactly the next layer's cells
        assert r["trials"] == sum(len(layers[i + 1]) for i in range(min(t, len(layers) - 1)))


def test_single_neighbour_threshold_is_the_edge_threshold(oracle_mod):
    veg = np.array([[1, 1]], dtype=np.uint8)
    T = np.zeros((1, 2, 8), dtype=np.uint32)
    T[0, 0, 2] = 3 << 30  # p = 3/4
    n = 20000
    hits = sum(oracle_mod.simulate_dense(veg, T, (0, 0), k, SEED)["burnt"] == 2 for k in range(n))
    assert abs(hits - 0.75 * n) <= 5 * np.sqrt(n * 0.75 * 0.25)


@pytest.mark.parametrize("case", [
    dict(W=3, H=2, ign=(0, 0), beta=(0.0, 0, 0, 0, 0), seed=None),
    dict(W=3, H=2, ign=(1, 0), beta=(0.3, -1.2, 0.8, 1.1, 2.0), seed=31),
    dict(W=2, H=3, ign=(1, 2), beta=(-0.5, 1.0, -0.7, 1.6, 3.0), seed=32),
])
def test_exact_distribution(oracle_mod, case):
    W, H = case["W"], case["H"]
    if case["seed"] is None:
        ls = synth.uniform_landscape(W, H)
    else:
        ls = synth.random_small_landscape(W, H, seed=case["seed"], p_blocked=0.0)
        ls["veg"][0, 0] = 1
    T = oracle_mod.thresholds(ls, case["beta"])
    probs = exact_enum.edge_probabilities_from_thresholds(T.tolist(), W, H)
    dist = exact_enum.final_distribution(W, H, ls["veg"] > 0, probs, case["ign"])
    n = 20000
    counts = {}
    for k in range(n):
        r = oracle_mod.simulate_dense(ls["veg"], T, case["ign"], k, SEED + 7)
        m = synth.unpack_bits(r["map"], W)
        key = frozenset((int(x), int(y)) for y, x in zip(*np.nonzero(m)))
        counts[key] = counts.get(key, 0) + 1
    assert set(counts) <= set(dist)
    obs = np.array([counts.get(k, 0) for k in dist], float)
    exp = np.array([float(p) * n for p in dist.values()])
    for o, e in zip(obs, exp):
        assert abs(o - e) <= 5 * np.sqrt(e * (1 - e / n)) + 1
    big = exp >= 5
    o = np.append(obs[big], obs[~big].sum())
    e = np.append(exp[big], exp[~big].sum())
    keep = e > 0
    chi2 = ((o[keep] - e[keep]) ** 2 / e[keep]).sum()
    assert stats.chi2.sf(chi2, max(keep.sum() - 1, 1)) > 1e-6


def test_same_law_as_per_edge_model(oracle_mod):
    ls = synth.make_landscape(48, 40, 101)
    T = oracle_mod.thresholds(ls, (-0.9, -0.5, 0.3, 0.8, 1.0))
    c = synth.nearest_burnable(ls["veg"], 24, 20)
    n = 3000
    dense = np.array([oracle_mod.simulate_dense(ls["veg"], T, c, k, SEED)["burnt"] for k in range(n)])
    edge = np.array([oracle_mod.simulate(ls["veg"], T, c, k, SEED + 1, want_map=False)["burnt"]
                     for k in range(n)])
    assert stats.ks_2samp(dense, edge).pvalue > 1e-4
    assert stats.mannwhitneyu(dense, edge).pvalue > 1e-4
    assert dense.std() > 0
    # not the same realisations
    assert np.mean(dense == edge) < 0.9
