"""Pins of the oracle's simulation (Methods, "Forest Fire Spread Simulation").

* p = 0 burns only the ignition; p = 1 burns exactly the cells of the
  8-connected burnable component within t steps (textbook BFS layers), with
  a trial count fixed by those layers.
* Non-burnable cells never burn; a non-burnable ignition burns nothing.
* With one fixed coin per directed edge (static-edge mode) the final burn is
  the set reachable from the ignition through open edges.
* On 2x2 and 3x2 lattices the Monte Carlo distribution of final burn maps
  matches the exact distribution obtained by summing over every coin outcome
  (tests/exact_enum.py), within binomial bounds and a chi-square test; the
  2x2 distributions also match hand-derived values (tests/golden).
"""
import json
import os
from collections import deque
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import exact_enum
from paper_1701_03549_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
OFFS = exact_enum.OFFSETS
SEED = 0x5EED0001
U32 = 0xFFFFFFFF


def bfs_layers(veg, ign):
    """Chebyshev BFS over burnable cells -> list of layers (sets of (x, y))."""
    H, W = veg.shape
    seen = {ign}
    layers = [{ign}]
    q = deque([ign])
    dist = {ign: 0}
    while q:
        c = q.popleft()
        for dx, dy in OFFS:
            t = (c[0] + dx, c[1] + dy)
            if 0 <= t[0] < W and 0 <= t[1] < H and veg[t[1], t[0]] != 0 and t not in seen:
                seen.add(t)
                dist[t] = dist[c] + 1
                if dist[t] == len(layers):
                    layers.append(set())
                layers[dist[t]].add(t)
                q.append(t)
    return layers


def mask_of(cells, W, H):
    m = np.zeros((H, W), dtype=bool)
    for x, y in cells:
        m[y, x] = True
    return m


def test_p_zero_burns_only_ignition(oracle_mod):
    ls = synth.make_landscape(40, 30, 7)
    T = oracle_mod.thresholds(ls, (-1000, 0, 0, 0, 0))
    ys, xs = np.nonzero(ls["veg"])
    for k in range(5):
        ign = (int(xs[k * 37]), int(ys[k * 37]))
        r = oracle_mod.simulate(ls["veg"], T, ign, k, SEED)
        assert r["burnt"] == 1 and r["steps"] == 1
        n_nb = sum(1 for dx, dy in OFFS
                   if 0 <= ign[0] + dx < 40 and 0 <= ign[1] + dy < 30 and ls["veg"][ign[1] + dy, ign[0] + dx])
        assert r["trials"] == n_nb
        assert np.array_equal(synth.unpack_bits(r["map"], 40), mask_of([ign], 40, 30))


@pytest.mark.parametrize("seed", [11, 12])
def test_p_one_is_bfs_ball(oracle_mod, seed):
    W, H = 45, 33
    ls = synth.make_landscape(W, H, seed)
    veg = ls["veg"]
    T = oracle_mod.thresholds(ls, (1000, 0, 0, 0, 0))
    ys, xs = np.nonzero(veg)
    ign = (int(xs[len(xs) // 2]), int(ys[len(ys) // 2]))
    layers = bfs_layers(veg, ign)
    for t in (0, 1, 2, 5, len(layers) - 1, len(layers), U32):
        r = oracle_mod.simulate(veg, T, ign, 3, SEED, max_steps=t)
        k = min(t, len(layers) - 1)
        ball = set().union(*layers[:k + 1])
        assert np.array_equal(synth.unpack_bits(r["map"], W), mask_of(ball, W, H)), t
        assert r["burnt"] == len(ball)
        assert r["steps"] == min(t, len(layers))
        # trials: every (layer-i cell, burnable neighbour not in layers 0..i) pair
        trials = 0
        for i in range(min(t, len(layers))):
            before = set().union(*layers[:i + 1])
            for (x, y) in layers[i]:
                for dx, dy in OFFS:
                    u = (x + dx, y + dy)
                    if 0 <= u[0] < W and 0 <= u[1] < H and veg[u[1], u[0]] and u not in before:
                        trials += 1
        assert r["trials"] == trials


def test_nonburnable_never_burns(oracle_mod):
    for seed in range(4):
        ls = synth.random_small_landscape(24, 19, seed=seed, p_blocked=0.3)
        T = oracle_mod.thresholds(ls, (0.5, 0.2, -0.3, 0.9, 1.0))
        ys, xs = np.nonzero(ls["veg"])
        for k in range(10):
            ign = (int(xs[k]), int(ys[k]))
            r = oracle_mod.simulate(ls["veg"], T, ign, k, SEED)
            m = synth.unpack_bits(r["map"], 24)
            assert not np.any(m & (ls["veg"] == 0))
            assert m[ign[1], ign[0]]
            assert m.sum() == r["burnt"]
            # the burnt set is 8-connected and contains the ignition
            comp = set().union(*bfs_layers(np.where(m, 1, 0).astype(np.uint8), ign))
            assert len(comp) == r["burnt"]


def test_nonburnable_ignition(oracle_mod):
    ls = synth.random_small_landscape(10, 10, seed=9, p_blocked=0.3)
    T = oracle_mod.thresholds(ls, (5, 0, 0, 0, 0))
    ys, xs = np.nonzero(ls["veg"] == 0)
    r = oracle_mod.simulate(ls["veg"], T, (int(xs[0]), int(ys[0])), 0, SEED)
    assert (r["burnt"], r["steps"], r["trials"]) == (0, 0, 0)
    assert not r["map"].any()


def test_max_steps_zero(oracle_mod):
    ls = synth.uniform_landscape(8, 8)
    T = oracle_mod.thresholds(ls, (5, 0, 0, 0, 0))
    r = oracle_mod.simulate(ls["veg"], T, (3, 3), 0, SEED, max_steps=0)
    assert (r["burnt"], r["steps"], r["trials"]) == (1, 0, 0)


def test_static_edges_is_open_edge_reachability(oracle_mod):
    W, H = 30, 22
    ls = synth.make_landscape(W, H, 21)
    veg = ls["veg"]
    T = oracle_mod.thresholds(ls, (-0.2, 0.3, 0.4, 0.9, 2.0))
    ys, xs = np.nonzero(veg)
    for sim in range(6):
        ign = (int(xs[sim * 50]), int(ys[sim * 50]))
        # open(s, d): the fixed coin of the edge under step word 0
        openset = {}
        for y in range(H):
            for x in range(W):
                s = y * W + x
                words = [oracle_mod.philox([sim, 0, s, g], [SEED, 0]) for g in (0, 1)]
                for d in range(8):
                    thr = int(T[y, x, d])
                    r = int(words[d // 4][d % 4])
                    openset[(x, y, d)] = thr == U32 or r < thr
        seen = {ign}
        q = deque([ign])
        while q:
            x, y = q.popleft()
            for d, (dx, dy) in enumerate(OFFS):
                t = (x + dx, y + dy)
                if 0 <= t[0] < W and 0 <= t[1] < H and veg[t[1], t[0]] and t not in seen \
                        and openset[(x, y, d)]:
                    seen.add(t)
                    q.append(t)
        r = oracle_mod.simulate(veg, T, ign, sim, SEED, static_edges=True)
        assert np.array_equal(synth.unpack_bits(r["map"], W), mask_of(seen, W, H))


def _mc_patterns(oracle_mod, veg, T, ign, n, seed):
    W = veg.shape[1]
    counts = {}
    for i in range(n):
        r = oracle_mod.simulate(veg, T, ign, i, seed)
        m = synth.unpack_bits(r["map"], W)
        key = frozenset((int(x), int(y)) for y, x in zip(*np.nonzero(m)))
        counts[key] = counts.get(key, 0) + 1
    return counts


def _check_distribution(counts, dist, n):
    assert set(counts) <= set(k for k, v in dist.items() if v > 0)
    obs, exp = [], []
    for k, p in dist.items():
        p = float(p)
        c = counts.get(k, 0)
        sd = np.sqrt(n * p * (1 - p))
        assert abs(c - n * p) <= 5 * sd + 1, (sorted(k), c, n * p)
        obs.append(c)
        exp.append(n * p)
    obs, exp = np.array(obs, float), np.array(exp, float)
    big = exp >= 5
    o = np.append(obs[big], obs[~big].sum())
    e = np.append(exp[big], exp[~big].sum())
    keep = e > 0
    chi2 = ((o[keep] - e[keep]) ** 2 / e[keep]).sum()
    assert stats.chi2.sf(chi2, max(keep.sum() - 1, 1)) > 1e-6


def test_golden_2x2(oracle_mod):
    with open(os.path.join(HERE, "golden", "tiny_lattices.json")) as f:
        g = json.load(f)
    for case in g["cases"]:
        W, H = case["W"], case["H"]
        ls = synth.uniform_landscape(W, H)
        T = oracle_mod.thresholds(ls, case["beta"])
        valid = T > 0
        assert np.all(T[valid] == case["threshold"])
        probs = exact_enum.edge_probabilities_from_thresholds(T.tolist(), W, H)
        dist = exact_enum.final_distribution(W, H, ls["veg"] > 0, probs, tuple(case["ign"]))
        want = {int(k): Fraction(v) for k, v in case["burnt_count"].items()}
        assert exact_enum.by_count(dist) == want
        n = 20000
        counts = _mc_patterns(oracle_mod, ls["veg"], T, tuple(case["ign"]), n, SEED)
        _check_distribution(counts, dist, n)


@pytest.mark.parametrize("case", [
    dict(W=3, H=2, ign=(0, 0), beta=(0.0, 0, 0, 0, 0), seed=None),
    dict(W=3, H=2, ign=(1, 0), beta=(0.3, -1.2, 0.8, 1.1, 2.0), seed=31),
    dict(W=2, H=3, ign=(1, 2), beta=(-0.5, 1.0, -0.7, 1.6, 3.0), seed=32),
    dict(W=3, H=2, ign=(2, 1), beta=(-0.1, 0.4, 1.5, -1.3, 0.0), seed=33),
])
def test_exact_distribution_tiny(oracle_mod, case):
    W, H = case["W"], case["H"]
    if case["seed"] is None:
        ls = synth.uniform_landscape(W, H)
    else:
        ls = synth.random_small_landscape(W, H, seed=case["seed"], p_blocked=0.0)
        ls["veg"][0, 0] = 1  # mixed forest / other
    T = oracle_mod.thresholds(ls, case["beta"])
    probs = exact_enum.edge_probabilities_from_thresholds(T.tolist(), W, H)
    dist = exact_enum.final_distribution(W, H, ls["veg"] > 0, probs, case["ign"])
    assert sum(dist.values()) == 1
    n = 20000
    counts = _mc_patterns(oracle_mod, ls["veg"], T, case["ign"], n, SEED + 1)
    _check_distribution(counts, dist, n)
