"""Pins of the oracle's turn-off time (Methods: burnt cells stay active for a
time set by their vegetation before they become inactive; the paper's
results use one step for every type).

* one step for every type is the pinned one-step model, bit for bit;
* 1x2 lattices with thresholds 0 and 2^32-1 fix burnt, steps and trials in
  closed form for any turn-off times;
* on tiny lattices the final-burn distribution matches an exact
  enumeration of the process with lifetimes (independent of the oracle);
* for two cells, the chance the neighbour burns is 1 - (1 - p)^tau;
* with one fixed coin per edge (static-edge mode) the final burn is the set
  reachable through open edges, whatever the turn-off times.
"""
from collections import deque

import numpy as np
import pytest
from scipy import stats

import exact_enum
from paper_1701_03549_amd import synth

SEED = 0x5EED0001
BETA = (-0.9, -0.5, 0.3, 0.8, 1.0)


def _steps(mapping):
    b = np.ones(256, dtype=np.uint8)
    for v, k in mapping.items():
        b[v] = k
    return b


def test_one_step_everywhere_is_the_one_step_model(oracle_mod):
    ls = synth.make_landscape(48, 40, 101)
    T = oracle_mod.thresholds(ls, BETA)
    c = synth.nearest_burnable(ls["veg"], 24, 20)
    for k in range(20):
        a = oracle_mod.simulate(ls["veg"], T, c, k, SEED)
        b = oracle_mod.simulate(ls["veg"], T, c, k, SEED, burn_steps=np.ones(256, np.uint8))
        assert (a["burnt"], a["steps"], a["trials"]) == (b["burnt"], b["steps"], b["trials"])
        assert np.array_equal(a["map"], b["map"])


def _pair(t01, t10):
    # 1x2 lattice, cell 0 at x=0, cell 1 at x=1 (direction E = 2, W = 6)
    T = np.zeros((1, 2, 8), dtype=np.uint32)
    T[0, 0, 2] = t01
    T[0, 1, 6] = t10
    return T


@pytest.mark.parametrize("tau0,tau1", [(1, 1), (3, 1), (1, 4), (5, 2)])
def test_pair_closed_forms(oracle_mod, tau0, tau1):
    veg = np.array([[1, 2]], dtype=np.uint8)
    bs = _steps({1: tau0, 2: tau1})
    # never spreads: the ignition stays active tau0 steps, one trial each
    r = oracle_mod.simulate(veg, _pair(0, 0), (0, 0), 0, SEED, burn_steps=bs)
    assert (r["burnt"], r["steps"], r["trials"]) == (1, tau0, tau0)
    # always spreads: cell 1 ignites at the first step and is active for
    # tau1 steps after it; only the first step has an unburnt target
    r = oracle_mod.simulate(veg, _pair(0xFFFFFFFF, 0xFFFFFFFF), (0, 0), 0, SEED, burn_steps=bs)
    assert (r["burnt"], r["steps"], r["trials"]) == (2, max(tau0, 1 + tau1), 1)
    # max_steps cuts the run
    r = oracle_mod.simulate(veg, _pair(0, 0), (0, 0), 0, SEED, max_steps=2, burn_steps=bs)
    assert r["steps"] == min(2, tau0)


def test_isolated_ignition_burns_for_its_turn_off_time(oracle_mod):
    veg = np.array([[0, 0, 0], [0, 3, 0], [0, 0, 0]], dtype=np.uint8)
    T = np.full((3, 3, 8), 0xFFFFFFFF, dtype=np.uint32)
    r = oracle_mod.simulate(veg, T, (1, 1), 0, SEED, burn_steps=_steps({3: 7}))
    assert (r["burnt"], r["steps"], r["trials"]) == (1, 7, 0)


def test_zero_turn_off_time_is_rejected(oracle_mod):
    veg = np.array([[1, 2]], dtype=np.uint8)
    with pytest.raises(ValueError):
        oracle_mod.simulate(veg, _pair(0, 0), (0, 0), 0, SEED, burn_steps=_steps({2: 0}))


@pytest.mark.parametrize("tau", [1, 2, 4])
def test_pair_spread_probability(oracle_mod, tau):
    veg = np.array([[1, 1]], dtype=np.uint8)
    p_thr = 1 << 30  # p = 1/4 per try
    n = 20000
    hits = sum(oracle_mod.simulate(veg, _pair(p_thr, 0), (0, 0), k, SEED,
                                   burn_steps=_steps({1: tau}))["burnt"] == 2 for k in range(n))
    p = 1 - (1 - 0.25) ** tau
    assert abs(hits - n * p) <= 5 * np.sqrt(n * p * (1 - p))


def _patterns(oracle_mod, veg, T, ign, n, seed, bs):
    counts = {}
    H, W = veg.shape
    for k in range(n):
        r = oracle_mod.simulate(veg, T, ign, k, seed, burn_steps=bs)
        m = synth.unpack_bits(r["map"], W)
        key = frozenset((int(x), int(y)) for y, x in zip(*np.nonzero(m)))
        counts[key] = counts.get(key, 0) + 1
    return counts


@pytest.mark.parametrize("case", [
    dict(W=3, H=2, ign=(0, 0), beta=(-1.5, 0.0, 0.0, 0.0, 0.0), seed=None, life={1: 2}),
    dict(W=3, H=2, ign=(1, 0), beta=(-1.2, -1.2, 0.8, 1.1, 2.0), seed=31, life={1: 3, 2: 1}),
    dict(W=2, H=3, ign=(1, 2), beta=(-1.5, 1.0, -0.7, 1.6, 3.0), seed=32, life={1: 1, 2: 2}),
])
def test_exact_distribution_with_turn_off_times(oracle_mod, case):
    W, H = case["W"], case["H"]
    if case["seed"] is None:
        ls = synth.uniform_landscape(W, H)
    else:
        ls = synth.random_small_landscape(W, H, seed=case["seed"], p_blocked=0.0)
        ls["veg"][0, 0] = 1
        ls["veg"][H - 1, W - 1] = 2
    veg = ls["veg"]
    bs = _steps(case["life"])
    T = oracle_mod.thresholds(ls, case["beta"])
    probs = exact_enum.edge_probabilities_from_thresholds(T.tolist(), W, H)
    life = {(x, y): int(bs[veg[y, x]]) for y in range(H) for x in range(W)}
    dist = exact_enum.final_distribution_dur(W, H, veg > 0, probs, case["ign"], life)
    assert sum(dist.values()) == 1
    n = 20000
    counts = _patterns(oracle_mod, veg, T, case["ign"], n, SEED + 3, bs)
    obs, exp = [], []
    for k, p in dist.items():
        p = float(p)
        c = counts.get(k, 0)
        assert abs(c - n * p) <= 5 * np.sqrt(n * p * (1 - p)) + 1, (sorted(k), c, n * p)
        obs.append(c)
        exp.append(n * p)
    assert sum(counts.values()) == sum(counts.get(k, 0) for k in dist)  # no impossible pattern
    obs, exp = np.array(obs, float), np.array(exp, float)
    big = exp >= 5
    o = np.append(obs[big], obs[~big].sum())
    e = np.append(exp[big], exp[~big].sum())
    keep = e > 0
    chi2 = ((o[keep] - e[keep]) ** 2 / e[keep]).sum()
    assert stats.chi2.sf(chi2, max(keep.sum() - 1, 1)) > 1e-6
    # a longer turn-off time never makes the fire smaller in expectation
    one = exact_enum.final_distribution(W, H, veg > 0, probs, case["ign"])
    mean = lambda d: sum(len(k) * v for k, v in d.items())
    assert mean(dist) >= mean(one)


def test_static_edges_reachability_with_turn_off_times(oracle_mod):
    ls = synth.make_landscape(40, 32, 105)
    veg = ls["veg"]
    T = oracle_mod.thresholds(ls, BETA)
    H, W = veg.shape
    bs = _steps({int(v): 1 + (int(v) % 4) for v in np.unique(veg) if v})
    c = synth.nearest_burnable(veg, 20, 16)
    key = [SEED & 0xFFFFFFFF, SEED >> 32]
    for sim in range(4):
        r = oracle_mod.simulate(veg, T, c, sim, SEED, static_edges=True, burn_steps=bs)
        # open edges from the same coins, then plain BFS
        seen = {c}
        dq = deque([c])
        while dq:
            x, y = dq.popleft()
            s = y * W + x
            for d, (dx, dy) in enumerate(exact_enum.OFFSETS):
                tx, ty = x + dx, y + dy
                if not (0 <= tx < W and 0 <= ty < H) or veg[ty, tx] == 0 or (tx, ty) in seen:
                    continue
                coin = int(oracle_mod.philox([sim, 0, s, d // 4], key)[d % 4])
                thr = int(T[y, x, d])
                if thr == 0xFFFFFFFF or coin < thr:
                    seen.add((tx, ty))
                    dq.append((tx, ty))
        m = synth.unpack_bits(r["map"], W)
        got = {(int(x), int(y)) for y, x in zip(*np.nonzero(m))}
        assert got == seen
