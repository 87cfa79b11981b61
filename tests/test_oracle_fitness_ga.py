"""Pins of the oracle's Eq. 2 fitness, GA operators (Appendix B) and the
ensemble / ignition-scan statistics.

Eq. 2: delta = (|A u A*| - |A n A*|) / |A| with A the reference and A* the
simulated map; 0 when the maps coincide. Checked against set arithmetic on
random maps. The GA operators are checked through the properties the
appendix states (elitism keeps the best, a tournament picks the better of
two, one-point crossover swaps gene tails, mutation is a small change whose
probability falls with the generation).
"""
import numpy as np
import pytest

from paper_1701_03549_amd import synth


def test_fitness_identities(oracle_mod):
    rng = np.random.default_rng(0)
    for W, H in ((1, 1), (5, 3), (33, 7), (64, 64), (70, 41)):
        for _ in range(5):
            a = rng.random((H, W)) < 0.4
            a[0, 0] = True
            b = rng.random((H, W)) < 0.3
            A = set(zip(*np.nonzero(a)))
            B = set(zip(*np.nonzero(b)))
            pa, pb = synth.pack_bits(a), synth.pack_bits(b)
            want = (len(A | B) - len(A & B)) / len(A)
            assert oracle_mod.fitness(pb, pa, W, H) == want
            assert oracle_mod.fitness(pa, pa, W, H) == 0.0
            assert oracle_mod.fitness(np.zeros_like(pa), pa, W, H) == 1.0
            assert oracle_mod.fitness(pb, pa, W, H) == len(A ^ B) / len(A)


def test_fitness_empty_reference_is_nan(oracle_mod):
    z = np.zeros((3, 1), dtype=np.uint32)
    assert np.isnan(oracle_mod.fitness(z, z, 5, 3))


GA = dict(elite=2, pm0=0.2, h=1.0, lo=-30.0, hi=30.0, generations=50, ga_seed=0x6A00001)


def _pop(P, G, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-30, 30, size=(P, G))


def test_ga_elitism_and_mean(oracle_mod):
    P, G, R = 64, 5, 20
    pop = _pop(P, G, 1)
    fit = np.random.default_rng(2).random((P, R))
    new, mean = oracle_mod.ga_step(pop, fit, gen=3, **GA)
    assert np.array_equal(mean, np.array([sum(fit[i, r] for r in range(R)) / R for i in range(P)]))
    order = sorted(range(P), key=lambda i: (mean[i], i))
    assert np.array_equal(new[0], pop[order[0]])
    assert np.array_equal(new[1], pop[order[1]])


def test_ga_tournament_and_crossover(oracle_mod):
    # G = 2: the cut is always 1, so gene 0 identifies the tournament winner
    P, G, R = 32, 2, 3
    pop = np.stack([np.arange(P, dtype=float), np.arange(P, dtype=float) + 100], axis=1)
    fit = np.random.default_rng(4).random((P, R))
    cfg = dict(GA, pm0=0.0)
    new, mean = oracle_mod.ga_step(pop, fit, gen=7, **cfg)
    key = [cfg["ga_seed"] & 0xFFFFFFFF, cfg["ga_seed"] >> 32]
    for i in range(2, P):
        w = int(new[i, 0])
        out = oracle_mod.philox([7, i, 0, 0], key)
        a = (int(out[0]) * P) >> 32
        b = (int(out[1]) * P) >> 32
        best = a if (mean[a], a) <= (mean[b], b) else b
        assert w == best
    # crossover swapped gene 1 within each non-elite pair
    for k in range((P - 2) // 2):
        u, v = new[2 + 2 * k], new[3 + 2 * k]
        assert u[1] == int(v[0]) + 100 and v[1] == int(u[0]) + 100


def test_ga_crossover_tails(oracle_mod):
    P, G, R = 16, 5, 2
    pop = _pop(P, G, 5)
    fit = np.random.default_rng(6).random((P, R))
    cfg = dict(GA, pm0=0.0)
    new, _ = oracle_mod.ga_step(pop, fit, gen=0, **cfg)
    rows = {tuple(r) for r in pop}
    for k in range((P - 2) // 2):
        u, v = new[2 + 2 * k], new[3 + 2 * k]
        # some cut c in 1..G-1 makes (u[:c]+v[c:]) and (v[:c]+u[c:]) parents
        ok = False
        for c in range(1, G):
            pu = tuple(np.concatenate([u[:c], v[c:]]))
            pv = tuple(np.concatenate([v[:c], u[c:]]))
            if pu in rows and pv in rows:
                ok = True
        assert ok


def test_ga_mutation_schedule(oracle_mod):
    P, G, R = 256, 5, 1
    pop = _pop(P, G, 7) * 0.5
    fit = np.zeros((P, R))  # all ties: tournament keeps the lower index
    cfg = dict(GA, pm0=0.5)
    for gen in (0, 25, 49):
        base, _ = oracle_mod.ga_step(pop, fit, gen=gen, **dict(cfg, pm0=0.0))
        new, _ = oracle_mod.ga_step(pop, fit, gen=gen, **cfg)
        diff = np.abs(new[2:] - base[2:])
        assert np.all(diff <= cfg["h"] + 1e-12)
        rate = np.mean(diff > 0)
        pm = 0.5 * (1 - gen / 50)
        n = diff.size
        assert abs(rate - pm) <= 5 * np.sqrt(pm * (1 - pm) / n) + 1e-9
        assert np.all(new >= -30) and np.all(new <= 30)


def test_ga_clamps(oracle_mod):
    P, G = 8, 3
    pop = np.full((P, G), 29.9)
    fit = np.zeros((P, 1))
    new, _ = oracle_mod.ga_step(pop, fit, gen=0, **dict(GA, pm0=1.0, h=5.0))
    assert np.all(new <= 30.0) and np.any(new == 30.0)


BOX7 = dict(lo=[-30, -30, -30, -30, -30, 0, 0], hi=[30, 30, 30, 30, 30, 127, 95],
            h=[1.0, 1.0, 0.0, 1.0, 1.0, 8.0, 4.0])


def test_ga_per_gene_boxes(oracle_mod):
    # 7 genes (beta[5], ignition x, y): each gene mutates by at most its own
    # width and stays in its own box; a gene of width 0 never mutates
    P, G, R = 256, 7, 1
    rng = np.random.default_rng(11)
    pop = np.concatenate([rng.uniform(-30, 30, (P, 5)), rng.uniform(0, 127, (P, 1)),
                          rng.uniform(0, 95, (P, 1))], axis=1)
    fit = np.zeros((P, R))
    cfg = dict(GA, **BOX7, pm0=0.9)
    base, _ = oracle_mod.ga_step(pop, fit, gen=0, **dict(cfg, pm0=0.0))
    new, _ = oracle_mod.ga_step(pop, fit, gen=0, **cfg)
    diff = np.abs(new[2:] - base[2:])
    for j in range(G):
        lo, hi, h = BOX7["lo"][j], BOX7["hi"][j], BOX7["h"][j]
        assert np.all(new[:, j] >= lo) and np.all(new[:, j] <= hi), j
        assert np.all(diff[:, j] <= h + 1e-12), j
        if h == 0.0:
            assert np.all(diff[:, j] == 0.0)
        else:
            assert np.mean(diff[:, j] > 0) > 0.7, j
    # the wide coordinate genes really use their width
    assert diff[:, 5].max() > 4.0 and diff[:, 6].max() > 2.0
    # a gene pinned by its box (lo == hi) is constant
    box = dict(BOX7, lo=[-30, -30, 1.5, -30, -30, 0, 0], hi=[30, 30, 1.5, 30, 30, 127, 95],
               h=[1.0] * 7)
    p2 = pop.copy()
    p2[:, 2] = 1.5
    new2, _ = oracle_mod.ga_step(p2, fit, gen=0, **dict(GA, **box, pm0=1.0))
    assert np.all(new2[:, 2] == 1.5)


def test_ignition_cell_reading(oracle_mod):
    W, H = 128, 96
    cases = {(2.5, 3.49): (3, 3), (2.49, 3.5): (2, 4), (-0.5, -0.49): (0, 0),
             (-0.51, -7.0): (0, 0), (127.49, 95.49): (127, 95), (127.5, 95.5): (127, 95),
             (400.0, 1e9): (127, 95), (0.0, 0.0): (0, 0), (63.0, 47.0): (63, 47)}
    for (gx, gy), want in cases.items():
        assert oracle_mod.ignition_cell(gx, gy, W, H) == want, (gx, gy)


def test_ga_converges_on_smooth_objective(oracle_mod):
    # the operators, iterated, minimise a smooth bowl (a weak end-to-end check)
    rng = np.random.default_rng(8)
    P, G = 64, 5
    pop = rng.uniform(-30, 30, size=(P, G))
    target = np.array([-1.0, 2.0, 0.5, 3.0, -2.0])
    for gen in range(50):
        fit = np.linalg.norm(pop - target, axis=1)[:, None]
        pop, _ = oracle_mod.ga_step(pop, fit, gen=gen, **GA)
    best = np.min(np.linalg.norm(pop - target, axis=1))
    assert best < 3.0


def test_ensemble_and_scan(oracle_mod):
    params = np.array([[0.0, 1.0], [2.0, 3.0], [4.0, 5.0], [6.0, 7.0]])
    deltas = np.array([0.5, 0.1, 0.2, 0.9])
    e = oracle_mod.ensemble(params, deltas, cutoff=0.3)
    assert e["best_index"] == 1 and e["n_accepted"] == 2
    assert np.allclose(e["accepted_mean"], [3.0, 4.0])
    assert np.allclose(e["spread"], [np.sqrt(2.0), np.sqrt(2.0)])
    d = np.array([[0.1, 0.5, 0.2, 0.9], [0.8, 0.7, 0.9, 0.6], [0.2, 0.25, 0.1, 0.29]])
    s = oracle_mod.scan_reduce(d, cutoff=0.3)
    assert np.allclose(s["accept"], [0.5, 0.0, 1.0])
    assert np.allclose(s["posterior"], [1 / 3, 0, 2 / 3])
    assert np.allclose(s["mean"], d.mean(axis=1))
    assert np.allclose(s["sd"], d.std(axis=1, ddof=1))
    s2 = oracle_mod.scan_reduce(d + 1.0, cutoff=0.3, tau=0.1)
    w = np.exp(-(d.mean(axis=1) + 1.0) / 0.1)
    assert np.allclose(s2["posterior"], w / w.sum())
