"""Host-side logic of the drivers (no GPU): the 7-gene GA's boxes and initial
population, the Monte Carlo sampler, the ignition-scan candidate grid and
the autotuner's candidate schedules."""
import numpy as np

from paper_1701_03549_amd import synth


def test_ignition_box_and_initial_population():
    from paper_1701_03549_amd import ga
    W, H = 96, 64
    lo, hi, h = ga.ignition_box(W, H)
    assert lo == [-30.0] * 5 + [0.0, 0.0] and hi == [30.0] * 5 + [95.0, 63.0]
    assert h[:5] == [1.0] * 5 and h[5] == h[6] == 3.0
    ref = np.zeros((H, W), dtype=bool)
    ref[10:20, 30:45] = True
    bits = synth.pack_bits(ref)
    pop = ga.initial_population_ignition(bits, W, H, 200, seed=3)
    assert pop.shape == (200, 7)
    assert np.all(ref[pop[:, 6].astype(int), pop[:, 5].astype(int)])  # burnt cells only
    assert np.all(pop[:, 5] == np.round(pop[:, 5])) and np.all(np.abs(pop[:, :5]) <= 30)
    assert len({(int(a), int(b)) for a, b in pop[:, 5:]}) > 50  # spread over the scar
    u = ga.initial_population_ignition(bits, W, H, 500, seed=4, prior_sd=None)
    assert u[:, :5].min() < -25 and u[:, :5].max() > 25  # uniform over the box


def test_monte_carlo_sampler_is_uniform_over_the_box():
    from paper_1701_03549_amd import mc
    p = mc.sample_params(20000, seed=1)
    assert p.shape == (20000, 5) and p.min() >= -30 and p.max() <= 30
    assert np.allclose(p.mean(axis=0), 0, atol=0.5)
    assert np.allclose(p.std(axis=0), 60 / np.sqrt(12), rtol=0.02)
    assert np.array_equal(p, mc.sample_params(20000, seed=1))


def test_scan_candidate_grid():
    from paper_1701_03549_amd import scan
    c = scan.candidate_grid((256, 259), 1024, 1024, spacing=4, half=8)
    assert len(c) == 256
    assert tuple(c.min(axis=0)) >= (0, 0) and tuple(c.max(axis=0)) < (1024, 1024)
    assert any((c == np.array([256, 259])).all(axis=1)) or \
        np.min(np.abs(c - np.array([256, 259])).sum(axis=1)) <= 4


def test_autotune_candidates():
    from paper_1701_03549_amd import autotune
    cs = list(autotune.candidates(True, side=512))
    wins = {c["window"] for c in cs}
    assert wins == {0, 128, 256, 384}
    assert {c["table_mode"] for c in cs} == {0, 1}
    assert all(c["threads"] in (128, 256, 512, 1024) for c in cs if c["wave"] == 0)
    assert all(c["wave"] == 0 for c in cs)
    assert not any(c["threads"] == 1024 and c["window"] > 0 for c in cs)
    assert {c["window"] for c in autotune.candidates(False, side=64)} == {0}


def test_load_balance_of_sim_clocks():
    from paper_1701_03549_amd.timing import load_balance
    # 4 slots, 8 simulations of 10 ticks packed back to back: no idle slot
    t = np.array([[100 + 10 * (i // 4), 110 + 10 * (i // 4)] for i in range(8)])
    lb = load_balance(t, hz=1.0)
    assert lb["slots"] == 4 and lb["span_ms"] == 20e3 and lb["efficiency"] == 1.0
    assert lb["tail_ms"] == 10e3 and lb["drain_ms"] == 0.0 and lb["sims"] == 8
    # 2 slots: one holds a 30-tick and then a 50-tick simulation, the other
    # four of 10 ticks; the straggler runs alone for its last 40 ticks
    t = np.array([[1000, 1030], [1000, 1010], [1010, 1020], [1020, 1030], [1030, 1080],
                  [1030, 1040]])
    lb = load_balance(t, hz=1.0)
    assert lb["slots"] == 2 and lb["span_ms"] == 80e3
    assert abs(lb["efficiency"] - 120 / (2 * 80)) < 1e-12
    assert lb["tail_ms"] == 50e3 and lb["drain_ms"] == 40e3 and lb["longest_sim_ms"] == 50e3
    # incomplete pairs (never taken, or not finished) are left out
    t = np.array([[0, 0], [5, 3], [1, 4]])  # never taken, no result, complete
    assert load_balance(t, hz=1.0)["sims"] == 1
