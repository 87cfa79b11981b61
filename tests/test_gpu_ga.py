"""GPU parity of the fitting operators against the oracle (through the C ABI):
the Appendix B GA step (bit-exact, exact IEEE operations only) and its
several-offspring-set form, a whole
captured-graph GA run against an oracle-driven GA loop (bit-exact), the plain
per-simulation GA against the batched one (identical histories), and the
ensemble / ignition-scan reductions (exact counts and indices, binary64 sums
within 1e-12 relative)."""
import numpy as np
import pytest

import oracle
from gpu_util import SEED, oracle_target, say
from paper_1701_03549_amd import synth

pytestmark = pytest.mark.gpu
GA_SEED = 0x6A00001


@pytest.fixture(scope="module")
def g():
    import torch
    from paper_1701_03549_amd import fire
    assert torch.cuda.is_available()
    ctx = fire.FireGPU(0)
    yield ctx
    ctx.close()


@pytest.mark.parametrize("P,G,R,elite", [(64, 5, 20, 2), (17, 7, 3, 1), (256, 5, 1, 0), (2, 2, 1, 2)])
def test_ga_step_bit_exact(g, P, G, R, elite):
    import torch
    say(f"ga_step P={P} G={G}")
    rng = np.random.default_rng(P * G)
    pop = rng.uniform(-30, 30, size=(P, G))
    cfg = g.ga_cfg(elite=elite, pm0=0.3, mut_h=1.5, lo=-30, hi=30, generations=10)
    d_pop = torch.from_numpy(pop.copy()).cuda()
    for gen in range(3):
        fit = rng.random((P, R))
        fit[1] = fit[0]  # a tie
        d_fit = torch.from_numpy(fit).cuda()
        mean = torch.empty(P, dtype=torch.float64, device="cuda")
        g.ga_step(d_pop, d_fit, cfg, gen, GA_SEED, mean_fit=mean)
        g.sync()
        want, want_mean = oracle.ga_step(pop, fit, elite=elite, pm0=0.3, h=1.5, lo=-30, hi=30,
                                         gen=gen, generations=10, ga_seed=GA_SEED)
        assert np.array_equal(d_pop.cpu().numpy(), want), gen
        assert np.array_equal(mean.cpu().numpy(), want_mean), gen
        pop = want


@pytest.mark.parametrize("P,G,R,elite,S", [(64, 5, 20, 2, 8), (17, 7, 3, 1, 3), (2, 2, 1, 0, 1)])
def test_ga_offspring_sets_bit_exact(g, P, G, R, elite, S):
    """fire_ga_offspring: set o equals the oracle's GA step under seed
    ga_seed + o * step (mod 2^64, here wrapping past 2^64), the parents stay
    unchanged, and an output overlapping the parents is refused."""
    import torch
    from paper_1701_03549_amd import fire
    say(f"ga_offspring P={P} G={G} S={S}")
    rng = np.random.default_rng(P * G + S)
    pop = rng.uniform(-30, 30, size=(P, G))
    fit = rng.random((P, R))
    fit[-1] = fit[0]  # a tie
    cfg = g.ga_cfg(elite=elite, pm0=0.3, mut_h=1.5, lo=-30, hi=30, generations=10)
    d_pop = torch.from_numpy(pop.copy()).cuda()
    d_fit = torch.from_numpy(fit).cuda()
    out = torch.zeros((S, P, G), dtype=torch.float64, device="cuda")
    seed, step = 2 ** 64 - 3, 0x9E3779B97F4A7C15
    g.ga_offspring(d_pop, d_fit, cfg, 4, seed, step, out)
    g.sync()
    assert np.array_equal(d_pop.cpu().numpy(), pop)
    got = out.cpu().numpy()
    for o in range(S):
        want, _ = oracle.ga_step(pop, fit, elite=elite, pm0=0.3, h=1.5, lo=-30, hi=30, gen=4,
                                 generations=10, ga_seed=(seed + o * step) % 2 ** 64)
        assert np.array_equal(got[o], want), o
    with pytest.raises(fire.FireError):
        whole = torch.zeros((S + 1, P, G), dtype=torch.float64, device="cuda")
        g.ga_offspring(whole[S], d_fit, cfg, 4, seed, step, whole[1:])


def _ga_fixture(g):
    W = H = 64
    ls = synth.make_landscape(W, H, 101)
    c = synth.nearest_burnable(ls["veg"], 32, 32)
    ref, _ = oracle_target(ls, (-0.9, -0.5, 0.3, 0.8, 1.0), c, lo=0.02, hi=0.5)
    lid = g.load_landscape(ls)
    tid = g.load_target(lid, ref)
    return ls, c, ref, lid, tid


def test_ga_run_matches_oracle_loop(g):
    from paper_1701_03549_amd import ga
    ls, c, ref, lid, tid = _ga_fixture(g)
    P, R, gens = 16, 4, 3
    rng = np.random.default_rng(5)
    pop0 = rng.normal(0, 1.0, size=(P, 5))
    pop0[:, 0] -= 1.0
    say("ga_run vs oracle loop")
    hp, hf = ga.run_batched(g, lid, tid, c, pop0, R=R, generations=gens, sim_seed=SEED,
                            ga_seed=GA_SEED)
    hp, hf = hp.cpu().numpy(), hf.cpu().numpy()
    pop = pop0.copy()
    H, W = ls["veg"].shape
    for gen in range(gens):
        assert np.array_equal(hp[gen], pop), gen
        fit = np.empty((P, R))
        for i in range(P):
            T = oracle.thresholds(ls, pop[i])
            for r in range(R):
                o = oracle.simulate(ls["veg"], T, c, (gen * P + i) * R + r, SEED)
                fit[i, r] = oracle.fitness(o["map"], ref, W, H)
        assert np.array_equal(hf[gen], fit), gen
        pop, _ = oracle.ga_step(pop, fit, elite=2, pm0=0.2, h=1.0, lo=-30, hi=30, gen=gen,
                                generations=gens, ga_seed=GA_SEED)
    g.free_landscape(lid)


def test_ga_plain_equals_batched(g):
    import torch
    from paper_1701_03549_amd import ga
    ls, c, ref, lid, tid = _ga_fixture(g)
    rng = np.random.default_rng(6)
    pop0 = rng.uniform(-3, 3, size=(8, 5))
    say("ga plain vs batched")
    hb = ga.run_batched(g, lid, tid, c, pop0, R=3, generations=4, sim_seed=SEED, ga_seed=GA_SEED)
    hpl = ga.run_plain(g, lid, tid, c, pop0, R=3, generations=4, sim_seed=SEED, ga_seed=GA_SEED)
    assert torch.equal(hb[0], hpl[0]) and torch.equal(hb[1], hpl[1])
    rec = ga.recovered(g, hb, cutoff=0.3)
    assert len(rec["best_params"]) == 5
    g.free_landscape(lid)


def test_ensemble_matches_oracle(g):
    import torch
    rng = np.random.default_rng(11)
    N, G, R = 300, 5, 7
    params = rng.normal(size=(N, G))
    deltas = rng.random((N, R))
    deltas[5, 3] = deltas[9, 0] = deltas.min() / 2  # tie for the best: first wins
    say("ensemble")
    e = g.ensemble(torch.from_numpy(params).cuda(), torch.from_numpy(deltas).cuda(), 0.3)
    g.sync()
    want = oracle.ensemble(np.repeat(params, R, axis=0), deltas.reshape(-1), 0.3)
    assert int(e["best_individual"].item()) == want["best_index"] // R == 5
    assert int(e["n_accepted"].item()) == want["n_accepted"]
    assert np.allclose(e["mean"].cpu().numpy(), want["accepted_mean"], rtol=1e-12, atol=1e-14)
    assert np.allclose(e["sd"].cpu().numpy(), want["spread"], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("shift", [0.0, 5.0])
def test_scan_reduce_matches_oracle(g, shift):
    import torch
    rng = np.random.default_rng(12)
    d = rng.random((256, 32)) * 1.2 + shift
    say(f"scan_reduce shift={shift}")
    s = g.scan_reduce(torch.from_numpy(d).cuda(), 0.3, tau=0.1)
    g.sync()
    want = oracle.scan_reduce(d, 0.3, tau=0.1)
    assert np.array_equal(s["accept"].cpu().numpy(), want["accept"])
    for k in ("mean", "sd", "posterior"):
        assert np.allclose(s[k].cpu().numpy(), want[k], rtol=1e-12, atol=1e-15), k
    assert abs(s["posterior"].sum().item() - 1.0) < 1e-12


def test_ignition_scan_matches_oracle(g):
    """Candidate scan on a 96x80 lattice with a smooth wind field: every
    replicate's Eq. 2 value bit-exact, the reduction within 1e-12."""
    from paper_1701_03549_amd import scan
    W, H = 96, 80
    ls = synth.make_landscape(W, H, 103, wind="smooth")
    beta = (-0.9, -0.5, 0.3, 0.8, 1.0)
    c = synth.nearest_burnable(ls["veg"], W // 2, H // 2)
    ref, _ = oracle_target(ls, beta, c, lo=0.02, hi=0.6)
    lid = g.load_landscape(ls)
    tid = g.load_target(lid, ref)
    cands = scan.candidate_grid(c, W, H, spacing=3, half=3)
    R = 6
    say("ignition scan")
    out = scan.run_scan(g, lid, tid, beta, cands, R=R, seed=SEED, cutoff=0.6)
    g.sync()
    T = oracle.thresholds(ls, beta)
    want = np.empty((len(cands), R))
    for k, (x, y) in enumerate(cands):
        for r in range(R):
            o = oracle.simulate(ls["veg"], T, (int(x), int(y)), k * R + r, SEED)
            want[k, r] = oracle.fitness(o["map"], ref, W, H)
    assert np.array_equal(out["deltas"].cpu().numpy(), want)
    red = oracle.scan_reduce(want, 0.6, tau=0.1)
    assert np.array_equal(out["accept"].cpu().numpy(), red["accept"])
    for k in ("mean", "sd", "posterior"):
        assert np.allclose(out[k].cpu().numpy(), red[k], rtol=1e-12, atol=1e-15), k
    # the true ignition is among the best-scoring candidates
    centre_k = int(np.argmin(np.abs(cands - np.array(c)).sum(axis=1)))
    assert out["mean"].cpu().numpy()[centre_k] <= np.sort(red["mean"])[len(cands) // 2]
    g.free_landscape(lid)


def test_monte_carlo_fit_matches_oracle(g):
    """Appendix C brute-force fit: every sampled vector's Eq. 2 value
    bit-exact against the oracle, ensemble statistics as the oracle's."""
    from paper_1701_03549_amd import mc
    ls, c, ref, lid, tid = _ga_fixture(g)
    H, W = ls["veg"].shape
    n = 300
    say("monte carlo fit")
    out = mc.run_mc(g, lid, tid, c, n, seed=77, sim_seed=SEED, box=(-3.0, 3.0), cutoff=1.0)
    params = out["params"]
    want = np.empty(n)
    for i in range(n):
        T = oracle.thresholds(ls, params[i])
        o = oracle.simulate(ls["veg"], T, c, i, SEED)
        want[i] = oracle.fitness(o["map"], ref, W, H)
    assert np.array_equal(out["deltas"].cpu().numpy(), want)
    e = oracle.ensemble(params, want, 1.0)
    assert out["best_index"] == e["best_index"] and out["n_accepted"] == e["n_accepted"]
    assert np.allclose(out["accepted_mean"], e["accepted_mean"], rtol=1e-12)
    assert np.allclose(out["accepted_sd"], e["spread"], rtol=1e-12)
    g.free_landscape(lid)
