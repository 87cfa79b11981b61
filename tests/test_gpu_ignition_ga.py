"""GPU parity of the 7-parameter search of Appendix B (beta[5] and the
ignition point) against the oracle, through the C ABI: the GA step with a
box and mutation width per gene (bit-exact), the descriptors built from the
ignition genes (exact cells: nearest, halves up, clamped to the lattice),
and a whole captured-graph run against an oracle-driven loop (bit-exact
populations and fitness values, including individuals whose ignition lands
on a non-burnable cell)."""
import numpy as np
import pytest

import oracle
from gpu_util import SEED, oracle_target, say
from paper_1701_03549_amd import synth

pytestmark = pytest.mark.gpu
GA_SEED = 0x6A00007
LO = [-30.0] * 5 + [0.0, 0.0]


@pytest.fixture(scope="module")
def g():
    import torch
    from paper_1701_03549_amd import fire
    assert torch.cuda.is_available()
    ctx = fire.FireGPU(0)
    yield ctx
    ctx.close()


@pytest.mark.parametrize("P,R,elite", [(48, 5, 2), (33, 1, 0), (600, 2, 4)])
def test_ga_step_genes_bit_exact(g, P, R, elite):
    import torch
    W, H = 200, 120
    lo, hi, h = LO, [30.0] * 5 + [W - 1.0, H - 1.0], [1.0, 0.5, 2.0, 1.0, 0.0, 9.0, 5.0]
    rng = np.random.default_rng(P)
    pop = np.concatenate([rng.uniform(-30, 30, (P, 5)), rng.uniform(0, W - 1, (P, 1)),
                          rng.uniform(0, H - 1, (P, 1))], axis=1)
    say(f"ga_step_genes P={P} R={R}")
    d_pop = torch.from_numpy(pop.copy()).cuda()
    for gen in range(3):
        fit = rng.random((P, R))
        d_fit = torch.from_numpy(fit).cuda()
        mean = torch.empty(P, dtype=torch.float64, device="cuda")
        g.ga_step_genes(d_pop, d_fit, elite=elite, pm0=0.6, lo=lo, hi=hi, h=h, generations=5,
                        gen=gen, ga_seed=GA_SEED, mean_fit=mean)
        g.sync()
        want, want_mean = oracle.ga_step(pop, fit, elite=elite, pm0=0.6, h=h, lo=lo, hi=hi,
                                         gen=gen, generations=5, ga_seed=GA_SEED)
        assert np.array_equal(d_pop.cpu().numpy(), want), gen
        assert np.array_equal(mean.cpu().numpy(), want_mean), gen
        pop = want


def test_ga_step_genes_rejects_oversized_population(g):
    import torch
    from paper_1701_03549_amd import fire
    P, G = 1024, 16  # 8*(P + 2PG) + 4P bytes of LDS: more than one workgroup holds
    pop = torch.zeros((P, G), dtype=torch.float64, device="cuda")
    fit = torch.zeros((P, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(fire.FireError):
        g.ga_step_genes(pop, fit, elite=2, pm0=0.1, lo=-1, hi=1, h=0.1, generations=2, gen=0,
                        ga_seed=1)


def test_sims_from_pop_cells(g):
    import torch
    from paper_1701_03549_amd import fire
    W, H = 96, 64
    ls = synth.make_landscape(W, H, 104)
    lid = g.load_landscape(ls)
    xy = [(2.5, 3.49), (2.49, 3.5), (-0.5, -0.49), (-0.51, -7.0), (95.49, 63.49), (95.5, 63.5),
          (400.0, 1e9), (0.0, 0.0), (47.0, 31.0), (10.25, 60.75)]
    P, R, gen = len(xy), 3, 4
    rng = np.random.default_rng(3)
    pop = np.concatenate([rng.normal(size=(P, 5)), np.array(xy)], axis=1)
    say("sims_from_pop")
    sims, betas = g.ga_sims_from_pop(torch.from_numpy(pop).cuda(), R, lid, -1, gen)
    g.sync()
    s = sims.cpu().numpy().reshape(-1).view(fire.SIM_DTYPE)
    assert np.array_equal(betas.cpu().numpy(), pop[:, :5])
    for i in range(P):
        cx, cy = oracle.ignition_cell(pop[i, 5], pop[i, 6], W, H)
        for r in range(R):
            d = s[i * R + r]
            assert (int(d["ign_x"]), int(d["ign_y"])) == (cx, cy), (i, xy[i])
            assert int(d["param_index"]) == i and int(d["landscape_id"]) == lid
            assert int(d["target_id"]) == -1
            assert int(d["sim_index"]) == (gen * P + i) * R + r
            assert int(d["max_steps"]) == 0xFFFFFFFF
    g.free_landscape(lid)


def test_ga_run_ignition_matches_oracle_loop(g):
    import torch
    from paper_1701_03549_amd import ga
    W = H = 64
    ls = synth.make_landscape(W, H, 101)
    c = synth.nearest_burnable(ls["veg"], 32, 32)
    ref, _ = oracle_target(ls, (-0.9, -0.5, 0.3, 0.8, 1.0), c, lo=0.02, hi=0.5)
    lid = g.load_landscape(ls)
    tid = g.load_target(lid, ref)
    P, R, gens = 16, 3, 3
    pop0 = ga.initial_population_ignition(ref, W, H, P, seed=9, prior_sd=1.0)
    pop0[:, 0] -= 1.0
    pop0[3, 5:] = (-3.0, 70.2)  # clamped to the border
    veg = ls["veg"]
    nb = np.argwhere(veg == 0)
    if nb.size:
        pop0[4, 5], pop0[4, 6] = nb[0][1], nb[0][0]  # a non-burnable ignition
    lo, hi, h = ga.ignition_box(W, H, xy_h=6.0)
    say("ga_run_ignition vs oracle loop")
    hp, hf = ga.run_ignition(g, lid, tid, pop0, R=R, generations=gens, sim_seed=SEED,
                             ga_seed=GA_SEED, box=(lo, hi, h))
    hp, hf = hp.cpu().numpy(), hf.cpu().numpy()
    pop = pop0.copy()
    for gen in range(gens):
        assert np.array_equal(hp[gen], pop), gen
        fit = np.empty((P, R))
        for i in range(P):
            T = oracle.thresholds(ls, pop[i, :5])
            cell = oracle.ignition_cell(pop[i, 5], pop[i, 6], W, H)
            for r in range(R):
                o = oracle.simulate(veg, T, cell, (gen * P + i) * R + r, SEED)
                fit[i, r] = oracle.fitness(o["map"], ref, W, H) if o["burnt"] else 1.0
        assert np.array_equal(hf[gen], fit), gen
        pop, _ = oracle.ga_step(pop, fit, elite=2, pm0=0.2, h=h, lo=lo, hi=hi, gen=gen,
                                generations=gens, ga_seed=GA_SEED)
    rec = ga.recovered(g, (torch.from_numpy(hp).cuda(), torch.from_numpy(hf).cuda()),
                       cutoff=1.5)
    assert len(rec["accepted_mean"]) == 7
    g.free_landscape(lid)
