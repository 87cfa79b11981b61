"""GPU parity of the per-cell ablation path (fire_run_dense: one thread per
cell, one uniform per candidate target per step, the paper's kernel form)
against the oracle's per-target simulation: maps, burnt, step and draw
counts and Eq. 2 bit-exact; and the same law of the burnt size as the
frontier path (fire_run), which draws per-edge coins."""
import numpy as np
import pytest
from scipy import stats

import oracle
from gpu_util import BETA_STAR, SEED, oracle_target, say
from paper_1701_03549_amd import synth

pytestmark = pytest.mark.gpu
BETA_SUB = (-0.9, -0.5, 0.3, 0.8, 1.0)


@pytest.fixture(scope="module")
def g():
    import torch
    from paper_1701_03549_amd import fire
    assert torch.cuda.is_available()
    ctx = fire.FireGPU(0)
    yield ctx
    ctx.close()


def _check(ls, betas, r, m, sims, ref=None):
    veg = ls["veg"]
    H, W = veg.shape
    Ts = {}
    for i, sd in enumerate(sims):
        p = int(sd["param_index"])
        if p not in Ts:
            Ts[p] = oracle.thresholds(ls, betas[p])
        o = oracle.simulate_dense(veg, Ts[p], (int(sd["ign_x"]), int(sd["ign_y"])),
                                  int(sd["sim_index"]), SEED, int(sd["max_steps"]))
        got = (int(r["burnt"][i]), int(r["steps"][i]), int(r["trials"][i]))
        assert got == (o["burnt"], o["steps"], o["trials"]), (i, got)
        assert np.array_equal(m[i][: H * ((W + 31) // 32)].reshape(H, -1), o["map"]), i
        if ref is not None:
            want = oracle.fitness(o["map"], ref, W, H) if o["burnt"] else 1.0
            assert r["fitness"][i] == want, i


def test_dense_matches_oracle_64(g):
    from paper_1701_03549_amd import fire
    W = H = 64
    ls = synth.make_landscape(W, H, 101)
    c = synth.nearest_burnable(ls["veg"], 32, 32)
    betas = np.array([BETA_SUB, (0.0, 0.0, 0.0, 0.0, 0.0)])
    ref, _ = oracle_target(ls, betas[0], c, lo=0.02, hi=0.5)
    lid = g.load_landscape(ls)
    tid = g.load_target(lid, ref)
    sims = fire.make_sims(40, lid, tid, c, param_index=np.arange(40) % 2)
    sims["max_steps"][::9] = 4
    zy, zx = np.nonzero(ls["veg"] == 0)
    sims["ign_x"][5], sims["ign_y"][5] = zx[0], zy[0]  # non-burnable ignition
    say("dense 64x64")
    res, maps = g.run_dense(betas, sims, SEED, want_maps=True)
    g.sync()
    r = fire.results_to_numpy(res)
    m = maps.cpu().numpy().view(np.uint32)
    _check(ls, betas, r, m, sims, ref)
    assert r["burnt"][5] == 0 and r["fitness"][5] == 1.0
    g.free_landscape(lid)


@pytest.mark.parametrize("W,H", [(1, 1), (33, 1), (31, 33), (65, 7), (100, 67)])
def test_dense_ragged(g, W, H):
    from paper_1701_03549_amd import fire
    ls = synth.random_small_landscape(W, H, seed=W * 3 + H, p_blocked=0.1)
    ls["veg"][0, 0] = 2
    betas = np.array([(0.5, -0.2, 0.3, 0.5, 1.0)])
    lid = g.load_landscape(ls)
    rng = np.random.default_rng(W + H)
    ign = np.stack([rng.integers(0, W, 12), rng.integers(0, H, 12)], axis=1)
    sims = fire.make_sims(12, lid, -1, ign)
    say(f"dense ragged {W}x{H}")
    res, maps = g.run_dense(betas, sims, SEED, want_maps=True)
    g.sync()
    _check(ls, betas, fire.results_to_numpy(res), maps.cpu().numpy().view(np.uint32), sims)
    g.free_landscape(lid)


def test_dense_same_law_as_frontier(g):
    from paper_1701_03549_amd import fire
    W = H = 64
    ls = synth.make_landscape(W, H, 101)
    c = synth.nearest_burnable(ls["veg"], 32, 32)
    lid = g.load_landscape(ls)
    n = 600
    sims = fire.make_sims(n, lid, -1, c)
    say("dense vs frontier law")
    rd, _ = g.run_dense(np.array([BETA_SUB]), sims, SEED)
    rf, _ = g.run(np.array([BETA_SUB]), sims, SEED + 1)
    g.sync()
    a = fire.results_to_numpy(rd)["burnt"].astype(float)
    b = fire.results_to_numpy(rf)["burnt"].astype(float)
    assert stats.ks_2samp(a, b).pvalue > 1e-4
    assert stats.mannwhitneyu(a, b).pvalue > 1e-4
    g.free_landscape(lid)


def test_dense_512_sampled(g):
    from paper_1701_03549_amd import fire
    W = H = 512
    ls = synth.make_landscape(W, H, 102)
    c = synth.ignition_site(ls)
    lid = g.load_landscape(ls)
    sims = fire.make_sims(4, lid, -1, c, sim_index=np.arange(4, dtype=np.uint32) * 97)
    say("dense 512x512")
    res, maps = g.run_dense(np.array([BETA_STAR]), sims, SEED, want_maps=True)
    g.sync()
    _check(ls, np.array([BETA_STAR]), fire.results_to_numpy(res),
           maps.cpu().numpy().view(np.uint32), sims)
    g.free_landscape(lid)


def test_dense_rejects_turn_off_times(g):
    from paper_1701_03549_amd import fire
    ls = synth.make_landscape(16, 16, 1)
    lid = g.load_landscape(ls)
    bs = np.full(256, 2, dtype=np.uint8)
    g.set_burn_steps(lid, bs)
    with pytest.raises(fire.FireError):
        g.run_dense(np.array([BETA_SUB]), fire.make_sims(1, lid, -1, (8, 8)), SEED)
    g.free_landscape(lid)
