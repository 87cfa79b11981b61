"""GPU parity of the turn-off-time model (burning cells stay active for a
number of steps set by their vegetation) against the oracle, through the C
ABI: burn maps, burnt, step and trial counts and Eq. 2 bit-exact, in table
and per-trial threshold modes, under schedules whose tiny LDS queues force
the spilled entries and their remaining-life bytes through global memory,
with landscapes with and without turn-off times in one call, and at 512x512
in the benchmark's launch shape (sampled)."""
import numpy as np
import pytest

import oracle
from gpu_util import BETA_STAR, SEED, compare_with_oracle, oracle_target, say
from paper_1701_03549_amd import synth

pytestmark = pytest.mark.gpu
BETA_SUB = (-1.6, -0.5, 0.3, 0.8, 1.0)


@pytest.fixture(scope="module")
def g():
    import torch
    from paper_1701_03549_amd import fire
    assert torch.cuda.is_available()
    ctx = fire.FireGPU(0)
    yield ctx
    ctx.close()


def _steps(ls, rng, hi=4):
    b = np.ones(256, dtype=np.uint8)
    for v in np.unique(ls["veg"]):
        if v:
            b[v] = rng.integers(1, hi + 1)
    return b


def _np(res, maps):
    from paper_1701_03549_amd import fire
    return fire.results_to_numpy(res), None if maps is None else maps.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("mode", ["table", "onthefly"])
def test_turn_off_times_match_oracle(g, mode):
    from paper_1701_03549_amd import fire
    W = H = 64
    ls = synth.make_landscape(W, H, 101)
    c = synth.nearest_burnable(ls["veg"], 32, 32)
    bs = _steps(ls, np.random.default_rng(1))
    bs[ls["veg"][c[1], c[0]]] = 3
    betas = np.array([BETA_SUB, (-2.5, 0.0, 0.0, 0.0, 0.0)])
    ref, _ = oracle_target(ls, betas[0], c, lo=0.02, hi=0.5)
    lid = g.load_landscape(ls)
    tid = g.load_target(lid, ref)
    g.set_burn_steps(lid, bs)
    T = [oracle.thresholds(ls, b) for b in betas]
    sims = fire.make_sims(60, lid, tid, c, param_index=np.arange(60) % 2)
    sims["max_steps"][::7] = 5
    for threads, qcap, wg in [(512, 1024, 4), (64, 64, 4), (256, 64, 2), (1024, 128, 1)]:
        say(f"turn-off {mode} threads={threads} qcap={qcap}")
        g.set_schedule(threads, qcap, 1 if mode == "table" else 0, wg)
        res, maps = g.run(betas, sims, SEED, want_maps=True)
        g.sync()
        r, m = _np(res, maps)
        compare_with_oracle(ls, T, r, m, sims, SEED, ref_bits=ref, burn_steps=bs)
    g.set_schedule(reset=True)
    # back to one step: the one-step oracle again
    g.set_burn_steps(lid, None)
    res, maps = g.run(betas, sims, SEED, want_maps=True)
    g.sync()
    r, m = _np(res, maps)
    compare_with_oracle(ls, T, r, m, sims, SEED, ref_bits=ref)
    g.free_landscape(lid)


def test_turn_off_times_ragged_and_isolated(g):
    from paper_1701_03549_amd import fire
    for W, H in [(1, 1), (33, 1), (31, 33), (65, 7)]:
        ls = synth.random_small_landscape(W, H, seed=W * 7 + H, p_blocked=0.15)
        ls["veg"][0, 0] = 2
        bs = np.ones(256, dtype=np.uint8)
        bs[1], bs[2] = 2, 5
        beta = np.array([(0.2, -0.2, 0.3, 0.5, 1.0)])
        T = [oracle.thresholds(ls, beta[0])]
        lid = g.load_landscape(ls)
        g.set_burn_steps(lid, bs)
        rng = np.random.default_rng(W * H)
        ign = np.stack([rng.integers(0, W, 30), rng.integers(0, H, 30)], axis=1)
        sims = fire.make_sims(30, lid, -1, ign)
        say(f"turn-off ragged {W}x{H}")
        res, maps = g.run(beta, sims, SEED, want_maps=True)
        g.sync()
        r, m = _np(res, maps)
        compare_with_oracle(ls, T, r, m, sims, SEED, burn_steps=bs)
        g.free_landscape(lid)


def test_mixed_with_and_without_turn_off_times(g):
    import torch
    from paper_1701_03549_amd import fire
    sizes = [(96, 80, 103), (128, 64, 104)]
    lss = [synth.make_landscape(W, H, s) for W, H, s in sizes]
    lids = [g.load_landscape(ls) for ls in lss]
    bs = _steps(lss[0], np.random.default_rng(5), hi=3)
    g.set_burn_steps(lids[0], bs)
    rng = np.random.default_rng(9)
    n = 40
    betas = rng.uniform(-2.5, 0.5, size=(n, 5))
    cs = [synth.nearest_burnable(ls["veg"], W // 2, H // 2) for ls, (W, H, _) in zip(lss, sizes)]
    sims = np.concatenate([fire.make_sims(1, lids[i % 2], -1, cs[i % 2], param_index=i,
                                          sim_index=500 + i) for i in range(n)])
    say("mixed turn-off / one-step, host descriptors and device descriptors")
    res, maps = g.run(betas, sims, SEED, want_maps=True)
    d_sims = torch.from_numpy(sims.view(np.uint8).copy()).cuda()
    out = torch.empty((n, 24), dtype=torch.uint8, device="cuda")
    g.run_dev(torch.from_numpy(betas).cuda(), d_sims, n, SEED, out)
    g.sync()
    assert torch.equal(res, out)
    r, m = _np(res, maps)
    for i in range(n):
        w = i % 2
        sd = sims[i:i + 1].copy()
        sd["param_index"] = 0
        compare_with_oracle(lss[w], [oracle.thresholds(lss[w], betas[i])], r[i:i + 1],
                            m[i:i + 1], sd, SEED, burn_steps=bs if w == 0 else None)
    for lid in lids:
        g.free_landscape(lid)


def test_zero_turn_off_time_rejected(g):
    from paper_1701_03549_amd import fire
    ls = synth.make_landscape(16, 16, 1)
    lid = g.load_landscape(ls)
    bs = np.ones(256, dtype=np.uint8)
    bs[7] = 0
    with pytest.raises(fire.FireError):
        g.set_burn_steps(lid, bs)
    g.free_landscape(lid)


def test_turn_off_times_512_sampled(g):
    """512x512 at the calibration vector with turn-off times of 2 steps for
    forest and 3 for the other vegetation, 1280 replicates in one launch,
    20 sampled simulations recomputed by the oracle."""
    from paper_1701_03549_amd import fire
    W = H = 512
    ls = synth.make_landscape(W, H, 102)
    c = synth.ignition_site(ls)
    bs = np.full(256, 3, dtype=np.uint8)
    bs[1] = 2
    lid = g.load_landscape(ls)
    g.set_burn_steps(lid, bs)
    sims = fire.make_sims(1280, lid, -1, c)
    say("turn-off 512^2 x 1280")
    res, maps = g.run(np.array([BETA_STAR]), sims, SEED, want_maps=True)
    g.sync()
    r, m = _np(res, maps)
    T = [oracle.thresholds(ls, BETA_STAR)]
    compare_with_oracle(ls, T, r, m, sims, SEED, idx=range(0, 1280, 64), burn_steps=bs)
    pop = np.array([int(np.unpackbits(m[i].view(np.uint8)).sum()) for i in range(1280)])
    assert np.array_equal(pop, r["burnt"])
    g.free_landscape(lid)
