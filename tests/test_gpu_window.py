"""GPU parity of window runs (each simulation first runs in an LDS window
around its ignition; a fire that comes within one cell of a window edge
inside the lattice is run again over the whole lattice) against the oracle
and against whole-lattice runs: maps (zero outside the window), burnt, step
and trial counts and Eq. 2 bit-exact, under small windows that force many
re-runs, spilling queues, turn-off times, mixed landscapes, device
descriptors and the captured GA."""
import numpy as np
import pytest

import oracle
from gpu_util import BETA_STAR, SEED, compare_with_oracle, oracle_target, say
from paper_1701_03549_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import torch
    from paper_1701_03549_amd import fire
    assert torch.cuda.is_available()
    ctx = fire.FireGPU(0)
    yield ctx
    ctx.close()


def _np(res, maps):
    from paper_1701_03549_amd import fire
    return fire.results_to_numpy(res), None if maps is None else maps.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("table", [1, 0])
def test_windows_match_oracle(g, table):
    from paper_1701_03549_amd import fire
    W, H = 100, 67
    ls = synth.make_landscape(W, H, 6)
    beta = np.array([(-0.4, -0.3, 0.2, 0.8, 1.0), (0.3, 0.0, 0.0, 0.0, 0.0)])
    ref, _ = oracle_target(ls, beta[0], (50, 33), lo=0.01)
    lid = g.load_landscape(ls)
    tid = g.load_target(lid, ref)
    T = [oracle.thresholds(ls, b) for b in beta]
    rng = np.random.default_rng(3)
    ign = np.stack([rng.integers(0, W, 48), rng.integers(0, H, 48)], axis=1)
    ign[:8] = (50, 33)
    sims = fire.make_sims(48, lid, tid, ign, param_index=np.arange(48) % 2)
    sims["max_steps"][::11] = 6
    for threads, qcap, wg, win in [(256, 256, 4, 64), (64, 64, 8, 64), (256, 512, 2, 96),
                                   (128, 128, 4, 128)]:
        say(f"window {win} table={table} threads={threads} qcap={qcap}")
        g.set_schedule(threads, qcap, table, wg, window=win)
        res, maps = g.run(beta, sims, SEED, want_maps=True)
        g.sync()
        r, m = _np(res, maps)
        compare_with_oracle(ls, T, r, m, sims, SEED, ref_bits=ref)
    g.set_schedule(reset=True)
    g.free_landscape(lid)


def test_window_512_default_equals_whole_lattice(g):
    """The calibration batch at 512x512: the built-in plan (a window) and a
    whole-lattice schedule give identical results; 16 sampled simulations
    against the oracle."""
    import torch
    from paper_1701_03549_amd import fire
    W = H = 512
    ls = synth.make_landscape(W, H, 102)
    c = synth.ignition_site(ls)
    ref, _ = oracle_target(ls, BETA_STAR, c, lo=0.01, hi=0.15)
    lid = g.load_landscape(ls)
    tid = g.load_target(lid, ref)
    n = 1280
    sims = fire.make_sims(n, lid, tid, c)
    d_sims = torch.from_numpy(sims.view(np.uint8).copy()).cuda()
    d_beta = torch.tensor([BETA_STAR], dtype=torch.float64, device="cuda")
    mw = H * (W // 32)
    outs = []
    for sched in (None, dict(threads=256, queue_cap=1016, table_mode=1, wg_per_cu=4, window=0),
                  dict(threads=256, queue_cap=512, table_mode=1, wg_per_cu=8, window=128)):
        say(f"512^2 schedule {sched}")
        if sched is None:
            g.set_schedule(reset=True)
            assert g.get_schedule(W * H, 1, n)["window"] > 0
        else:
            g.set_schedule(**sched)
        out = torch.empty((n, 24), dtype=torch.uint8, device="cuda")
        maps = torch.empty((n, mw), dtype=torch.int32, device="cuda")
        g.run_dev(d_beta, d_sims, n, SEED, out, maps, mw)
        g.sync()
        outs.append((out, maps))
    g.set_schedule(reset=True)
    for o, m in outs[1:]:
        assert torch.equal(o, outs[0][0]) and torch.equal(m, outs[0][1])
    r, m = _np(*outs[0])
    compare_with_oracle(ls, [oracle.thresholds(ls, BETA_STAR)], r, m, sims, SEED, ref_bits=ref,
                        idx=range(0, n, n // 16))
    g.free_landscape(lid)


def test_window_turn_off_times_and_mixed(g):
    """Turn-off times in window runs, two landscapes in one call, host and
    device descriptors."""
    import torch
    from paper_1701_03549_amd import fire
    sizes = [(160, 128, 103), (128, 96, 104)]
    lss = [synth.make_landscape(W, H, s) for W, H, s in sizes]
    lids = [g.load_landscape(ls) for ls in lss]
    bs = np.ones(256, dtype=np.uint8)
    bs[1], bs[2], bs[3] = 2, 3, 1
    g.set_burn_steps(lids[0], bs)
    rng = np.random.default_rng(12)
    n = 40
    betas = rng.uniform(-2.5, 0.5, size=(n, 5))
    cs = [synth.nearest_burnable(ls["veg"], W // 2, H // 2) for ls, (W, H, _) in zip(lss, sizes)]
    sims = np.concatenate([fire.make_sims(1, lids[i % 2], -1, cs[i % 2], param_index=i,
                                          sim_index=700 + i) for i in range(n)])
    g.set_schedule(256, 256, 0, 4, window=64)
    say("window 64: turn-off times, mixed landscapes")
    res, maps = g.run(betas, sims, SEED, want_maps=True)
    d_sims = torch.from_numpy(sims.view(np.uint8).copy()).cuda()
    out = torch.empty((n, 24), dtype=torch.uint8, device="cuda")
    g.run_dev(torch.from_numpy(betas).cuda(), d_sims, n, SEED, out)
    g.sync()
    g.set_schedule(reset=True)
    assert torch.equal(res, out)
    r, m = _np(res, maps)
    for i in range(n):
        w = i % 2
        sd = sims[i:i + 1].copy()
        sd["param_index"] = 0
        compare_with_oracle(lss[w], [oracle.thresholds(lss[w], betas[i])], r[i:i + 1], m[i:i + 1],
                            sd, SEED, burn_steps=bs if w == 0 else None)
    for lid in lids:
        g.free_landscape(lid)


def test_window_ga_run_equals_whole_lattice(g):
    from paper_1701_03549_amd import ga
    W = H = 128
    ls = synth.make_landscape(W, H, 105)
    c = synth.nearest_burnable(ls["veg"], 64, 64)
    ref, _ = oracle_target(ls, (-0.9, -0.5, 0.3, 0.8, 1.0), c, lo=0.02, hi=0.5)
    lid = g.load_landscape(ls)
    tid = g.load_target(lid, ref)
    pop0 = np.random.default_rng(4).normal(0, 1.0, size=(16, 5)) - np.array([1, 0, 0, 0, 0])
    hist = []
    for win in (0, 64):
        say(f"GA with window {win}")
        g.set_schedule(256, 256, 0, 4, window=win)
        hp, hf = ga.run_batched(g, lid, tid, c, pop0, R=4, generations=4, sim_seed=SEED,
                                ga_seed=0x6A00001)
        g.sync()
        hist.append((hp.cpu().numpy(), hf.cpu().numpy()))
    g.set_schedule(reset=True)
    assert np.array_equal(hist[0][0], hist[1][0]) and np.array_equal(hist[0][1], hist[1][1])
    g.free_landscape(lid)


@pytest.mark.parametrize("threads,wg", [
    pytest.param(1024, 1, marks=pytest.mark.skip(
        reason="a 1024-thread window run whose fires all outgrow the window stopped responding "
               "on the GPU (also after the end-of-run flag was moved to rotating slots); the "
               "library now runs 1024-thread schedules without a window, and this case stays "
               "off the GPU until the cause is found")),
    (512, 2)])
def test_window_large_workgroups_end_together(g, threads, wg):
    """Many waves per workgroup with a window every fire outgrows: every
    wave must leave a run at the same step (the end-of-run flag is read at
    the top of a step and written only after that step's first barrier)."""
    import torch
    from paper_1701_03549_amd import fire
    W = H = 512
    ls = synth.make_landscape(W, H, 102)
    c = synth.ignition_site(ls)
    lid = g.load_landscape(ls)
    n = 256
    sims = fire.make_sims(n, lid, -1, c)
    d_sims = torch.from_numpy(sims.view(np.uint8).copy()).cuda()
    d_beta = torch.tensor([BETA_STAR], dtype=torch.float64, device="cuda")
    outs = []
    for win in (0, 128):
        say(f"threads={threads} window {win}")
        g.set_schedule(threads, 1024, 1, wg, window=win)
        out = torch.empty((n, 24), dtype=torch.uint8, device="cuda")
        g.run_dev(d_beta, d_sims, n, SEED, out)
        g.sync()
        outs.append(out)
    g.set_schedule(reset=True)
    assert torch.equal(outs[0], outs[1])
    g.free_landscape(lid)


def test_auto_window_turns_off_after_repeats():
    """The built-in plan gives a 512x512 batch an LDS window; when the fires
    outgrow it (every simulation is run again), the re-run count reported by
    the second launch turns windows off for that landscape, and results
    equal whole-lattice runs throughout."""
    import torch
    from paper_1701_03549_amd import fire
    W = H = 512
    n = 1280
    ctx = fire.FireGPU(0)
    try:
        ls = synth.make_landscape(W, H, 102)
        c = synth.ignition_site(ls)
        lid = ctx.load_landscape(ls)
        sims = fire.make_sims(n, lid, -1, c)
        d_sims = torch.from_numpy(sims.view(np.uint8).copy()).cuda()
        # a large intercept: fires reach the whole burnable lattice
        d_beta = torch.tensor([[6.0, 0.0, 0.0, 0.0, 0.0]], dtype=torch.float64, device="cuda")
        before = ctx.get_schedule(W * H, 1, n)
        assert before["window"] > 0
        outs = []
        for label in ("auto, window", "auto, after repeats"):
            say(f"512x512 {label}")
            out = torch.empty((n, 24), dtype=torch.uint8, device="cuda")
            ctx.run_dev(d_beta, d_sims, n, SEED, out)
            ctx.sync()
            outs.append(out)
        assert ctx.get_schedule(W * H, 1, n)["window"] == 0
        say("512x512 whole lattice")
        ctx.set_schedule(before["threads"], before["queue_cap"], before["table_mode"],
                         before["wg_per_cu"], window=0)
        out = torch.empty((n, 24), dtype=torch.uint8, device="cuda")
        ctx.run_dev(d_beta, d_sims, n, SEED, out)
        ctx.sync()
        for o in outs:
            assert torch.equal(o, out)
        r = fire.results_to_numpy(out)
        assert r["burnt"].min() > W * H // 4
    finally:
        ctx.close()


def test_bad_window_rejected(g):
    from paper_1701_03549_amd import fire
    for win in (32, 100, 8192, -2):
        with pytest.raises(fire.FireError):
            g.set_schedule(256, 256, 1, 4, window=win)
