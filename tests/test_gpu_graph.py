"""Graph capture of a simulation launch (device descriptors) and size-class
grouping: replays of a captured batch reproduce the eager results exactly,
with the program's own work between replays."""
import numpy as np
import pytest

import oracle
from gpu_util import SEED, compare_with_oracle, say
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


def _mixed(g, n=96):
    from paper_1701_03549_amd import fire
    sizes = [(128, 128, 101), (96, 200, 102), (160, 64, 103)]
    lss = [synth.make_landscape(W, H, s) for W, H, s in sizes]
    lids = [g.load_landscape(ls) for ls in lss]
    rng = np.random.default_rng(31)
    betas = rng.uniform(-4, 3, size=(n, 5))
    which = rng.integers(0, 3, size=n)
    sims = np.concatenate([
        fire.make_sims(1, lids[w], -1, synth.nearest_burnable(lss[w]["veg"], sizes[w][0] // 2,
                                                                sizes[w][1] // 2),
                       param_index=i, sim_index=7000 + i) for i, w in enumerate(which)])
    return lss, lids, betas, which, sims


def test_captured_run_replays_match_eager(g):
    import torch
    lss, lids, betas, which, sims = _mixed(g)
    n = len(sims)
    d_sims = torch.from_numpy(sims.view(np.uint8).copy()).cuda()
    d_beta = torch.from_numpy(betas.copy()).cuda()
    out = torch.empty((n, 24), dtype=torch.uint8, device="cuda")
    say("graph: eager")
    g.run_dev(d_beta, d_sims, n, SEED, out)
    g.sync()
    eager = out.clone()
    graph = torch.cuda.CUDAGraph()
    say("graph: capture")
    with torch.cuda.graph(graph):
        g.run_dev(d_beta, d_sims, n, SEED, out, stream=torch.cuda.current_stream())
    for k in range(3):
        say(f"graph: replay {k}")
        out.zero_()
        scratch = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), k
        assert torch.isfinite(scratch)
    g.sync()
    for lid in lids:
        g.free_landscape(lid)


def test_grouped_classes_match_single_launch_and_oracle(g):
    """fire_run groups by landscape into concurrent launches; the results
    equal the single-launch device path and the oracle."""
    import torch
    from paper_1701_03549_amd import fire
    lss, lids, betas, which, sims = _mixed(g, n=60)
    n = len(sims)
    say("grouped vs single")
    res, _ = g.run(betas, sims, SEED)
    g.sync()
    d_sims = torch.from_numpy(sims.view(np.uint8).copy()).cuda()
    d_beta = torch.from_numpy(betas.copy()).cuda()
    out = torch.empty((n, 24), dtype=torch.uint8, device="cuda")
    g.run_dev(d_beta, d_sims, n, SEED, out)
    g.sync()
    assert torch.equal(res, out)
    r = fire.results_to_numpy(res)
    for i in range(0, n, 4):
        ls = lss[which[i]]
        sd = sims[i:i + 1].copy()
        sd["param_index"] = 0
        compare_with_oracle(ls, [oracle.thresholds(ls, betas[i])], r[i:i + 1], None, sd, SEED)
    # a class schedule changes nothing either
    g.set_class_schedule(128 * 128, {"threads": 512, "queue_cap": 1024, "table_mode": 0,
                                     "wg_per_cu": 2}, kind="scattered")
    assert g.get_schedule(128 * 128, 60, 60)["threads"] == 512
    res2, _ = g.run(betas, sims, SEED)
    g.sync()
    assert torch.equal(res, res2)
    g.set_class_schedule(128 * 128, None)
    for lid in lids:
        g.free_landscape(lid)


def test_capture_rules(g):
    """fire_run refuses stream capture (its host staging would be read at
    replay time); a captured fire_run_dev stays valid after a later, larger
    eager call grows the context's scratch buffers (they are retired, not
    freed), and its replays still equal the eager results."""
    import torch
    from paper_1701_03549_amd import fire
    W, H = 96, 80
    ls = synth.make_landscape(W, H, 21)
    lid = g.load_landscape(ls)
    c = synth.nearest_burnable(ls["veg"], W // 2, H // 2)
    n = 64
    betas = np.array([(-0.4, -0.3, 0.2, 0.8, 1.0)])
    sims = fire.make_sims(n, lid, -1, c)
    d_sims = torch.from_numpy(sims.view(np.uint8).copy()).cuda()
    d_beta = torch.from_numpy(betas.copy()).cuda()
    out = torch.empty((n, 24), dtype=torch.uint8, device="cuda")
    say("capture rules: eager")
    g.run_dev(d_beta, d_sims, n, SEED, out)
    g.sync()
    eager = out.clone()
    graph = torch.cuda.CUDAGraph()
    err = None
    say("capture rules: capture (fire_run refused, fire_run_dev recorded)")
    with torch.cuda.graph(graph):
        try:
            g.run(betas, sims, SEED, stream=torch.cuda.current_stream())
        except fire.FireError as e:
            err = e
        g.run_dev(d_beta, d_sims, n, SEED, out, stream=torch.cuda.current_stream())
    assert err is not None and err.status == -4, err
    # a larger eager call: 512x512 landscape, 1280 simulations (spill area,
    # retry list and threshold tables all grow)
    big = synth.make_landscape(512, 512, 102)
    lid2 = g.load_landscape(big)
    bs = fire.make_sims(1280, lid2, -1, synth.ignition_site(big))
    say("capture rules: larger eager call")
    res_big, _ = g.run(np.array([(-3.0, -0.5, 6.0, 1.0, 2.0)]), bs, SEED)
    g.sync()
    assert fire.results_to_numpy(res_big)["burnt"].min() >= 1
    g.free_landscape(lid2)
    for k in range(3):
        say(f"capture rules: replay {k}")
        out.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), k
    g.sync()
    del graph
    g.free_landscape(lid)


def test_sim_timing_clocks(g):
    """Per-simulation clocks: results with the clocks on equal results with
    them off; every simulation gets a take and a later finish stamp, and the
    load-balance summary is consistent (slots at most the simulations, span
    at least the longest simulation)."""
    import torch
    from paper_1701_03549_amd import fire
    from paper_1701_03549_amd.timing import load_balance
    lss, lids, betas, which, sims = _mixed(g, n=200)
    n = len(sims)
    d_sims = torch.from_numpy(sims.view(np.uint8).copy()).cuda()
    d_beta = torch.from_numpy(betas.copy()).cuda()
    out0 = torch.empty((n, 24), dtype=torch.uint8, device="cuda")
    out1 = torch.empty_like(out0)
    say("timing: off")
    g.run_dev(d_beta, d_sims, n, SEED, out0)
    g.sync()
    clocks = torch.zeros((n, 2), dtype=torch.int64, device="cuda")
    g.set_sim_timing(clocks)
    say("timing: on (device descriptors, then grouped host path)")
    g.run_dev(d_beta, d_sims, n, SEED, out1)
    g.sync()
    t = clocks.cpu().numpy()
    assert torch.equal(out0, out1)
    assert np.all(t[:, 0] > 0) and np.all(t[:, 1] >= t[:, 0])
    lb = load_balance(t)
    assert lb["sims"] == n and 1 <= lb["slots"] <= n
    assert lb["span_ms"] >= lb["longest_sim_ms"] > 0 and 0 < lb["efficiency"] <= 1
    clocks.zero_()
    res, _ = g.run(betas, sims, SEED)
    g.sync()
    assert torch.equal(res, out0)
    t = clocks.cpu().numpy()
    assert np.all(t[:, 0] > 0) and np.all(t[:, 1] >= t[:, 0])
    # a buffer shorter than the batch: stamps only below its capacity
    short = torch.zeros((n // 2, 2), dtype=torch.int64, device="cuda")
    g.set_sim_timing(short)
    g.run_dev(d_beta, d_sims, n, SEED, out1)
    g.sync()
    assert torch.equal(out0, out1) and np.all(short.cpu().numpy()[:, 0] > 0)
    g.set_sim_timing(None)
    with pytest.raises(ValueError):
        g.set_sim_timing(torch.zeros(8, dtype=torch.int64, device="cuda"))
    for lid in lids:
        g.free_landscape(lid)


def test_ordered_descriptors_captured_match_fire_run(g):
    """fire_order_sims gives the longest-expected-first permutation fire_run
    uses (checked against its documented key); a captured fire_run_dev over
    descriptors uploaded in that order reproduces fire_run's rows."""
    import torch
    lss, lids, betas, which, sims = _mixed(g, n=60)
    n = len(sims)
    say("order_sims")
    order = g.order_sims(betas, sims)
    assert sorted(order.tolist()) == list(range(n))
    # the documented key: burnable cells x the Eq. 1 probability averaged
    # over forest and other burnable cells at the mean aspect and slope terms
    sig = lambda v: 1.0 / (1.0 + np.exp(-v))
    key = np.empty(n)
    for i in range(n):
        ls = lss[which[i]]
        veg = ls["veg"].ravel()
        m = veg != 0
        sl = ls["slope_deg"].ravel()[m].astype(np.float64)
        asp = ls["aspect_deg"].ravel()[m].astype(np.float64)
        nb = m.sum()
        mf = (veg[m] == 1).sum() / nb
        psi = np.where(sl > 5.0, np.cos((asp - 315.0) * np.pi / 180.0), 0.0).sum() / nb
        sgm = (0.5 * sl / 100.0).sum() / nb
        b = betas[sims[i]["param_index"]]
        x = b[0] + b[2] * psi + b[4] * sgm
        key[i] = nb * (mf * sig(x + b[1]) + (1.0 - mf) * sig(x))
    k = key[order]
    assert np.all(k[1:] <= k[:-1] * (1 + 1e-9) + 1e-9)
    res, _ = g.run(betas, sims, SEED)
    g.sync()
    d_sims = torch.from_numpy(sims[order].view(np.uint8).copy()).cuda()
    d_beta = torch.from_numpy(betas.copy()).cuda()
    out = torch.empty((n, 24), dtype=torch.uint8, device="cuda")
    g.run_dev(d_beta, d_sims, n, SEED, out)
    g.sync()
    idx = torch.from_numpy(order.astype(np.int64)).cuda()
    assert torch.equal(out, res[idx])
    out_g = torch.empty_like(out)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g.run_dev(d_beta, d_sims, n, SEED, out_g, stream=torch.cuda.current_stream())
    for _ in range(2):
        out_g.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out_g, res[idx])
    del graph
    bad = sims.copy()
    bad[3]["landscape_id"] = 999
    with pytest.raises(Exception):
        g.order_sims(betas, bad)
    assert len(g.order_sims(betas, sims[:0])) == 0
    for lid in lids:
        g.free_landscape(lid)
