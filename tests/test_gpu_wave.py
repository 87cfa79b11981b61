"""GPU parity of the wavefront-per-simulation kernel (one 64-lane wavefront
runs a simulation with its frontier queues in LDS; fires whose front
outgrows them, or that reach a window edge, are run again by the workgroup
kernel) against the oracle: maps, burnt, steps, trials and Eq. 2 bit-exact,
with small queues and windows that force many re-runs, both threshold
modes, step caps, non-burnable ignitions; built-in plans do not choose it."""
import numpy as np
import pytest

import oracle
from gpu_util import BETA_STAR, SEED, check_batch_against_oracle, oracle_target, say
from paper_1701_03549_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import torch
    from paper_1701_03549_amd import fire
    assert torch.cuda.is_available()
    ctx = fire.FireGPU(0)
    yield ctx
    ctx.set_schedule(reset=True)
    ctx.close()


def _np(res, maps):
    from paper_1701_03549_amd import fire
    return fire.results_to_numpy(res), None if maps is None else maps.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("table", [1, 0])
@pytest.mark.parametrize("qcap,window", [(64, 0), (64, 64), (128, 96), (512, 0), (1024, 128)])
def test_wave_kernel_matches_oracle(g, table, qcap, window):
    from paper_1701_03549_amd import fire
    W, H = 100, 67
    ls = synth.make_landscape(W, H, 6)
    betas = np.array([(-0.4, -0.3, 0.2, 0.8, 1.0), (0.3, 0.0, 0.0, 0.0, 0.0),
                      (-2.0, 0.0, 0.0, 0.0, 0.0)])
    ref, _ = oracle_target(ls, betas[0], (50, 33), lo=0.01)
    lid = g.load_landscape(ls)
    tid = g.load_target(lid, ref)
    rng = np.random.default_rng(5)
    n = 96
    ign = np.stack([rng.integers(0, W, n), rng.integers(0, H, n)], axis=1)
    ign[:12] = (50, 33)
    sims = fire.make_sims(n, lid, tid, ign, param_index=np.arange(n) % 3)
    sims["max_steps"][::13] = 5
    sims["max_steps"][7] = 0
    say(f"wave kernel table={table} queue_cap={qcap} window={window}")
    g.set_schedule(64, qcap, table, 1, window=window, wave=1)
    assert g.get_schedule(W * H, 3, n)["wave"] == 1
    res, maps = g.run(betas, sims, SEED, want_maps=True)
    g.sync()
    g.set_schedule(reset=True)
    r, m = _np(res, maps)
    check_batch_against_oracle({lid: ls}, betas, sims, r, m, SEED, refs={tid: ref})
    g.free_landscape(lid)


def test_wave_kernel_equals_workgroup_kernel_512(g):
    """The calibration batch: the built-in plan (workgroup kernel), the
    wavefront kernel in a 416-cell window and over the whole lattice, and the
    workgroup kernel with a fixed schedule give identical results and maps;
    all 1280 against the oracle."""
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
    g.set_schedule(reset=True)
    sched = g.get_schedule(W * H, 1, n)
    say(f"built-in plan at 512^2: {sched}")
    assert sched["wave"] == 0
    outs = []
    for s in (None, dict(threads=64, queue_cap=512, table_mode=1, wg_per_cu=1, window=416, wave=1),
              dict(threads=64, queue_cap=512, table_mode=1, wg_per_cu=1, window=0, wave=1),
              dict(threads=256, queue_cap=1016, table_mode=1, wg_per_cu=4, window=0, wave=0)):
        say(f"512^2 schedule {s}")
        if s is None:
            g.set_schedule(reset=True)
        else:
            g.set_schedule(**s)
        out = torch.empty((n, 24), dtype=torch.uint8, device="cuda")
        maps = torch.empty((n, mw), dtype=torch.int32, device="cuda")
        g.run_dev(d_beta, d_sims, n, SEED, out, maps, mw)
        g.sync()
        outs.append((out, maps))
    g.set_schedule(reset=True)
    for o, m in outs[1:]:
        assert torch.equal(o, outs[0][0]) and torch.equal(m, outs[0][1])
    r, m = _np(*outs[0])
    check_batch_against_oracle({lid: ls}, [BETA_STAR], sims, r, m, SEED, refs={tid: ref})
    g.free_landscape(lid)


def test_wave_kernel_uneven_and_lattice_edges(g):
    """Mixed landscape sizes in one fire_run with the wavefront kernel, fires
    that run into the lattice border (no window) and ignitions on its corners
    and on non-burnable cells."""
    from paper_1701_03549_amd import fire
    sizes = [(64, 64, 101), (37, 23, 5), (128, 96, 104)]
    lss, lids = {}, []
    for W, H, sd in sizes:
        ls = synth.make_landscape(W, H, sd)
        lid = g.load_landscape(ls)
        lss[lid] = ls
        lids.append(lid)
    rng = np.random.default_rng(17)
    n = 120
    betas = rng.uniform(-3.0, 2.0, size=(n, 5))
    rows = []
    for i in range(n):
        k = i % 3
        W, H, _ = sizes[k]
        veg = lss[lids[k]]["veg"]
        if i % 10 == 0:
            ign = (0, 0) if i % 20 == 0 else (W - 1, H - 1)
        elif i % 10 == 1:
            ys, xs = np.nonzero(veg == 0)
            ign = (int(xs[0]), int(ys[0]))
        else:
            ign = (int(rng.integers(0, W)), int(rng.integers(0, H)))
        rows.append(fire.make_sims(1, lids[k], -1, ign, param_index=i, sim_index=3000 + i))
    sims = np.concatenate(rows)
    g.set_schedule(64, 256, 0, 1, window=0, wave=1)
    say("wave kernel, three landscapes, border fires")
    res, maps = g.run(betas, sims, SEED, want_maps=True)
    g.sync()
    g.set_schedule(reset=True)
    r, m = _np(res, maps)
    check_batch_against_oracle(lss, betas, sims, r, m, SEED)
    for lid in lids:
        g.free_landscape(lid)
