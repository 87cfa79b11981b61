"""The no-allocation entry point (fire_run_dev_noalloc, scratch in a
per-GPU device array) against fire_run_dev: identical results and maps on
two calls in a row, the second with a smaller input, under the built-in and
a fixed schedule, with the caller's threshold table and with per-trial
thresholds; a batch whose re-run list and spill area cannot fit the scratch
is rejected before any device work."""
import numpy as np
import pytest

from gpu_util import BETA_STAR, SEED, say
from paper_1701_03549_amd import synth

pytestmark = pytest.mark.gpu


def _run_both(g, d_beta, d_sims, n, mw, override=None):
    import torch
    outs = []
    for f in (g.run_dev, g.run_dev_noalloc):
        out = torch.full((n, 24), 0xAB, dtype=torch.uint8, device="cuda")
        maps = torch.full((n, mw), -1, dtype=torch.int32, device="cuda")
        f(d_beta, d_sims, n, SEED, out, maps, mw, override=override)
        g.sync()
        outs.append((out, maps))
    return outs


def test_noalloc_equals_run_dev_two_calls():
    import torch
    from paper_1701_03549_amd import fire
    g = fire.FireGPU(0)
    try:
        # first call: the 512x512 calibration batch, the caller's table
        W = H = 512
        ls = synth.make_landscape(W, H, 102)
        c = synth.ignition_site(ls)
        lid = g.load_landscape(ls)
        n = 1280
        sims = fire.make_sims(n, lid, -1, c)
        d_sims = torch.from_numpy(sims.view(np.uint8).copy()).cuda()
        d_beta = torch.tensor([BETA_STAR], dtype=torch.float64, device="cuda")
        table = g.thresholds(lid, BETA_STAR)
        mw = H * (W // 32)
        say("no-alloc: 512^2 x 1280 with the caller's table")
        (a, am), (b, bm) = _run_both(g, d_beta, d_sims, n, mw, override=table)
        assert torch.equal(a, b) and torch.equal(am, bm)
        assert fire.results_to_numpy(b)["burnt"].min() >= 1
        say("no-alloc: same batch, per-trial thresholds, workgroup kernel")
        g.set_schedule(256, 512, 0, 4, window=0)
        (a, am), (b, bm) = _run_both(g, d_beta, d_sims, n, mw)
        assert torch.equal(a, b) and torch.equal(am, bm)
        g.set_schedule(reset=True)
        g.free_landscape(lid)
        # second call: a smaller input (96x80, 64 simulations, three vectors)
        W2, H2 = 96, 80
        ls2 = synth.make_landscape(W2, H2, 21)
        lid2 = g.load_landscape(ls2)
        c2 = synth.nearest_burnable(ls2["veg"], W2 // 2, H2 // 2)
        n2 = 64
        betas2 = np.array([(-0.4, -0.3, 0.2, 0.8, 1.0), (0.5, 0, 0, 0, 0), (-2, 0, 0, 0, 0)])
        sims2 = fire.make_sims(n2, lid2, -1, c2, param_index=np.arange(n2) % 3)
        d_sims2 = torch.from_numpy(sims2.view(np.uint8).copy()).cuda()
        d_beta2 = torch.from_numpy(betas2).cuda()
        mw2 = H2 * ((W2 + 31) // 32)
        say("no-alloc: 96x80 x 64, three parameter vectors")
        (a, am), (b, bm) = _run_both(g, d_beta2, d_sims2, n2, mw2)
        assert torch.equal(a, b) and torch.equal(am, bm)
        # a batch whose re-run list and spill area do not fit the scratch
        # (2^24 descriptors) is rejected before any device work
        lid3 = g.load_landscape(ls2)
        n3 = 1 << 24
        d3 = torch.zeros((n3, 28), dtype=torch.uint8, device="cuda")
        out3 = torch.empty((1, 24), dtype=torch.uint8, device="cuda")
        say("no-alloc: oversized batch rejected")
        with pytest.raises(fire.FireError) as ei:
            g.run_dev_noalloc(d_beta2, d3, n3, SEED, out3)
        assert ei.value.status == -1 and "no-allocation scratch" in str(ei.value)
        g.sync()
        g.free_landscape(lid3)
    finally:
        g.close()
