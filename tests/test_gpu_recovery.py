"""Recovery of the generating parameters by the batched GA (Appendix B) at
512x512: 64 individuals x 20 replicates x 50 generations from the Gaussian
prior of Table 1, against a reference fire made at the calibration vector.
Bounds (set from a pilot before timing): the best individual's mean fitness
is below the stochastic floor of replicates at the generating vector (0.054),
and the wind coefficient, the best identified one, is recovered within 1 by
the accepted ensemble (fitness < 0.3)."""
import numpy as np
import pytest

from gpu_util import say
from paper_1701_03549_amd import synth

pytestmark = pytest.mark.gpu
BETA_STAR = (-3.0, -0.5, 6.0, 1.0, 2.0)


def test_ga_recovers_calibration_vector():
    from paper_1701_03549_amd import fire, ga
    g = fire.FireGPU(0)
    W = H = 512
    ls = synth.make_landscape(W, H, 102)
    c = synth.ignition_site(ls)
    lid = g.load_landscape(ls)
    res, maps = g.run(np.array([BETA_STAR]), fire.make_sims(32, lid, -1, c), 0x7A26E7,
                      want_maps=True)
    g.sync()
    r = fire.results_to_numpy(res)
    k = int(np.argmax(r["burnt"] >= 0.01 * W * H))
    tid = g.load_target(lid, maps.cpu().numpy().view(np.uint32)[k].reshape(H, -1))
    pop0 = np.clip(np.random.default_rng(2024).normal(0.0, 5.0, size=(64, 5)), -30, 30)
    say("GA recovery at 512x512")
    hist = ga.run_batched(g, lid, tid, c, pop0, R=20, generations=50, sim_seed=0x5EED0001,
                          ga_seed=0x6A00001)
    rec = ga.recovered(g, hist, cutoff=0.3)
    say(f"best mean fitness {rec['best_mean_fitness']:.4f}, accepted {rec['n_accepted']}, "
        f"mean {np.round(rec['accepted_mean'], 2)}")
    assert rec["best_mean_fitness"] < 0.054
    assert rec["n_accepted"] > 1000
    assert abs(rec["accepted_mean"][3] - BETA_STAR[3]) < 1.0
    g.close()
