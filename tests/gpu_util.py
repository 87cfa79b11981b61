"""Shared helpers of the GPU tests: a library context, oracle-side references."""
import numpy as np
import pytest

import oracle
from paper_1701_03549_amd import synth

SEED = 0x5EED0001
TARGET_SEED = 0x7A26E7
BETA_STAR = (-3.0, -0.5, 6.0, 1.0, 2.0)


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def oracle_target(ls, beta, ign, seed=TARGET_SEED, lo=0.0, hi=1.0, tries=200):
    """Reference map from the oracle: the first sim_index whose burnt fraction
    lies in [lo, hi] (a contained reference fire)."""
    veg = ls["veg"]
    H, W = veg.shape
    T = oracle.thresholds(ls, beta)
    for k in range(tries):
        r = oracle.simulate(veg, T, ign, k, seed)
        frac = r["burnt"] / (W * H)
        if lo <= frac <= hi:
            return r["map"], k
    raise RuntimeError("no reference fire in range")


def compare_with_oracle(ls, T_oracle, res, maps, sims, seed, ref_bits=None, idx=None,
                        burn_steps=None):
    """Bit-exact check of GPU results (and maps) against the oracle."""
    veg = ls["veg"]
    H, W = veg.shape
    idx = range(len(sims)) if idx is None else idx
    for i in idx:
        sd = sims[i]
        o = oracle.simulate(veg, T_oracle[int(sd["param_index"])], (int(sd["ign_x"]), int(sd["ign_y"])),
                            int(sd["sim_index"]), seed, int(sd["max_steps"]),
                            burn_steps=burn_steps)
        got = (int(res["burnt"][i]), int(res["steps"][i]), int(res["trials"][i]))
        want = (o["burnt"], o["steps"], o["trials"])
        assert got == want, (i, got, want)
        if maps is not None:
            m = maps[i][: H * ((W + 31) // 32)].reshape(H, -1)
            assert np.array_equal(m, o["map"]), i
        if ref_bits is not None:
            f = oracle.fitness(o["map"], ref_bits, W, H) if o["burnt"] else 1.0
            assert res["fitness"][i] == f, (i, res["fitness"][i], f)
