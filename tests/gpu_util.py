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


def oracle_threads():
    """Worker threads for oracle batches (at most 16 host threads)."""
    import os
    return max(1, min(16, os.cpu_count() or 1))


def check_batch_against_oracle(landscapes, betas, sims, res, maps, seed, refs=None,
                               threads=None, table_cache_max=8):
    """Every simulation of a batch, per element, against the oracle: map words,
    burnt, steps, trials and Eq. 2 fitness, bit for bit.

    landscapes: {landscape_id: landscape dict}; betas: [n_params][5]; sims:
    the descriptors; res: numpy results; maps: numpy uint32 [n][map_words] or
    None; refs: {target_id: packed reference map}. Oracle thresholds are
    computed once per (landscape, parameter vector) when there are at most
    table_cache_max such pairs, else inside each worker (per-simulation
    vectors). Runs on a thread pool (the oracle releases the GIL). Returns
    the number of simulations checked; raises AssertionError on the first
    mismatch, naming the simulation."""
    from concurrent.futures import ThreadPoolExecutor
    refs = refs or {}
    betas = np.asarray(betas, dtype=np.float64).reshape(-1, 5)
    pairs = sorted({(int(s["landscape_id"]), int(s["param_index"])) for s in sims})
    cache = {}
    if len(pairs) <= table_cache_max:
        for lid, p in pairs:
            cache[(lid, p)] = oracle.thresholds(landscapes[lid], betas[p])

    def one(i):
        sd = sims[i]
        lid, p = int(sd["landscape_id"]), int(sd["param_index"])
        ls = landscapes[lid]
        H, W = ls["veg"].shape
        T = cache.get((lid, p))
        if T is None:
            T = oracle.thresholds(ls, betas[p])
        o = oracle.simulate(ls["veg"], T, (int(sd["ign_x"]), int(sd["ign_y"])),
                            int(sd["sim_index"]), seed, int(sd["max_steps"]))
        got = (int(res["burnt"][i]), int(res["steps"][i]), int(res["trials"][i]))
        want = (o["burnt"], o["steps"], o["trials"])
        if got != want:
            return f"simulation {i}: (burnt, steps, trials) {got} != oracle {want}"
        if maps is not None:
            m = maps[i][: H * ((W + 31) // 32)].reshape(H, -1)
            if not np.array_equal(m, o["map"]):
                bad = int(np.count_nonzero(m != o["map"]))
                return f"simulation {i}: {bad} map words differ from the oracle"
        tgt = int(sd["target_id"])
        if tgt >= 0:
            f = oracle.fitness(o["map"], refs[tgt], W, H) if o["burnt"] else 1.0
            if not (res["fitness"][i] == f):
                return f"simulation {i}: fitness {res['fitness'][i]!r} != oracle {f!r}"
        return None

    with ThreadPoolExecutor(max_workers=threads or oracle_threads()) as ex:
        errors = [e for e in ex.map(one, range(len(sims))) if e is not None]
    assert not errors, f"{len(errors)} of {len(sims)} simulations differ; first: {errors[0]}"
    return len(sims)
