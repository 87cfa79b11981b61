"""CPU oracle for the stochastic CA fire model of Denham & Laneri (arXiv 1701.03549).

TEST INFRASTRUCTURE. This package is the plain, slow reference the GPU library is
checked against. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it; the product package never does, and it shares
no code with the GPU sources.

The arithmetic of the model lives in ``fire_oracle.c`` (plain C, binary64, built
with ``-ffp-contract=off``); this module only loads it through ``ctypes`` and adds
the ensemble statistics of the fitting drivers in plain numpy (binary64).

Functions and the passages of the paper they follow:

* :func:`philox` -- Philox4x32-10 (Salmon et al., SC'11), the counter-based
  generator named in the CUDA-implementation section.
* :func:`thresholds` -- Eq. 1 and the covariate definitions after it (Methods,
  "Forest Fire Spread Simulation"), quantised to 32-bit thresholds.
* :func:`simulate` -- the propagation rules of the same section: synchronous
  steps, ignition through independent per-edge coins, a burn duration of one
  step (the paper's setting) or a turn-off time per vegetation type (the
  four-state model of the same section).
* :func:`simulate_dense` -- the per-target form of the same rule (one uniform per
  candidate target per step against 1 - prod(1 - p_i)), as the paper's kernel draws it.
* :func:`fitness` -- Eq. 2.
* :func:`ga_step` -- Appendix B (elitism, tournament of two, one-point
  crossover, dynamic mutation).
* :func:`ensemble` -- best fit and spread of the accepted ensemble (Methods
  rules; Appendix D, "More results").
* :func:`scan_reduce` -- per-candidate ignition statistics (Methods rules on
  ignition points; the cutoff rule of the CUDA-implementation section).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fire_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

U32_MAX = 0xFFFFFFFF


def build(force: bool = False) -> str:
    """Compile ``fire_oracle.c`` into ``liboracle.so`` with gcc (binary64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build()
        lib = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        lib.oracle_philox4x32_10.restype = None
        lib.oracle_quantise_p.argtypes = [ctypes.c_double]
        lib.oracle_quantise_p.restype = ctypes.c_uint32
        lib.oracle_spread_probability.argtypes = [ctypes.POINTER(ctypes.c_double)] + [ctypes.c_double] * 4
        lib.oracle_spread_probability.restype = ctypes.c_double
        lib.oracle_thresholds.argtypes = [ctypes.c_int, ctypes.c_int] + [ctypes.c_void_p] * 5 + [
            ctypes.c_uint8, ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_thresholds.restype = ctypes.c_int
        lib.oracle_simulate.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
            ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
            ctypes.POINTER(ctypes.c_uint64)]
        lib.oracle_simulate.restype = ctypes.c_int
        lib.oracle_simulate_dense.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
            ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p,
            ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
            ctypes.POINTER(ctypes.c_uint64)]
        lib.oracle_simulate_dense.restype = ctypes.c_int
        lib.oracle_fitness.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_fitness.restype = ctypes.c_double
        lib.oracle_ga_step.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
            ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_ga_step.restype = ctypes.c_int
        _lib = lib
        return lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def philox(counter, key) -> np.ndarray:
    """Philox4x32-10 of one 4-word counter under a 2-word key -> 4 uint32 words."""
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*[int(v) & U32_MAX for v in counter])
    k = (ctypes.c_uint32 * 2)(*[int(v) & U32_MAX for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib.oracle_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def spread_probability(beta, i_f: float, psi: float, omega: float, sigma: float) -> float:
    """Eq. 1 for given covariate values (binary64, left-to-right sum)."""
    lib = _load()
    b = (ctypes.c_double * 5)(*[float(v) for v in beta])
    return lib.oracle_spread_probability(b, float(i_f), float(psi), float(omega), float(sigma))


def quantise(p: float) -> int:
    """p -> 32-bit threshold (round half to even of p * 2^32, saturating)."""
    return int(_load().oracle_quantise_p(float(p)))


def _landscape_arrays(ls):
    veg = np.ascontiguousarray(ls["veg"], dtype=np.uint8)
    H, W = veg.shape
    arrs = [veg] + [np.ascontiguousarray(ls[k], dtype=np.float32)
                    for k in ("elev_m", "slope_deg", "aspect_deg", "wind_to_deg")]
    for a in arrs[1:]:
        assert a.shape == (H, W)
    return W, H, arrs


def thresholds(ls, beta, forest_class: int = 1) -> np.ndarray:
    """Threshold table T[y, x, d] (uint32) of Eq. 1 for every directed edge."""
    lib = _load()
    W, H, (veg, elev, slope, aspect, wind) = _landscape_arrays(ls)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    assert b.shape == (5,)
    T = np.empty((H, W, 8), dtype=np.uint32)
    rc = lib.oracle_thresholds(W, H, _ptr(veg), _ptr(elev), _ptr(slope), _ptr(aspect), _ptr(wind),
                               int(forest_class), _ptr(b), _ptr(T))
    if rc != 0:
        raise ValueError("oracle_thresholds failed")
    return T


def words_per_row(W: int) -> int:
    return (W + 31) // 32


def simulate(veg: np.ndarray, T: np.ndarray, ign, sim_index: int, seed: int,
             max_steps: int = U32_MAX, static_edges: bool = False, want_map: bool = True,
             burn_steps=None):
    """One simulation. burn_steps: None (every cell active for one step) or
    256 turn-off times indexed by vegetation value. Returns dict(map, burnt,
    steps, trials)."""
    lib = _load()
    if burn_steps is not None:
        burn_steps = np.ascontiguousarray(burn_steps, dtype=np.uint8)
        assert burn_steps.shape == (256,)
    veg = np.ascontiguousarray(veg, dtype=np.uint8)
    H, W = veg.shape
    T = np.ascontiguousarray(T, dtype=np.uint32)
    assert T.shape == (H, W, 8)
    bits = np.zeros((H, words_per_row(W)), dtype=np.uint32) if want_map else None
    burnt = ctypes.c_uint32()
    steps = ctypes.c_uint32()
    trials = ctypes.c_uint64()
    rc = lib.oracle_simulate(W, H, _ptr(veg), _ptr(T), int(ign[0]), int(ign[1]),
                             int(sim_index) & U32_MAX, int(seed) & ((1 << 64) - 1),
                             int(max_steps) & U32_MAX, 1 if static_edges else 0,
                             _ptr(burn_steps) if burn_steps is not None else None,
                             _ptr(bits) if want_map else None,
                             ctypes.byref(burnt), ctypes.byref(steps), ctypes.byref(trials))
    if rc != 0:
        raise ValueError(f"oracle_simulate failed ({rc})")
    return {"map": bits, "burnt": burnt.value, "steps": steps.value, "trials": trials.value}


def simulate_dense(veg: np.ndarray, T: np.ndarray, ign, sim_index: int, seed: int,
                   max_steps: int = U32_MAX):
    """One simulation of the per-target form of the rule (one uniform per
    candidate target per step). Returns dict(map, burnt, steps, trials)."""
    lib = _load()
    veg = np.ascontiguousarray(veg, dtype=np.uint8)
    H, W = veg.shape
    T = np.ascontiguousarray(T, dtype=np.uint32)
    assert T.shape == (H, W, 8)
    bits = np.zeros((H, words_per_row(W)), dtype=np.uint32)
    burnt, steps, trials = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
    rc = lib.oracle_simulate_dense(W, H, _ptr(veg), _ptr(T), int(ign[0]), int(ign[1]),
                                   int(sim_index) & U32_MAX, int(seed) & ((1 << 64) - 1),
                                   int(max_steps) & U32_MAX, _ptr(bits), ctypes.byref(burnt),
                                   ctypes.byref(steps), ctypes.byref(trials))
    if rc != 0:
        raise ValueError(f"oracle_simulate_dense failed ({rc})")
    return {"map": bits, "burnt": burnt.value, "steps": steps.value, "trials": trials.value}


def fitness(sim_bits: np.ndarray, ref_bits: np.ndarray, W: int, H: int) -> float:
    """Eq. 2 between a simulated and a reference packed burn map."""
    lib = _load()
    a = np.ascontiguousarray(sim_bits, dtype=np.uint32)
    b = np.ascontiguousarray(ref_bits, dtype=np.uint32)
    assert a.shape == b.shape == (H, words_per_row(W))
    return lib.oracle_fitness(W, H, _ptr(a), _ptr(b))


def run_batch(veg, T_by_param, sims, seed, ref_bits=None, want_maps=False, threads=1,
              burn_steps=None):
    """Run many simulations (a list of dicts with param, ign, sim_index, max_steps).

    Returns a list of result dicts (burnt, steps, trials, fitness[, map]); each
    simulation is an independent call of :func:`simulate`, spread over a pool of
    ``threads`` worker threads.
    """
    H, W = np.asarray(veg).shape

    def one(sd):
        r = simulate(veg, T_by_param[sd["param"]], sd["ign"], sd["sim_index"], seed,
                     sd.get("max_steps", U32_MAX), want_map=True, burn_steps=burn_steps)
        r["fitness"] = fitness(r["map"], ref_bits, W, H) if ref_bits is not None else float("nan")
        if not want_maps:
            r["map"] = None
        return r

    if threads <= 1:
        return [one(s) for s in sims]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(one, sims))


def ga_step(pop: np.ndarray, fit: np.ndarray, *, elite: int, pm0: float, h, lo, hi, gen: int,
            generations: int, ga_seed: int):
    """One GA generation (Appendix B). h, lo, hi: a scalar for every gene or
    one value per gene. Returns (new_pop, mean_fitness)."""
    lib = _load()
    pop = np.ascontiguousarray(pop, dtype=np.float64)
    fit = np.ascontiguousarray(fit, dtype=np.float64)
    P, G = pop.shape
    R = fit.shape[1]
    assert fit.shape[0] == P
    h, lo, hi = (np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (G,)))
                 for a in (h, lo, hi))
    new = np.empty_like(pop)
    mean = np.empty(P, dtype=np.float64)
    rc = lib.oracle_ga_step(_ptr(pop), _ptr(fit), P, G, R, int(elite), float(pm0), _ptr(h),
                            _ptr(lo), _ptr(hi), int(gen), int(generations),
                            int(ga_seed) & ((1 << 64) - 1), _ptr(new), _ptr(mean))
    if rc != 0:
        raise ValueError("oracle_ga_step failed")
    return new, mean


def ignition_cell(gx: float, gy: float, W: int, H: int):
    """The lattice cell of an individual's ignition genes (Appendix B, 7
    parameters): the paper treats the coordinates as real parameters
    without saying how a simulation starts from them; the reading here is
    the nearest cell, halves rounded up (floor(g + 1/2)), clamped to the
    lattice."""
    x = int(np.floor(gx + 0.5))
    y = int(np.floor(gy + 0.5))
    return min(max(x, 0), W - 1), min(max(y, 0), H - 1)


def _sample_sd(x: np.ndarray, axis=None) -> np.ndarray:
    """Standard deviation with the n-1 denominator (0 for a single value)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[axis] if axis is not None else x.size
    if n <= 1:
        return np.zeros(np.delete(x.shape, axis) if axis is not None else ())
    m = x.mean(axis=axis, keepdims=True)
    return np.sqrt(((x - m) ** 2).sum(axis=axis) / (n - 1))


def ensemble(params: np.ndarray, deltas: np.ndarray, cutoff: float):
    """Best fit and spread of the accepted ensemble.

    params[k] are the parameters of simulation k and deltas[k] its Eq. 2
    fitness. The best set is the one with the minimum fitness (first on ties);
    the accepted ensemble holds the simulations with fitness below ``cutoff``
    and its spread is the per-parameter standard deviation (n-1 denominator).
    """
    params = np.asarray(params, dtype=np.float64)
    deltas = np.asarray(deltas, dtype=np.float64)
    best = int(np.argmin(deltas))
    acc = deltas < cutoff
    spread = _sample_sd(params[acc], axis=0) if acc.sum() > 1 else np.zeros(params.shape[1])
    mean = params[acc].mean(axis=0) if acc.any() else np.full(params.shape[1], np.nan)
    return {"best_index": best, "best_params": params[best], "best_fitness": float(deltas[best]),
            "n_accepted": int(acc.sum()), "accepted_mean": mean, "spread": spread}


def scan_reduce(deltas: np.ndarray, cutoff: float, tau: float = 0.1):
    """Per-candidate ignition statistics over replicate fitness values.

    deltas is [n_candidates][R]. Returns mean, sd (n-1), acceptance rate
    #(delta < cutoff)/R and a normalised map: acceptance / sum(acceptance), or,
    when no replicate of any candidate is accepted, softmin weights
    exp(-mean/tau) normalised to 1.
    """
    d = np.asarray(deltas, dtype=np.float64)
    mean = d.mean(axis=1)
    sd = _sample_sd(d, axis=1)
    acc = (d < cutoff).sum(axis=1) / d.shape[1]
    if acc.sum() > 0:
        post = acc / acc.sum()
    else:
        w = np.exp(-(mean - mean.min()) / tau)
        post = w / w.sum()
    return {"mean": mean, "sd": sd, "accept": acc, "posterior": post}
