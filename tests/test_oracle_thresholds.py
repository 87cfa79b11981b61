"""Pins of the oracle's Eq. 1 thresholds.

Eq. 1 (Methods, "Forest Fire Spread Simulation") gives the spread probability
p = 1/(1 + exp(-(b0 + b1 I_f + b2 psi + b3 omega + b4 sigma))) with the
covariates of the target cell. The oracle evaluates it in binary64 and
quantises p to T = round(p * 2^32). Here each table entry is recomputed with
mpmath at 60 digits from the same binary64 inputs (a closed form evaluated to
far more precision than the oracle) and must agree within one unit, and
special landscapes isolate every covariate, its sign and its direction index.
"""
import mpmath
import numpy as np
import pytest

from paper_1701_03549_amd import synth

mpmath.mp.dps = 60
OFFS = [(0, -1), (1, -1), (1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1)]
U32 = 0xFFFFFFFF


def exact_T(beta, i_f, psi, omega, sigma):
    x = (mpmath.mpf(beta[0]) + mpmath.mpf(beta[1]) * i_f + mpmath.mpf(beta[2]) * psi
         + mpmath.mpf(beta[3]) * omega + mpmath.mpf(beta[4]) * sigma)
    p = 1 / (1 + mpmath.exp(-x))
    v = p * mpmath.mpf(2) ** 32
    r = int(mpmath.nint(v))  # round half even
    return min(r, U32)


def mp_cos_deg(a):
    return mpmath.cos(mpmath.mpf(a) * mpmath.pi / 180)


def exact_table(ls, beta, forest=1):
    veg = ls["veg"]
    H, W = veg.shape
    T = np.zeros((H, W, 8), dtype=np.int64)
    for y in range(H):
        for x in range(W):
            for d, (dx, dy) in enumerate(OFFS):
                tx, ty = x + dx, y + dy
                if not (0 <= tx < W and 0 <= ty < H) or veg[ty, tx] == 0:
                    continue
                sl = float(ls["slope_deg"][ty, tx])
                i_f = 1 if veg[ty, tx] == forest else 0
                psi = mp_cos_deg(float(ls["aspect_deg"][ty, tx]) - 315.0) if sl > 5.0 else 0
                omega = mp_cos_deg(float(ls["wind_to_deg"][ty, tx]) - 45.0 * d)
                up = ls["elev_m"][ty, tx] > ls["elev_m"][y, x]
                sigma = mpmath.mpf(sl) / 100 if up else 0
                T[y, x, d] = exact_T(beta, i_f, psi, omega, sigma)
    return T


@pytest.mark.parametrize("beta", [
    (0.0, 0.0, 0.0, 0.0, 0.0),
    (-1.15, -0.5, 0.3, 0.8, 1.0),
    (-5.0, -10.0, 5.0, 18.1, -5.0),
    (3.3, 7.1, -12.5, 2.25, 29.0),
])
def test_table_matches_mpmath(oracle_mod, beta):
    ls = synth.random_small_landscape(9, 7, seed=5)
    T = oracle_mod.thresholds(ls, beta).astype(np.int64)
    ref = exact_table(ls, beta)
    assert np.max(np.abs(T - ref)) <= 1
    # off-by-one only at rare rounding boundaries
    assert np.mean(T != ref) < 0.01


def test_zero_beta_is_exactly_half(oracle_mod):
    ls = synth.random_small_landscape(6, 5, seed=2)
    T = oracle_mod.thresholds(ls, (0, 0, 0, 0, 0))
    valid = exact_table(ls, (0, 0, 0, 0, 0)) > 0
    assert np.all(T[valid] == 1 << 31)
    assert np.all(T[~valid] == 0)


def test_saturation_and_zero(oracle_mod):
    ls = synth.random_small_landscape(6, 5, seed=3, p_blocked=0.0)
    assert np.all(oracle_mod.thresholds(ls, (-1000, 0, 0, 0, 0)) == 0)
    T = oracle_mod.thresholds(ls, (1000, 0, 0, 0, 0))
    # border sources have out-of-lattice targets -> 0; all others saturate
    inner = T[1:-1, 1:-1, :]
    assert np.all(inner == U32)
    assert np.all(T[0, :, 0] == 0) and np.all(T[-1, :, 4] == 0)
    assert np.all(T[:, 0, 6] == 0) and np.all(T[:, -1, 2] == 0)


def test_quantise_rules(oracle_mod):
    q = oracle_mod.quantise
    assert q(0.0) == 0 and q(-0.0) == 0
    assert q(1.0) == U32
    assert q(0.5) == 1 << 31
    assert q(2.0 ** -33) == 0          # 0.5 rounds to even 0
    assert q(3 * 2.0 ** -33) == 2      # 1.5 rounds to even 2
    assert q(1.0 - 2.0 ** -33) == U32  # rounds to 2^32 then saturates
    assert q(1.0 - 2.0 ** -31) == U32 - 1


def _single_edge_landscape(d, veg_t=2, slope=0.0, aspect=0.0, wind=0.0, up=False):
    """3x3 flat landscape; only the neighbour of the centre in direction d burns."""
    ls = synth.uniform_landscape(3, 3, veg_class=0)
    dx, dy = OFFS[d]
    tx, ty = 1 + dx, 1 + dy
    ls["veg"][1, 1] = 2
    ls["veg"][ty, tx] = veg_t
    ls["slope_deg"][ty, tx] = slope
    ls["aspect_deg"][ty, tx] = aspect
    ls["wind_to_deg"][:, :] = wind
    if up:
        ls["elev_m"][ty, tx] = 10.0
    return ls, (tx, ty)


@pytest.mark.parametrize("d", range(8))
def test_direction_index_and_wind(oracle_mod, d):
    # wind blowing toward compass 45*d: omega = +1 exactly for edge d
    beta = (-0.3, 0.0, 0.0, 1.7, 0.0)
    ls, _ = _single_edge_landscape(d, wind=45.0 * d)
    T = oracle_mod.thresholds(ls, beta)
    nz = [dd for dd in range(8) if T[1, 1, dd] != 0]
    assert nz == [d]                        # layout T[y, x, d] keyed by direction
    assert abs(int(T[1, 1, d]) - exact_T(beta, 0, 0, 1, 0)) <= 1
    # wind blowing the opposite way: omega = -1
    ls2, _ = _single_edge_landscape(d, wind=(45.0 * d + 180.0) % 360.0)
    assert abs(int(oracle_mod.thresholds(ls2, beta)[1, 1, d]) - exact_T(beta, 0, 0, -1, 0)) <= 1
    # crosswind: omega = cos(90 deg)
    ls3, _ = _single_edge_landscape(d, wind=(45.0 * d + 90.0) % 360.0)
    ref = exact_T(beta, 0, 0, mp_cos_deg(90.0), 0)
    assert abs(int(oracle_mod.thresholds(ls3, beta)[1, 1, d]) - ref) <= 1


def test_forest_indicator(oracle_mod):
    beta = (-0.4, -2.5, 0.0, 0.0, 0.0)
    for veg_t, i_f in ((1, 1), (2, 0), (3, 0)):
        ls, _ = _single_edge_landscape(2, veg_t=veg_t, wind=0.0)
        T = oracle_mod.thresholds(ls, beta)
        assert abs(int(T[1, 1, 2]) - exact_T(beta, i_f, 0, mp_cos_deg(-90.0), 0)) <= 1
    # forest class is configurable
    ls, _ = _single_edge_landscape(2, veg_t=3, wind=0.0)
    T = oracle_mod.thresholds(ls, beta, forest_class=3)
    assert abs(int(T[1, 1, 2]) - exact_T(beta, 1, 0, mp_cos_deg(-90.0), 0)) <= 1


def test_aspect_covariate(oracle_mod):
    beta = (0.2, 0.0, 1.3, 0.0, 0.0)
    # NW facing, steep: psi = +1; SE facing: psi = -1; not steep: psi = 0
    for aspect, slope, psi in ((315.0, 10.0, 1), (135.0, 10.0, -1), (315.0, 5.0, 0), (45.0, 6.0, None)):
        ls, _ = _single_edge_landscape(4, slope=slope, aspect=aspect)
        T = oracle_mod.thresholds(ls, beta)
        ps = mp_cos_deg(aspect - 315.0) if psi is None else psi
        assert abs(int(T[1, 1, 4]) - exact_T(beta, 0, ps, mp_cos_deg(-180.0), 0)) <= 1


def test_slope_covariate_only_uphill(oracle_mod):
    beta = (-0.7, 0.0, 0.0, 0.0, 3.0)
    ls, _ = _single_edge_landscape(6, slope=4.0, up=True)
    T = oracle_mod.thresholds(ls, beta)
    sig = mpmath.mpf(4.0) / 100
    assert abs(int(T[1, 1, 6]) - exact_T(beta, 0, 0, mp_cos_deg(-270.0), sig)) <= 1
    ls2, _ = _single_edge_landscape(6, slope=4.0, up=False)  # equal elevation
    T2 = oracle_mod.thresholds(ls2, beta)
    assert abs(int(T2[1, 1, 6]) - exact_T(beta, 0, 0, mp_cos_deg(-270.0), 0)) <= 1
    assert T[1, 1, 6] > T2[1, 1, 6]


def test_spread_probability_sum_order(oracle_mod):
    # the binary64 result of the left-to-right sum, compared with mpmath
    beta = (1e-3, 2.5, -7.25, 18.1, -5.0)
    p = oracle_mod.spread_probability(beta, 1.0, 0.25, -0.5, 0.1)
    x = mpmath.mpf(1e-3) + mpmath.mpf(2.5) + mpmath.mpf(-7.25) * mpmath.mpf(0.25) + \
        mpmath.mpf(18.1) * mpmath.mpf(-0.5) + mpmath.mpf(-5.0) * mpmath.mpf(0.1)
    assert abs(p - float(1 / (1 + mpmath.exp(-x)))) < 4e-16
