"""Pins of the surrogate reference: its analytic backward against central
finite differences of the binary64 loss (no bf16 rounding), the bf16 rounding
rule against known values, and the upsample/convolution pieces against
direct sums."""
import numpy as np

from oracle import surrogate_ref as S


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-scale, scale, size=S.num_params())
    d = S.unflatten(p)
    d["W1"][7:] = 0.0
    for k in ("c1", "c2", "c3", "cd"):
        d[k] = rng.uniform(0.05, 0.2, size=d[k].shape)  # keep most ReLUs active
    return S.flatten(d)


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.0e-3, 0.0])
    r = S.round_bf16(v)
    assert r[0] == 1.0
    assert r[1] == 1.0                    # tie -> even
    assert r[2] == 1.0 + 2 ** -6          # tie -> even (up)
    assert r[3] == -2.5 and r[5] == 0.0
    assert abs(r[4] - 3.0e-3) / 3.0e-3 < 2 ** -8


def test_conv_against_direct_sum():
    rng = np.random.default_rng(0)
    a = rng.normal(size=(2, 3, 5, 5))
    K = rng.normal(size=(4, 3, 3, 3))
    k = rng.normal(size=4)
    out = S.conv3x3(a, K, k)
    b, o, y, x = 1, 2, 0, 4
    want = k[o]
    for ci in range(3):
        for dy in range(3):
            for dx in range(3):
                yy, xx = y + dy - 1, x + dx - 1
                if 0 <= yy < 5 and 0 <= xx < 5:
                    want += K[o, ci, dy, dx] * a[b, ci, yy, xx]
    assert abs(out[b, o, y, x] - want) < 1e-12
    u = S.upsample2(a)
    assert u.shape == (2, 3, 10, 10) and u[1, 2, 7, 3] == a[1, 2, 3, 1]


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = _params(2)
    B, W, H = 3, 128, 96
    x = np.column_stack([rng.uniform(-3, 3, size=(B, 5)), rng.integers(0, W, B), rng.integers(0, H, B)])
    y_t = rng.uniform(0, 2, size=B)
    y_map = (rng.random((B, 128, 128)) < 0.3).astype(np.uint8)
    w_map = 0.7
    lf, lm, g = S.loss_and_grads(p, x, y_t, y_map, W, H, w_map, bf16=False)
    assert abs(lf + w_map * lm - S.total_loss(p, x, y_t, y_map, W, H, w_map)) < 1e-12
    lay = S.layout()
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in lay])
    checked = 0
    for (name, shape), o0, o1 in zip(lay, offs[:-1], offs[1:]):
        idx = rng.choice(np.arange(o0, o1), size=min(3, o1 - o0), replace=False)
        if name == "W1":
            idx = o0 + rng.choice(7 * S.H, size=3, replace=False)
        for i in idx:
            h = 1e-7
            pp, pm = p.copy(), p.copy()
            pp[i] += h
            pm[i] -= h
            fd = (S.total_loss(pp, x, y_t, y_map, W, H, w_map) -
                  S.total_loss(pm, x, y_t, y_map, W, H, w_map)) / (2 * h)
            assert abs(fd - g[i]) <= 1e-6 + 1e-4 * abs(fd), (name, i, fd, g[i])
            checked += 1
    assert checked >= 40
