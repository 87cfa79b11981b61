"""Per-element tolerances for the GPU surrogate's gradients (test helper).

The GPU evaluates the network with bf16 matrix inputs and fp32 accumulation;
the reference (oracle/surrogate_ref, bf16=True) rounds the same operands to
bf16 at the same points and computes everything else in binary64. Every
gradient element g_ij is the last contraction of a chain,
g_ij = sum_k A_ik B_kj (a weight gradient: activations times back-propagated
errors over the batch; a bias gradient: a column sum; a convolution kernel
gradient: a sum over batch and pixels). With M_ij = sum_k |A_ik| |B_kj| the
magnitude of that contraction (reference operands), the difference between
GPU and reference is bounded per element by

  tol_ij = (rho + 8 sqrt(K) 2^-24 + c_up 2^-8) M_ij

* rho = 4 u (u = 2^-8, the bf16 unit roundoff) when both operands are bf16
  values rounded from an fp32 (GPU) or binary64 (reference) value: the two
  sides round identically unless the value sits within its fp32 error of a
  bf16 rounding midpoint, where they differ by one bf16 ulp (<= 2u |v|); a
  product of two such operands differs by at most (2u + 2u + 4u^2) |a||b|.
  rho = 2 u when one operand is such a bf16 value and the other is exact
  (the bias gradients of the convolutions: sums of bf16 errors); rho = 0
  for fp32 operands (the dense layers' bias gradients).
* 8 sqrt(K) 2^-24: fp32 accumulation of K terms, the probabilistic bound of
  Higham and Mary (SIAM J. Sci. Comput. 41, 2019) at lambda = 8: it holds
  with probability >= 1 - 2K exp(-32), over 1 - 1e-8 for every sum here.
* c_up u: differences carried in from upstream layers. A rounding flip
  upstream changes one term of an upstream sum by one bf16 ulp; such flips
  are rare (a value must lie within ~sqrt(K) 2^-24 of a midpoint, relative)
  and each moves this contraction by a small share of one term. An fp32
  emulation of the network with the GPU's rounding points, over four seeds
  and batches of 6, 7 and 13, moved no element by more than 0.005 u M_ij
  beyond the local terms; c_up = 1/4 leaves a margin of 50.

A ReLU mask can differ between the two sides where the pre-activation lies
within its own error of zero: the pre-activation v counts as near zero when
|v| <= 8 sqrt(K) 2^-24 M_v + f, its own contraction's accumulation bound plus
an allowance f for upstream rounding flips: every layer, dense or
convolution, has bf16 inputs, each flip moves v by one ulp of one of its K
terms, and f = 4u max_k|a_k w_k| allows two. Where it is, the back-propagated value that the
mask gates may be |g| on one side and 0 on the other. Those possible jumps
are carried downstream in absolute value, D (|.| of each later linear map
applied to them, seeded only at the near-zero entries, so D stays sparse),
and every gradient element's tolerance adds sum_k |A_ik| D_kj for its
second operand (the local mask counts as open there).

A worst-case bound propagated element by element through the layers is no
use here: every cancelling sum multiplies it by about sqrt(K), and after four
layers it exceeds the gradients themselves by orders of magnitude.

The tolerance is per element and in units of that element's own magnitude
product, so one wrong element (for instance a wrong column of a bias
gradient) fails unless its error is within a few bf16 ulps of M_ij.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import surrogate_ref as S

U = 2.0 ** -8
U32 = 2.0 ** -24
LAMBDA = 8.0
C_UP = 0.25


def _dK_abs(a, g):
    """Sum over batch and pixels of |g| |a| for every 3x3 kernel tap."""
    K0 = np.zeros((g.shape[1], a.shape[1], 3, 3))
    return S.conv3x3_backward(np.abs(a), K0, np.abs(g))[1]


def _convT_abs(g, K):
    """Data gradient of a 3x3 convolution in absolute values (|K|, |g|)."""
    a = np.zeros((g.shape[0], K.shape[1], g.shape[2], g.shape[3]))
    return S.conv3x3_backward(a, np.abs(K), np.abs(g))[0]


def _max_term(u, K):
    """For every output of conv3x3(u, K): its largest term |u| |K|."""
    B, Ci, S_, _ = u.shape
    p = np.zeros((B, Ci, S_ + 2, S_ + 2))
    p[:, :, 1:-1, 1:-1] = np.abs(u)
    out = np.zeros((B, K.shape[0], S_, S_))
    for dy in range(3):
        for dx in range(3):
            for ci in range(Ci):
                t = p[:, ci, dy:dy + S_, dx:dx + S_][:, None] * \
                    np.abs(K[:, ci, dy, dx])[None, :, None, None]
                np.maximum(out, t, out=out)
    return out


def _near_zero(pre, Mpre, k, flip):
    """Pre-activations within their possible difference of zero: fp32
    accumulation of k terms, plus `flip` (upstream rounding flips)."""
    return np.abs(pre) <= LAMBDA * math.sqrt(k) * U32 * Mpre + flip


def gradient_tolerances(params, x_raw, y_t, y_map, W, H, w_map):
    """Reference gradients (binary64, bf16 matrix inputs), the per-element
    tolerance and the magnitude products M, each flat in parameter order.
    Returns (g_ref, tol, M)."""
    P = S.unflatten(np.asarray(params, dtype=np.float64))
    r = S.round_bf16
    B = x_raw.shape[0]
    c = S.forward(P, x_raw, W, H, bf16=True)
    # masks that may differ: pre-activations within their tolerance of zero
    Wb = {k: r(P[k]) for k in ("W1", "W2", "W3", "Wd")}
    inputs = {"h1": (c["x"], "W1", "c1"), "h2": (r(c["h1"]), "W2", "c2"),
              "h3": (r(c["h2"]), "W3", "c3"), "d0": (r(c["h3"]), "Wd", "cd")}
    near, open_ = {}, {}
    for a, (inb, Wn, cn) in inputs.items():
        pre = inb @ Wb[Wn] + P[cn]
        Mpre = np.abs(inb) @ np.abs(Wb[Wn]) + np.abs(P[cn])
        # two of its bf16 inputs may have rounded the other way, each by one
        # ulp (<= 2u of the term): at most 4u times its largest term
        maxterm = (np.abs(inb)[:, :, None] * np.abs(Wb[Wn])[None, :, :]).max(axis=1)
        near[a] = _near_zero(pre, Mpre, inb.shape[1] + 2, 4 * U * maxterm)
        open_[a] = (pre > 0) | near[a]
    for a, u, Kn, kn in (("d1", c["u0"], "K1", "k1"), ("d2", c["u1"], "K2", "k2")):
        ub, Kb = r(u), r(P[Kn])
        pre = S.conv3x3(ub, Kb, P[kn])
        Mpre = S.conv3x3(np.abs(ub), np.abs(Kb), np.abs(P[kn]))
        near[a] = _near_zero(pre, Mpre, 9 * u.shape[1] + 1, 4 * U * _max_term(ub, Kb))
        open_[a] = (pre > 0) | near[a]
    M = {name: np.zeros(shape) for name, shape in S.layout()}
    extra = {name: np.zeros(shape) for name, shape in S.layout()}
    K = {}
    rho = {}

    dh = np.zeros((B, S.H))
    Dh = np.zeros((B, S.H))  # possible jumps carried from near-zero masks
    h3b = r(c["h3"])
    if y_map is not None and w_map > 0:
        z = c["z"]
        y = np.asarray(y_map, dtype=np.float64).reshape(z.shape)
        dz = w_map * (1.0 / (1.0 + np.exp(-z)) - y) / z.size
        # the convolutions take their inputs, kernels and errors as bf16
        dzb = r(dz)[:, None]
        du2 = S.conv3x3_backward(r(c["u2"]), r(P["K3"]), dzb)[0]
        M["K3"], M["k3"] = _dK_abs(r(c["u2"]), dzb), np.abs(dzb).sum(axis=(0, 2, 3))
        g2 = S.downsample2_sum(du2)
        dd2 = g2 * (c["d2"] > 0)
        D2 = np.abs(g2) * near["d2"]
        dd2b = r(dd2)
        du1 = S.conv3x3_backward(r(c["u1"]), r(P["K2"]), dd2b)[0]
        M["K2"] = _dK_abs(r(c["u1"]), np.abs(dd2b) + D2)
        M["k2"] = (np.abs(dd2b) + D2).sum(axis=(0, 2, 3))
        g1 = S.downsample2_sum(du1)
        dd1 = g1 * (c["d1"] > 0)
        D1 = (S.downsample2_sum(_convT_abs(D2, r(P["K2"]))) * open_["d1"]
              + np.abs(g1) * near["d1"])
        dd1b = r(dd1)
        du0 = S.conv3x3_backward(r(c["u0"]), r(P["K1"]), dd1b)[0]
        M["K1"] = _dK_abs(r(c["u0"]), np.abs(dd1b) + D1)
        M["k1"] = (np.abs(dd1b) + D1).sum(axis=(0, 2, 3))
        for layer, side in ((1, 32), (2, 64), (3, 128)):
            K[f"K{layer}"] = K[f"k{layer}"] = B * side * side
            rho[f"K{layer}"], rho[f"k{layer}"] = 4 * U, 2 * U
        g0 = S.downsample2_sum(du0).reshape(B, -1)
        dd0 = g0 * (c["d0"] > 0)
        D0 = (S.downsample2_sum(_convT_abs(D1, r(P["K1"]))).reshape(B, -1) * open_["d0"]
              + np.abs(g0) * near["d0"])
        dd0b = r(dd0)
        M["Wd"], K["Wd"], rho["Wd"] = np.abs(h3b).T @ np.abs(dd0b), B, 4 * U
        extra["Wd"] = np.abs(h3b).T @ D0
        M["cd"], K["cd"] = np.abs(dd0).sum(axis=0), B
        extra["cd"] = D0.sum(axis=0)
        dh = dh + dd0b @ r(P["Wd"]).T
        Dh = Dh + D0 @ np.abs(r(P["Wd"])).T
    dt = 2.0 * (c["t"] - np.asarray(y_t, dtype=np.float64)) / B
    dtb = r(dt)
    M["Wf"], K["Wf"], rho["Wf"] = np.abs(h3b).T @ np.abs(dtb)[:, None], B, 4 * U
    M["cf"], K["cf"] = np.array([np.abs(dt).sum()]), B
    dh = dh + dtb[:, None] @ r(P["Wf"]).T
    for Wn, cn, inb, act, a in [("W3", "c3", r(c["h2"]), c["h3"], "h3"),
                                ("W2", "c2", r(c["h1"]), c["h2"], "h2"),
                                ("W1", "c1", c["x"], c["h1"], "h1")]:
        dp = dh * (act > 0)
        Dp = Dh * open_[a] + np.abs(dh) * near[a]
        dpb = r(dp)
        M[Wn], K[Wn], rho[Wn] = np.abs(inb).T @ np.abs(dpb), B, 4 * U
        extra[Wn] = np.abs(inb).T @ Dp
        M[cn], K[cn] = np.abs(dp).sum(axis=0), B
        extra[cn] = Dp.sum(axis=0)
        dh = dpb @ r(P[Wn]).T
        Dh = Dp @ np.abs(r(P[Wn])).T
    tol = {name: (rho.get(name, 0.0) + LAMBDA * math.sqrt(K.get(name, 1)) * U32 + C_UP * U)
           * M[name] + (1.0 + C_UP * U) * extra[name] for name, _ in S.layout()}
    _, _, g_ref = S.loss_and_grads(np.asarray(params, dtype=np.float64), x_raw, y_t, y_map, W, H,
                                   w_map, bf16=True)
    return g_ref, S.flatten(tol), S.flatten(M)
