"""Reference (binary64, numpy) forward and backward of the learned surrogate.

TEST INFRASTRUCTURE. The GPU surrogate (include/fire_nn.h) is checked against
this plain implementation; it shares no code with the HIP sources. The network
is the one fire_nn.h documents: a 7 -> 256 -> 256 -> 256 -> 1 MLP predicting
log(1 + delta) of Eq. 2, and a dense + three (2x nearest upsample, 3x3 conv)
decoder producing 128x128 burn-map logits.

With ``bf16=True`` the inputs of every matrix product and every decoder
convolution (activations, weights and back-propagated errors) are first
rounded to bfloat16 (round-half-even), as the GPU's MFMA kernels consume
them; everything else is binary64. With ``bf16=False`` the network is
evaluated in plain binary64, which the finite-difference test uses to pin
the analytic backward below.
"""
from __future__ import annotations

import numpy as np

H = 256
IN = 16
DEC_C, DEC_S = 8, 16
DEC = DEC_C * DEC_S * DEC_S
MAP = 128


def layout():
    """(name, shape) of the flattened parameter vector, in order."""
    return [("W1", (IN, H)), ("c1", (H,)), ("W2", (H, H)), ("c2", (H,)), ("W3", (H, H)),
            ("c3", (H,)), ("Wf", (H, 1)), ("cf", (1,)), ("Wd", (H, DEC)), ("cd", (DEC,)),
            ("K1", (DEC_C, DEC_C, 3, 3)), ("k1", (DEC_C,)), ("K2", (DEC_C, DEC_C, 3, 3)),
            ("k2", (DEC_C,)), ("K3", (1, DEC_C, 3, 3)), ("k3", (1,))]


def num_params():
    return sum(int(np.prod(s)) for _, s in layout())


def unflatten(flat):
    out, o = {}, 0
    for name, shape in layout():
        n = int(np.prod(shape))
        out[name] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def flatten(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in layout()])


def round_bf16(x):
    """Round binary64 values to the nearest bfloat16 (ties to even), through
    binary32 as the GPU holds them."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def prep_input(x_raw, W, H_):
    """Raw (beta[5], x, y) -> network input, zero-padded to 16 columns."""
    x_raw = np.asarray(x_raw, dtype=np.float64)
    B = x_raw.shape[0]
    x = np.zeros((B, IN))
    x[:, :5] = x_raw[:, :5] / 30.0
    x[:, 5] = 2.0 * x_raw[:, 5] / W - 1.0
    x[:, 6] = 2.0 * x_raw[:, 6] / H_ - 1.0
    return x


def upsample2(a):
    return a.repeat(2, axis=2).repeat(2, axis=3)


def conv3x3(a, K, k):
    """Zero-padded 3x3 convolution: a [B][Ci][S][S], K [Co][Ci][3][3]."""
    B, Ci, S, _ = a.shape
    p = np.zeros((B, Ci, S + 2, S + 2))
    p[:, :, 1:-1, 1:-1] = a
    out = np.zeros((B, K.shape[0], S, S)) + k[None, :, None, None]
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("bcyx,oc->boyx", p[:, :, dy:dy + S, dx:dx + S], K[:, :, dy, dx])
    return out


def conv3x3_backward(a, K, g):
    """Gradients of conv3x3 w.r.t. its input, kernel and bias."""
    B, Ci, S, _ = a.shape
    p = np.zeros((B, Ci, S + 2, S + 2))
    p[:, :, 1:-1, 1:-1] = a
    dp = np.zeros_like(p)
    dK = np.zeros_like(K)
    for dy in range(3):
        for dx in range(3):
            dK[:, :, dy, dx] = np.einsum("boyx,bcyx->oc", g, p[:, :, dy:dy + S, dx:dx + S])
            dp[:, :, dy:dy + S, dx:dx + S] += np.einsum("boyx,oc->bcyx", g, K[:, :, dy, dx])
    return dp[:, :, 1:-1, 1:-1], dK, g.sum(axis=(0, 2, 3))


def forward(params, x_raw, W, H_, bf16=True):
    P = unflatten(params) if not isinstance(params, dict) else params
    r = round_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    c = {}
    c["x"] = r(prep_input(x_raw, W, H_))
    c["h1"] = np.maximum(c["x"] @ r(P["W1"]) + P["c1"], 0.0)
    c["h2"] = np.maximum(r(c["h1"]) @ r(P["W2"]) + P["c2"], 0.0)
    c["h3"] = np.maximum(r(c["h2"]) @ r(P["W3"]) + P["c3"], 0.0)
    c["t"] = (r(c["h3"]) @ r(P["Wf"]) + P["cf"])[:, 0]
    c["d0"] = np.maximum(r(c["h3"]) @ r(P["Wd"]) + P["cd"], 0.0)
    B = c["d0"].shape[0]
    d0 = c["d0"].reshape(B, DEC_C, DEC_S, DEC_S)
    c["u0"] = upsample2(d0)
    c["d1"] = np.maximum(conv3x3(r(c["u0"]), r(P["K1"]), P["k1"]), 0.0)
    c["u1"] = upsample2(c["d1"])
    c["d2"] = np.maximum(conv3x3(r(c["u1"]), r(P["K2"]), P["k2"]), 0.0)
    c["u2"] = upsample2(c["d2"])
    c["z"] = conv3x3(r(c["u2"]), r(P["K3"]), P["k3"])[:, 0]
    return c


def downsample2_sum(g):
    B, C, S, _ = g.shape
    return g.reshape(B, C, S // 2, 2, S // 2, 2).sum(axis=(3, 5))


def loss_and_grads(params, x_raw, y_t, y_map, W, H_, w_map, bf16=True):
    """Loss (fitness, map) and the gradient of their sum w.r.t. the flat
    parameters, through the same bf16-rounded matrix inputs as forward()."""
    P = unflatten(params)
    r = round_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    c = forward(P, x_raw, W, H_, bf16=bf16)
    B = c["t"].shape[0]
    y_t = np.asarray(y_t, dtype=np.float64)
    e = c["t"] - y_t
    loss_fit = float(np.mean(e ** 2))
    g = {name: np.zeros(shape) for name, shape in layout()}
    dt = 2.0 * e / B
    dh3 = np.zeros((B, H))
    loss_map = 0.0
    if y_map is not None and w_map > 0:
        z = c["z"]
        y = np.asarray(y_map, dtype=np.float64).reshape(z.shape)
        n = z.size
        loss_map = float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))
        dz = w_map * (1.0 / (1.0 + np.exp(-z)) - y) / n
        # each convolution's back-propagated error enters its two products
        # (data and kernel gradients) and its bias gradient as bf16
        du2, g["K3"], g["k3"] = conv3x3_backward(r(c["u2"]), r(P["K3"]), r(dz[:, None]))
        dd2 = downsample2_sum(du2) * (c["d2"] > 0)
        du1, g["K2"], g["k2"] = conv3x3_backward(r(c["u1"]), r(P["K2"]), r(dd2))
        dd1 = downsample2_sum(du1) * (c["d1"] > 0)
        du0, g["K1"], g["k1"] = conv3x3_backward(r(c["u0"]), r(P["K1"]), r(dd1))
        dd0 = (downsample2_sum(du0).reshape(B, DEC) * (c["d0"] > 0))
        dd0r = r(dd0)
        g["Wd"] = r(c["h3"]).T @ dd0r
        g["cd"] = dd0.sum(axis=0)
        dh3 += dd0r @ r(P["Wd"]).T
    dtr = r(dt)
    g["Wf"] = r(c["h3"]).T @ dtr[:, None]
    g["cf"] = np.array([dt.sum()])
    dh3 += dtr[:, None] @ r(P["Wf"]).T
    dp3 = dh3 * (c["h3"] > 0)
    g["W3"] = r(c["h2"]).T @ r(dp3)
    g["c3"] = dp3.sum(axis=0)
    dp2 = (r(dp3) @ r(P["W3"]).T) * (c["h2"] > 0)
    g["W2"] = r(c["h1"]).T @ r(dp2)
    g["c2"] = dp2.sum(axis=0)
    dp1 = (r(dp2) @ r(P["W2"]).T) * (c["h1"] > 0)
    g["W1"] = c["x"].T @ r(dp1)
    g["c1"] = dp1.sum(axis=0)
    return loss_fit, loss_map, flatten(g)


def total_loss(params, x_raw, y_t, y_map, W, H_, w_map):
    """Binary64 loss of the unrounded network (finite-difference target)."""
    c = forward(params, x_raw, W, H_, bf16=False)
    lf = float(np.mean((c["t"] - np.asarray(y_t)) ** 2))
    if y_map is None or w_map == 0:
        return lf
    z = c["z"]
    y = np.asarray(y_map, dtype=np.float64).reshape(z.shape)
    return lf + w_map * float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))
