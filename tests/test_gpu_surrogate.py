"""GPU checks of the learned surrogate (through the C ABI in fire_nn.h).

* the MFMA bf16 GEMM against binary64 products of the same bf16 inputs, for
  every transpose pattern the network uses and each way an operand's tile is
  loaded (16-byte loads along k or along rows, element by element), ragged
  sizes and the epilogues;
* burn-map pooling against numpy;
* loss and every parameter gradient of the whole network against the
  binary64 reference with the same bf16 rounding points (oracle/surrogate_ref),
  element by element, each within a tolerance derived from its own magnitude
  product (tests/surrogate_bounds.py);
* the bias-gradient column sums in their fixed order, exactly;
* Adam training on a fixed batch lowers the loss;
* the pipeline's data movers (rows from simulator results, row gathers,
  screening candidates) against numpy.
"""
import numpy as np
import pytest

from gpu_util import say
from oracle import surrogate_ref as S

pytestmark = pytest.mark.gpu


def _bf16_tensor(a):
    import torch
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).cuda().to(torch.bfloat16)


def _bits(t):
    import torch
    return t.view(torch.int16)


@pytest.mark.parametrize("M,N,K,ta,tb", [(64, 64, 32, 0, 0), (100, 37, 70, 0, 0),
                                          (256, 16, 513, 1, 0), (33, 300, 17, 0, 1),
                                          (7, 1, 256, 0, 0), (256, 2048, 9, 1, 0),
                                          (130, 257, 129, 1, 1), (96, 80, 64, 0, 1),
                                          (72, 136, 40, 1, 1), (512, 256, 256, 0, 0),
                                          (256, 256, 512, 1, 0)])
def test_gemm_bf16_against_binary64(M, N, K, ta, tb):
    import torch
    from paper_1701_03549_amd import nn
    say(f"gemm {M}x{N}x{K} ta={ta} tb={tb}")
    rng = np.random.default_rng(M * N + K)
    a = S.round_bf16(rng.normal(size=(M, K)))
    b = S.round_bf16(rng.normal(size=(K, N)))
    bias = rng.normal(size=N).astype(np.float32)
    A = _bf16_tensor(a.T.copy() if ta else a)
    Bm = _bf16_tensor(b.T.copy() if tb else b)
    sam, sak = (1, M) if ta else (K, 1)
    sbk, sbn = (1, K) if tb else (N, 1)
    C = torch.full((M, N), 0.5, dtype=torch.float32, device="cuda")
    Cb = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")
    nn.gemm_bf16(_bits(A), _bits(Bm), M, N, K, sam, sak, sbk, sbn, C, N,
                 bias=torch.from_numpy(bias).cuda(), relu=True, accumulate=True, Cb=_bits(Cb))
    torch.cuda.synchronize()
    want = np.maximum(a @ b + bias + 0.5, 0.0)
    got = C.cpu().numpy().astype(np.float64)
    # fp32 accumulation of K products of bf16 values
    tol = 1e-5 * np.sqrt(K) * (np.abs(a) @ np.abs(b) + 1.0)
    assert np.all(np.abs(got - want) <= tol)
    assert np.array_equal(Cb.float().cpu().numpy(), S.round_bf16(got).astype(np.float32))


def test_pool_maps():
    import torch
    from paper_1701_03549_amd import nn, synth
    rng = np.random.default_rng(3)
    W, H, n = 256, 200, 5
    m = rng.random((n, H, W)) < 0.01
    packed = np.stack([synth.pack_bits(x) for x in m])
    mw = packed.shape[1] * packed.shape[2]
    t = torch.from_numpy(packed.reshape(n, -1).view(np.int32)).cuda()
    say("pool maps")
    out = nn.pool_maps(t, n, W, H, mw, 128, 100).cpu().numpy()
    want = m.reshape(n, 100, 2, 128, 2).any(axis=(2, 4))
    assert np.array_equal(out.astype(bool), want)


def _random_problem(B, seed, W=256, H=256):
    rng = np.random.default_rng(seed)
    x = np.column_stack([rng.uniform(-10, 10, size=(B, 5)), rng.integers(0, W, B),
                         rng.integers(0, H, B)]).astype(np.float32)
    y_t = rng.uniform(0, 3, size=B).astype(np.float32)
    y_map = (rng.random((B, 128, 128)) < 0.2).astype(np.uint8)
    return x, y_t, y_map


def _surrogate_instance(seed, bias_lo, bias_hi):
    """Flat fp32 parameters: weights as initialised by the library (seed 11),
    biases drawn in [bias_lo, bias_hi) so that most ReLUs are active."""
    import torch
    from paper_1701_03549_amd import nn
    net = nn.Surrogate(max_batch=64, lattice=(256, 256), w_map=0.5, seed=11)
    p = net.get_params().cpu().numpy().astype(np.float64)
    d = S.unflatten(p)
    rng = np.random.default_rng(seed)
    for k in ("c1", "c2", "c3", "cd", "k1", "k2"):
        d[k] = rng.uniform(bias_lo, bias_hi, size=d[k].shape)
    p = S.flatten(d).astype(np.float32)
    net.set_params(torch.from_numpy(p))
    return net, p


@pytest.mark.parametrize("B,seed,blo,bhi", [(6, 4, 0.02, 0.1), (13, 8, 0.02, 0.1), (7, 9, 0.3, 0.5)])
def test_gradients_match_reference_per_element(B, seed, blo, bhi):
    """Every gradient element within its own tolerance (tests/surrogate_bounds:
    a few bf16 ulps of that element's magnitude product, plus the possible
    jumps of ReLU masks whose pre-activation is within its error of zero)."""
    import torch
    import surrogate_bounds as SB
    W = H = 256
    net, p = _surrogate_instance(seed, blo, bhi)
    x, y_t, y_map = _random_problem(B, seed + 1, W, H)
    say(f"surrogate gradients B={B}")
    loss, g = net.gradients(torch.from_numpy(x), torch.from_numpy(y_t),
                            torch.from_numpy(y_map).cuda())
    torch.cuda.synchronize()
    g_ref, tol, M = SB.gradient_tolerances(p.astype(np.float64), x, y_t, y_map, W, H, 0.5)
    lf, lm, _ = S.loss_and_grads(p.astype(np.float64), x, y_t, y_map, W, H, 0.5, bf16=True)
    loss = loss.cpu().numpy()
    assert abs(loss[0] - lf) <= 1e-3 * abs(lf) + 1e-6
    assert abs(loss[1] - lm) <= 1e-3 * abs(lm) + 1e-6
    g = g.cpu().numpy().astype(np.float64)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in S.layout()])
    bad = []
    for (name, _), o0, o1 in zip(S.layout(), offs[:-1], offs[1:]):
        d = np.abs(g[o0:o1] - g_ref[o0:o1])
        over = np.nonzero(d > tol[o0:o1])[0]
        ref = np.abs(g_ref[o0:o1])
        nz = ref > 0
        power = float(np.mean(0.1 * ref[nz] > tol[o0:o1][nz])) if nz.any() else 0.0
        say(f"  {name}: max |d|/tol {np.max(d / np.maximum(tol[o0:o1], 1e-300)):.3f}, "
            f"a 10% error detectable in {power:.0%} of elements")
        if over.size:
            k = int(over[0])
            bad.append(f"{name}[{k}]: gpu {g[o0 + k]!r} ref {g_ref[o0 + k]!r} tol {tol[o0 + k]:.3e}")
    assert not bad, f"{len(bad)} tensors with elements out of tolerance: {bad[:4]}"
    # forward agrees too
    t, mp = net.forward(torch.from_numpy(x), want_map=True)
    c = S.forward(p.astype(np.float64), x, W, H, bf16=True)
    assert np.allclose(t.cpu().numpy(), c["t"], rtol=1e-2, atol=1e-3)
    assert np.allclose(mp.cpu().numpy(), 1 / (1 + np.exp(-c["z"])), atol=2e-3)
    net.close()


@pytest.mark.parametrize("M,N", [(1, 1), (6, 256), (13, 1), (7, 2048), (5, 100), (64, 65), (4, 64),
                                 (512, 256), (37, 17)])
def test_colsum_order_and_values(M, N):
    """Bias-gradient column sums: integer data (every partial sum exact in
    fp32) equals the binary64 sum exactly; random data equals the sum in
    the fixed order (rows r, r+16, ... per group r = 0..15, then a pairwise
    tree over the 16 partial sums) evaluated in fp32, bit for bit."""
    import torch
    from paper_1701_03549_amd import nn
    rng = np.random.default_rng(M * 1000 + N)
    ints = rng.integers(-1000, 1000, size=(M, N)).astype(np.float32)
    got = nn.colsum(torch.from_numpy(ints).cuda()).cpu().numpy()
    assert np.array_equal(got.astype(np.float64), ints.astype(np.float64).sum(axis=0))
    x = rng.normal(size=(M, N)).astype(np.float32)
    got = nn.colsum(torch.from_numpy(x).cuda()).cpu().numpy()
    parts = []
    for r in range(16):
        acc = np.zeros(N, dtype=np.float32)
        for m in range(r, M, 16):
            acc = (acc + x[m]).astype(np.float32)
        parts.append(acc)
    while len(parts) > 1:
        parts = [(parts[2 * i] + parts[2 * i + 1]).astype(np.float32)
                 for i in range(len(parts) // 2)]
    want = parts[0]
    assert np.array_equal(got, want.astype(np.float32))
    np.testing.assert_allclose(got, x.astype(np.float64).sum(axis=0),
                               rtol=0, atol=1e-5 * np.abs(x).sum(axis=0).max())


def test_training_lowers_loss():
    import torch
    from paper_1701_03549_amd import nn
    B = 64
    net = nn.Surrogate(max_batch=B, lattice=(256, 256), w_map=1.0, seed=3)
    x, _, _ = _random_problem(B, 9)
    # a smooth target of the inputs and a map that depends on the ignition
    y_t = (np.tanh(x[:, 0] / 10.0) + 0.5 * np.cos(x[:, 1] / 5.0) + 1.5).astype(np.float32)
    yy, xx = np.mgrid[0:128, 0:128]
    y_map = np.stack([((xx - xi / 2) ** 2 + (yy - yi / 2) ** 2 < 400) for xi, yi in x[:, 5:7]])
    xt = torch.from_numpy(x).cuda()
    yt = torch.from_numpy(y_t).cuda()
    ym = torch.from_numpy(y_map.astype(np.uint8)).cuda()
    say("surrogate training")
    first = net.train_step(xt, yt, ym, lr=1e-3).cpu().numpy()
    for _ in range(150):
        last = net.train_step(xt, yt, ym, lr=1e-3)
    last = last.cpu().numpy()
    assert last[0] < 0.2 * first[0]
    assert last[1] < first[1]
    net.close()


@pytest.mark.parametrize("n,reps,per_row_ign", [(1, 1, True), (777, 1, True), (1280, 20, False),
                                                 (4096, 4096, True)])
def test_rows_from_results(n, reps, per_row_ign):
    """Network rows from simulator results against numpy: parameters of row
    i // reps rounded to fp32, the ignition, log(1 + delta) (within one fp32
    unit: the two libraries' binary64 log1p may differ in the last place)
    and delta copied bit for bit; NaN fitness (no target) gives NaN."""
    import torch
    from paper_1701_03549_amd import fire, nn
    rng = np.random.default_rng(n + reps)
    n_par = (n + reps - 1) // reps
    params = rng.uniform(-30, 30, (n_par, 5))
    res = np.zeros(n, dtype=fire.RESULT_DTYPE)
    res["fitness"] = rng.uniform(0, 3, n) ** 3
    res["fitness"][:: 97] = np.nan
    res["fitness"][1:: 89] = 0.0
    ign = rng.integers(0, 1024, (n, 2)).astype(np.float32)
    d_res = torch.from_numpy(res.view(np.uint8).copy()).cuda()
    x = torch.full((n, 7), -1.0, dtype=torch.float32, device="cuda")
    y = torch.full((n,), -1.0, dtype=torch.float32, device="cuda")
    fit = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    say(f"rows from results n={n} reps={reps}")
    nn.rows_from_results(d_res, n, params=torch.from_numpy(params).cuda(), reps=reps,
                         ign=torch.from_numpy(ign).cuda() if per_row_ign else None,
                         ign_xy=(17.0, 23.0), out_x=x, out_y=y, out_fit=fit)
    xh, yh, fh = x.cpu().numpy(), y.cpu().numpy(), fit.cpu().numpy()
    want_x = np.empty((n, 7), np.float32)
    want_x[:, :5] = params[np.arange(n) // reps].astype(np.float32)
    want_x[:, 5:] = ign if per_row_ign else np.array([17.0, 23.0], np.float32)
    assert np.array_equal(xh, want_x)
    assert np.array_equal(fh.view(np.uint64), res["fitness"].view(np.uint64))
    want_y = np.log1p(res["fitness"]).astype(np.float32)
    nan = np.isnan(want_y)
    assert np.array_equal(np.isnan(yh), nan)
    ulp = np.spacing(np.abs(want_y[~nan]))
    assert np.all(np.abs(yh[~nan] - want_y[~nan]) <= ulp)
    # outputs may be omitted
    fit2 = torch.empty((n,), dtype=torch.float64, device="cuda")
    nn.rows_from_results(d_res, n, out_fit=fit2)
    assert np.array_equal(fit2.cpu().numpy().view(np.uint64), fh.view(np.uint64))


@pytest.mark.parametrize("row_shape,dtype", [((7,), "float32"), ((1,), "float32"),
                                             ((128, 128), "uint8"), ((4,), "float64")])
def test_gather_rows(row_shape, dtype):
    """Row gather against numpy fancy indexing: 28-byte rows (4-byte moves),
    4-byte rows, 16 KiB map rows (16-byte moves), repeated and unordered row
    indices, an empty gather."""
    import torch
    from paper_1701_03549_amd import nn
    rng = np.random.default_rng(len(row_shape) * 7 + row_shape[0])
    N = 3000
    src = rng.integers(0, 255, (N,) + row_shape).astype(dtype)
    rows = rng.integers(0, N, 1111).astype(np.int64)
    rows[:5] = [0, N - 1, 7, 7, 0]
    d_src = torch.from_numpy(src).cuda()
    out = torch.zeros((len(rows),) + row_shape, dtype=d_src.dtype, device="cuda")
    say(f"gather rows {row_shape} {dtype}")
    nn.gather_rows(d_src, torch.from_numpy(rows).cuda(), out)
    assert np.array_equal(out.cpu().numpy(), src[rows])
    nn.gather_rows(d_src, torch.zeros(0, dtype=torch.int64, device="cuda"), out)
    assert np.array_equal(out.cpu().numpy(), src[rows])


@pytest.mark.parametrize("S,P,E", [(1, 64, 2), (8, 64, 2), (3, 5, 0), (4, 10, 9)])
def test_candidates(S, P, E):
    """Screening candidates against numpy: all of set 0, then rows E.. of
    every later set, and their fp32 network inputs with the ignition."""
    import torch
    from paper_1701_03549_amd import nn
    rng = np.random.default_rng(S * 100 + P + E)
    sets = rng.normal(0, 5, (S, P, 5))
    n = P + (S - 1) * (P - E)
    cand = torch.zeros((n, 5), dtype=torch.float64, device="cuda")
    x = torch.zeros((n, 7), dtype=torch.float32, device="cuda")
    say(f"candidates S={S} P={P} E={E}")
    nn.candidates(torch.from_numpy(sets).cuda(), E, (256.0, 259.0), cand, x)
    want = np.concatenate([sets[0]] + [sets[o][E:] for o in range(1, S)])
    assert np.array_equal(cand.cpu().numpy(), want)
    want_x = np.column_stack([want.astype(np.float32), np.full((n, 2), [256.0, 259.0], np.float32)])
    assert np.array_equal(x.cpu().numpy(), want_x)
