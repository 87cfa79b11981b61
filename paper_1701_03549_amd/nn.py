"""Python binding of include/fire_nn.h (argument marshalling only): the
learned surrogate of the simulator, its MFMA GEMM building block and the
burn-map pooling used to build its training targets."""
from __future__ import annotations

import ctypes

import torch

from . import fire

EXPORTS = ["fire_nn_create", "fire_nn_destroy", "fire_nn_last_error", "fire_nn_num_params",
           "fire_nn_get_params", "fire_nn_set_params", "fire_nn_forward", "fire_nn_gradients",
           "fire_nn_train_step", "fire_gemm_bf16", "fire_pool_maps", "fire_nn_select", "fire_colsum_f32",
           "fire_nn_rows_from_results", "fire_gather_rows", "fire_nn_candidates"]
MAP = 128


class NNCfg(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("lattice_w", ctypes.c_int32),
                ("lattice_h", ctypes.c_int32), ("w_map", ctypes.c_float),
                ("adam_b1", ctypes.c_float), ("adam_b2", ctypes.c_float),
                ("adam_eps", ctypes.c_float)]


_done = False


def _lib():
    global _done
    lib = fire.load_library()
    if _done:
        return lib
    vp, i32, i64, u64, f32 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                              ctypes.c_float)
    sig = {
        "fire_nn_create": (i32, [ctypes.c_int, ctypes.POINTER(NNCfg), u64, ctypes.POINTER(vp)]),
        "fire_nn_destroy": (None, [vp]),
        "fire_nn_last_error": (ctypes.c_char_p, [vp]),
        "fire_nn_num_params": (i64, [vp]),
        "fire_nn_get_params": (i32, [vp, vp, vp]),
        "fire_nn_set_params": (i32, [vp, vp, vp]),
        "fire_nn_forward": (i32, [vp, vp, i32, vp, vp, vp]),
        "fire_nn_gradients": (i32, [vp, vp, vp, vp, i32, vp, vp, vp]),
        "fire_nn_train_step": (i32, [vp, vp, vp, vp, i32, f32, i32, vp, vp]),
        "fire_gemm_bf16": (i32, [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, i64, i64, vp, i64,
                                 i64, vp, i64, vp, ctypes.c_int, ctypes.c_int, vp, vp]),
        "fire_pool_maps": (i32, [vp, i32, i32, i32, i64, i32, i32, vp, vp]),
        "fire_nn_select": (i32, [vp, vp, i32, i32, i32, i32, vp, vp, vp]),
        "fire_colsum_f32": (i32, [vp, i32, i32, vp, vp]),
        "fire_nn_rows_from_results": (i32, [vp, i32, vp, f32, f32, vp, i32, vp, vp, vp, vp]),
        "fire_gather_rows": (i32, [vp, i64, vp, i32, vp, vp]),
        "fire_nn_candidates": (i32, [vp, i32, i32, i32, f32, f32, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _done = True
    return lib


def _p(t):
    return 0 if t is None else int(t.data_ptr())


def _s(stream=None):
    return fire._stream(stream)


def gemm_bf16(A, Bm, M, N, K, sam, sak, sbk, sbn, C, ldc, bias=None, relu=False,
              accumulate=False, Cb=None, stream=None):
    """C = op(A) op(B) (+ bias) (+ C); A, B bf16 tensors (any shape, strides
    given in elements), C fp32."""
    lib = _lib()
    st = lib.fire_gemm_bf16(M, N, K, _p(A), sam, sak, _p(Bm), sbk, sbn, _p(C), ldc, _p(bias),
                            int(relu), int(accumulate), _p(Cb), _s(stream))
    if st != 0:
        raise fire.FireError(st, "fire_gemm_bf16 failed")


def pool_maps(maps: torch.Tensor, n: int, W: int, H: int, map_words: int, out_w=MAP, out_h=MAP,
              stream=None) -> torch.Tensor:
    lib = _lib()
    out = torch.empty((n, out_h, out_w), dtype=torch.uint8, device=maps.device)
    st = lib.fire_pool_maps(_p(maps), n, W, H, map_words, out_w, out_h, _p(out), _s(stream))
    if st != 0:
        raise fire.FireError(st, "fire_pool_maps failed")
    return out


def colsum(d: torch.Tensor, stream=None) -> torch.Tensor:
    """Column sums of a [M][N] fp32 device matrix in the backward pass's order."""
    lib = _lib()
    d = d.contiguous()
    M, N = d.shape
    out = torch.empty(N, dtype=torch.float32, device=d.device)
    st = lib.fire_colsum_f32(_p(d), M, N, _p(out), _s(stream))
    if st != 0:
        raise fire.FireError(st, "fire_colsum_f32 failed")
    return out


def select(cand: torch.Tensor, score: torch.Tensor, keep: int, k: int, out=None, stream=None):
    """Keep the first `keep` rows, then the k - keep lowest-score rows
    (into `out` [k][G] when given)."""
    lib = _lib()
    n, G = cand.shape
    if out is None:
        out = torch.empty((k, G), dtype=torch.float64, device=cand.device)
    assert out.shape == (k, G) and out.dtype == torch.float64 and out.is_contiguous()
    idx = torch.empty(k, dtype=torch.int32, device=cand.device)
    st = lib.fire_nn_select(_p(cand.contiguous()), _p(score.contiguous()), n, G, keep, k, _p(out),
                            _p(idx), _s(stream))
    if st != 0:
        raise fire.FireError(st, "fire_nn_select failed")
    return out, idx


def rows_from_results(results: torch.Tensor, n: int, params=None, reps: int = 1, ign=None,
                      ign_xy=(0.0, 0.0), out_x=None, out_y=None, out_fit=None, stream=None):
    """fire_nn_rows_from_results: network input rows [n][7], targets
    log(1 + delta) [n] and the fitness [n] of n simulator results (any of
    the outputs may be omitted)."""
    for t, shape, dt in ((out_x, (n, 7), torch.float32), (out_y, (n,), torch.float32),
                         (out_fit, (n,), torch.float64), (ign, (n, 2), torch.float32)):
        if t is not None:
            assert t.numel() == shape[0] * (shape[1] if len(shape) > 1 else 1) and t.dtype == dt \
                and t.is_contiguous()
    if params is not None:
        assert params.dtype == torch.float64 and params.is_contiguous() \
            and params.numel() >= 5 * ((n + reps - 1) // reps)
    assert results.numel() >= 24 * n
    st = _lib().fire_nn_rows_from_results(_p(params), int(reps), _p(ign), float(ign_xy[0]),
                                          float(ign_xy[1]), _p(results), int(n), _p(out_x),
                                          _p(out_y), _p(out_fit), _s(stream))
    if st != 0:
        raise fire.FireError(st, "fire_nn_rows_from_results failed")


def gather_rows(src: torch.Tensor, rows: torch.Tensor, out: torch.Tensor, stream=None):
    """fire_gather_rows: out[k] = src[rows[k]] for row-major contiguous
    tensors with rows of the same byte size."""
    n = rows.numel()
    row_bytes = src[0].numel() * src.element_size()
    assert src.is_contiguous() and out.is_contiguous() and rows.dtype == torch.int64
    assert out.shape[0] >= n and out[0].numel() * out.element_size() == row_bytes
    st = _lib().fire_gather_rows(_p(src), int(row_bytes), _p(rows.contiguous()), int(n), _p(out),
                                 _s(stream))
    if st != 0:
        raise fire.FireError(st, "fire_gather_rows failed")


def candidates(sets: torch.Tensor, E: int, ign_xy, cand: torch.Tensor, x: torch.Tensor,
               stream=None):
    """fire_nn_candidates: screening candidates [P + (S-1)(P-E)][5] and their
    network inputs from S offspring sets [S][P][5]."""
    S, P, G = sets.shape
    n = P + (S - 1) * (P - E)
    assert G == 5 and sets.dtype == torch.float64 and sets.is_contiguous()
    assert cand.shape == (n, 5) and x.shape == (n, 7) and cand.is_contiguous() and x.is_contiguous()
    st = _lib().fire_nn_candidates(_p(sets), int(S), int(P), int(E), float(ign_xy[0]),
                                   float(ign_xy[1]), _p(cand), _p(x), _s(stream))
    if st != 0:
        raise fire.FireError(st, "fire_nn_candidates failed")


class Surrogate:
    """A fire_nn handle: forward, gradients, Adam steps."""

    def __init__(self, device=0, max_batch=512, lattice=(256, 256), w_map=1.0, seed=1,
                 adam=(0.9, 0.999, 1e-8)):
        self.lib = _lib()
        self.device = torch.device("cuda", device)
        cfg = NNCfg(int(max_batch), int(lattice[0]), int(lattice[1]), float(w_map),
                    float(adam[0]), float(adam[1]), float(adam[2]))
        h = ctypes.c_void_p()
        st = self.lib.fire_nn_create(device, ctypes.byref(cfg), int(seed) & (2 ** 64 - 1),
                                     ctypes.byref(h))
        if st != 0:
            raise fire.FireError(st, "fire_nn_create failed")
        self.h = h
        self.max_batch = int(max_batch)
        self.num_params = int(self.lib.fire_nn_num_params(h))
        self.steps = 0
        self._args = dict(device=device, max_batch=max_batch, lattice=tuple(lattice),
                          w_map=w_map, seed=seed, adam=tuple(adam))

    def clone(self) -> "Surrogate":
        """A new handle with this one's configuration and parameters and a
        fresh optimiser (zero Adam moments, step count 0)."""
        c = Surrogate(**self._args)
        c.set_params(self.get_params())
        torch.cuda.synchronize()
        return c

    def close(self):
        if getattr(self, "h", None):
            self.lib.fire_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise fire.FireError(st, self.lib.fire_nn_last_error(self.h).decode())

    def get_params(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.num_params, dtype=torch.float32, device=self.device)
        self._check(self.lib.fire_nn_get_params(self.h, _p(out), _s(stream)))
        return out

    def set_params(self, p: torch.Tensor, stream=None):
        p = p.to(self.device, torch.float32).contiguous()
        self._check(self.lib.fire_nn_set_params(self.h, _p(p), _s(stream)))

    def forward(self, x: torch.Tensor, want_map=False, stream=None):
        x = x.to(self.device, torch.float32).contiguous()
        B = x.shape[0]
        t = torch.empty(B, dtype=torch.float32, device=self.device)
        m = torch.empty((B, MAP, MAP), dtype=torch.float32, device=self.device) if want_map else None
        self._check(self.lib.fire_nn_forward(self.h, _p(x), B, _p(t), _p(m), _s(stream)))
        return t, m

    def predict(self, x: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Predicted log(1 + delta) for any number of rows of fp32 inputs
        (forward passes of at most max_batch rows, into `out` when given)."""
        assert x.dtype == torch.float32 and x.is_contiguous() and x.device == self.device
        B = x.shape[0]
        if out is None:
            out = torch.empty(B, dtype=torch.float32, device=self.device)
        assert out.numel() == B and out.dtype == torch.float32 and out.is_contiguous()
        for i in range(0, B, self.max_batch):
            nb = min(self.max_batch, B - i)
            self._check(self.lib.fire_nn_forward(self.h, _p(x[i:i + nb]), nb, _p(out[i:i + nb]),
                                                 0, _s(stream)))
        return out

    def gradients(self, x, y_t, y_map=None, stream=None):
        x = x.to(self.device, torch.float32).contiguous()
        y_t = y_t.to(self.device, torch.float32).contiguous()
        B = x.shape[0]
        loss = torch.empty(2, dtype=torch.float32, device=self.device)
        g = torch.empty(self.num_params, dtype=torch.float32, device=self.device)
        self._check(self.lib.fire_nn_gradients(self.h, _p(x), _p(y_t), _p(y_map), B, _p(loss),
                                               _p(g), _s(stream)))
        return loss, g

    def train_step(self, x, y_t, y_map=None, lr=1e-3, out_loss=None, stream=None):
        """One Adam step; the two losses go to `out_loss` (2 fp32) when given."""
        self.steps += 1
        loss = torch.empty(2, dtype=torch.float32, device=self.device) if out_loss is None \
            else out_loss
        assert loss.numel() == 2 and loss.dtype == torch.float32 and loss.is_contiguous()
        self._check(self.lib.fire_nn_train_step(self.h, _p(x), _p(y_t), _p(y_map), x.shape[0],
                                                float(lr), self.steps, _p(loss), _s(stream)))
        return loss
