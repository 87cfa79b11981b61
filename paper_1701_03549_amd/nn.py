"""Python binding of include/fire_nn.h (argument marshalling only): the
learned surrogate of the simulator, its MFMA GEMM building block and the
burn-map pooling used to build its training targets."""
from __future__ import annotations

import ctypes

import torch

from . import fire

EXPORTS = ["fire_nn_create", "fire_nn_destroy", "fire_nn_last_error", "fire_nn_num_params",
           "fire_nn_get_params", "fire_nn_set_params", "fire_nn_forward", "fire_nn_gradients",
           "fire_nn_train_step", "fire_gemm_bf16", "fire_pool_maps", "fire_nn_select", "fire_colsum_f32"]
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


def select(cand: torch.Tensor, score: torch.Tensor, keep: int, k: int, stream=None):
    """Keep the first `keep` rows, then the k - keep lowest-score rows."""
    lib = _lib()
    n, G = cand.shape
    out = torch.empty((k, G), dtype=torch.float64, device=cand.device)
    idx = torch.empty(k, dtype=torch.int32, device=cand.device)
    st = lib.fire_nn_select(_p(cand.contiguous()), _p(score.contiguous()), n, G, keep, k, _p(out),
                            _p(idx), _s(stream))
    if st != 0:
        raise fire.FireError(st, "fire_nn_select failed")
    return out, idx


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

    def predict(self, x: torch.Tensor, stream=None) -> torch.Tensor:
        """Predicted log(1 + delta) for any number of rows (batched)."""
        outs = []
        for i in range(0, x.shape[0], self.max_batch):
            outs.append(self.forward(x[i:i + self.max_batch], stream=stream)[0])
        return torch.cat(outs)

    def gradients(self, x, y_t, y_map=None, stream=None):
        x = x.to(self.device, torch.float32).contiguous()
        y_t = y_t.to(self.device, torch.float32).contiguous()
        B = x.shape[0]
        loss = torch.empty(2, dtype=torch.float32, device=self.device)
        g = torch.empty(self.num_params, dtype=torch.float32, device=self.device)
        self._check(self.lib.fire_nn_gradients(self.h, _p(x), _p(y_t), _p(y_map), B, _p(loss),
                                               _p(g), _s(stream)))
        return loss, g

    def train_step(self, x, y_t, y_map=None, lr=1e-3, stream=None):
        self.steps += 1
        loss = torch.empty(2, dtype=torch.float32, device=self.device)
        self._check(self.lib.fire_nn_train_step(self.h, _p(x), _p(y_t), _p(y_map), x.shape[0],
                                                float(lr), self.steps, _p(loss), _s(stream)))
        return loss
