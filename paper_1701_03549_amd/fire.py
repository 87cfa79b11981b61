"""Python binding of the C ABI in include/fire.h (argument marshalling only).

Every computation runs in the HIP library ``libfiregpu.so`` built in this
package directory; PyTorch provides device memory and streams. There is no
fallback: if the library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # imported before the library so one HIP runtime serves both

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfiregpu.so")

SIM_DTYPE = np.dtype([("landscape_id", "<i4"), ("target_id", "<i4"), ("ign_x", "<i4"),
                      ("ign_y", "<i4"), ("param_index", "<u4"), ("sim_index", "<u4"),
                      ("max_steps", "<u4")])
RESULT_DTYPE = np.dtype([("burnt", "<u4"), ("steps", "<u4"), ("trials", "<u8"),
                         ("fitness", "<f8")])
assert SIM_DTYPE.itemsize == 28 and RESULT_DTYPE.itemsize == 24
RUN_TO_EXTINCTION = 0xFFFFFFFF

STATUS = {0: "FIRE_OK", -1: "FIRE_E_INVALID", -2: "FIRE_E_OOM", -3: "FIRE_E_DEVICE",
          -4: "FIRE_E_UNSUPPORTED"}

EXPORTS = ["fire_ctx_create", "fire_ctx_destroy", "fire_last_error", "fire_sync", "fire_version",
           "fire_landscape_load", "fire_landscape_free", "fire_landscape_set_burn_steps",
           "fire_target_load", "fire_target_free",
           "fire_thresholds", "fire_thresholds_dev", "fire_run", "fire_order_sims", "fire_run_dev", "fire_run_dev_noalloc", "fire_run_dense",
           "fire_set_sim_timing",
           "fire_set_schedule",
           "fire_get_schedule", "fire_set_class_schedule", "fire_ga_step", "fire_ga_offspring", "fire_ga_step_genes",
           "fire_ga_sims_from_pop", "fire_ga_run", "fire_ga_run_ignition", "fire_ensemble", "fire_scan_reduce"]


class FireError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class LandscapeDesc(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("cell_m", ctypes.c_float),
                ("veg", ctypes.c_void_p), ("elev_m", ctypes.c_void_p),
                ("slope_deg", ctypes.c_void_p), ("aspect_deg", ctypes.c_void_p),
                ("wind_to_deg", ctypes.c_void_p), ("forest_class", ctypes.c_uint8),
                ("on_device", ctypes.c_int32)]


class Schedule(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("queue_cap", ctypes.c_int32),
                ("table_mode", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("window", ctypes.c_int32), ("wave", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class GACfg(ctypes.Structure):
    _fields_ = [("elite", ctypes.c_int32), ("pm0", ctypes.c_double), ("mut_h", ctypes.c_double),
                ("lo", ctypes.c_double), ("hi", ctypes.c_double), ("generations", ctypes.c_uint32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfiregpu.so (no GPU calls); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with `python -m paper_1701_03549_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, u32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32,
                                   ctypes.c_int64, ctypes.c_uint64, ctypes.c_double)
    sig = {
        "fire_ctx_create": (i32, [ctypes.c_int, ctypes.POINTER(vp)]),
        "fire_ctx_destroy": (None, [vp]),
        "fire_last_error": (ctypes.c_char_p, [vp]),
        "fire_sync": (i32, [vp, vp]),
        "fire_version": (ctypes.c_char_p, []),
        "fire_landscape_load": (i32, [vp, ctypes.POINTER(LandscapeDesc), ctypes.POINTER(i32)]),
        "fire_landscape_free": (i32, [vp, i32]),
        "fire_target_load": (i32, [vp, i32, vp, ctypes.POINTER(i32)]),
        "fire_target_free": (i32, [vp, i32]),
        "fire_landscape_set_burn_steps": (i32, [vp, i32, vp]),
        "fire_thresholds": (i32, [vp, i32, vp, vp, vp]),
        "fire_thresholds_dev": (i32, [vp, i32, vp, i32, vp, vp]),
        "fire_run": (i32, [vp, vp, i32, vp, i32, u64, vp, vp, vp, i64, vp]),
        "fire_order_sims": (i32, [vp, vp, i32, vp, i32, vp]),
        "fire_run_dev": (i32, [vp, vp, i32, vp, i32, u64, vp, vp, vp, i64, vp]),
        "fire_run_dev_noalloc": (i32, [vp, vp, i32, vp, i32, u64, vp, vp, vp, i64, vp]),
        "fire_run_dense": (i32, [vp, vp, i32, vp, i32, u64, vp, vp, i64, vp]),
        "fire_set_sim_timing": (i32, [vp, vp, i64]),
        "fire_set_schedule": (i32, [vp, ctypes.POINTER(Schedule)]),
        "fire_get_schedule": (i32, [vp, i64, i32, i32, ctypes.POINTER(Schedule)]),
        "fire_set_class_schedule": (i32, [vp, i64, i32, ctypes.POINTER(Schedule)]),
        "fire_ga_step": (i32, [vp, vp, vp, vp, i32, i32, i32, ctypes.POINTER(GACfg), u32, u64, vp]),
        "fire_ga_offspring": (i32, [vp, vp, vp, i32, i32, i32, ctypes.POINTER(GACfg), u32, u64, u64,
                                    i32, vp, vp]),
        "fire_ga_step_genes": (i32, [vp, vp, vp, vp, i32, i32, i32, i32, dbl, vp, vp, vp, u32, u32,
                                     u64, vp]),
        "fire_ga_sims_from_pop": (i32, [vp, vp, i32, i32, i32, i32, i32, u32, vp, vp, vp]),
        "fire_ga_run": (i32, [vp, i32, i32, i32, i32, vp, i32, i32, ctypes.POINTER(GACfg), u64,
                              u64, vp, vp, vp]),
        "fire_ga_run_ignition": (i32, [vp, i32, i32, vp, i32, i32, i32, dbl, u32, vp, vp, vp, u64,
                                       u64, vp, vp, vp]),
        "fire_ensemble": (i32, [vp, vp, vp, i32, i32, i32, dbl, vp, vp, vp, vp, vp]),
        "fire_scan_reduce": (i32, [vp, vp, i32, i32, dbl, dbl, vp, vp, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream(stream) -> int:
    if stream is None:
        return int(torch.cuda.current_stream().cuda_stream)
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def results_to_numpy(res: torch.Tensor) -> np.ndarray:
    """Device result buffer (uint8 [n, 24]) -> numpy structured array."""
    return res.cpu().numpy().reshape(-1).view(RESULT_DTYPE)


def make_sims(n, landscape_id=0, target_id=-1, ign=(0, 0), param_index=0, sim_index=None,
              max_steps=RUN_TO_EXTINCTION) -> np.ndarray:
    s = np.zeros(n, dtype=SIM_DTYPE)
    s["landscape_id"] = landscape_id
    s["target_id"] = target_id
    s["ign_x"] = np.asarray(ign)[..., 0] if np.ndim(ign) > 1 else ign[0]
    s["ign_y"] = np.asarray(ign)[..., 1] if np.ndim(ign) > 1 else ign[1]
    s["param_index"] = param_index
    s["sim_index"] = np.arange(n, dtype=np.uint32) if sim_index is None else sim_index
    s["max_steps"] = max_steps
    return s


class FireGPU:
    """A library context on one GPU (wraps fire_ctx)."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the fire library has no CPU path")
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        h = ctypes.c_void_p()
        st = self.lib.fire_ctx_create(device, ctypes.byref(h))
        if st != 0:
            raise FireError(st, "fire_ctx_create failed")
        self.ctx = h
        self.dims = {}

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.fire_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise FireError(st, self.lib.fire_last_error(self.ctx).decode())

    def sync(self, stream=None):
        self._check(self.lib.fire_sync(self.ctx, _stream(stream)))

    # -- landscapes and targets ---------------------------------------------
    def load_landscape(self, ls: dict, forest_class: int = 1) -> int:
        veg = np.ascontiguousarray(ls["veg"], dtype=np.uint8)
        H, W = veg.shape
        f = [np.ascontiguousarray(ls[k], dtype=np.float32)
             for k in ("elev_m", "slope_deg", "aspect_deg", "wind_to_deg")]
        d = LandscapeDesc(W, H, float(ls.get("cell_m", 30.0)), veg.ctypes.data, f[0].ctypes.data,
                          f[1].ctypes.data, f[2].ctypes.data, f[3].ctypes.data, forest_class, 0)
        out = ctypes.c_int32()
        self._check(self.lib.fire_landscape_load(self.ctx, ctypes.byref(d), ctypes.byref(out)))
        self.dims[out.value] = (W, H)
        return out.value

    def set_burn_steps(self, lid: int, steps=None):
        """Turn-off time per vegetation value (uint8 [256]), or None for the
        one-step model."""
        if steps is None:
            self._check(self.lib.fire_landscape_set_burn_steps(self.ctx, lid, None))
            return
        a = np.ascontiguousarray(steps, dtype=np.uint8)
        if a.shape != (256,):
            raise ValueError("steps must have 256 entries")
        self._check(self.lib.fire_landscape_set_burn_steps(self.ctx, lid, a.ctypes.data))

    def free_landscape(self, lid: int):
        self._check(self.lib.fire_landscape_free(self.ctx, lid))
        self.dims.pop(lid, None)

    def load_target(self, lid: int, bits: np.ndarray) -> int:
        b = np.ascontiguousarray(bits, dtype=np.uint32)
        W, H = self.dims[lid]
        assert b.shape == (H, (W + 31) // 32)
        out = ctypes.c_int32()
        self._check(self.lib.fire_target_load(self.ctx, lid, b.ctypes.data, ctypes.byref(out)))
        return out.value

    def free_target(self, tid: int):
        self._check(self.lib.fire_target_free(self.ctx, tid))

    # -- Eq. 1 ---------------------------------------------------------------
    def thresholds(self, lid: int, beta, out: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
        """Eq. 1 table [H][W][8] (int32 storage of the uint32 thresholds)."""
        W, H = self.dims[lid]
        b = (ctypes.c_double * 5)(*[float(v) for v in beta])
        if out is None:
            out = torch.empty((H, W, 8), dtype=torch.int32, device=self.device)
        assert out.numel() == H * W * 8 and out.is_contiguous()
        self._check(self.lib.fire_thresholds(self.ctx, lid, b, _ptr(out), _stream(stream)))
        return out

    def thresholds_dev(self, lid: int, betas_dev: torch.Tensor, out: torch.Tensor | None = None,
                       stream=None) -> torch.Tensor:
        """fire_thresholds_dev: Eq. 1 tables [n_params][H][W][8] for the
        float64 parameter rows of `betas_dev` (on the device); no host
        synchronisation, capturable."""
        W, H = self.dims[lid]
        if betas_dev.dtype != torch.float64 or not betas_dev.is_contiguous() \
                or betas_dev.numel() % 5 != 0 or betas_dev.numel() == 0:
            raise ValueError("betas_dev must be a contiguous float64 tensor of n x 5 values")
        n = betas_dev.numel() // 5
        if out is None:
            out = torch.empty((n, H, W, 8), dtype=torch.int32, device=self.device)
        assert out.numel() == n * H * W * 8 and out.is_contiguous()
        self._check(self.lib.fire_thresholds_dev(self.ctx, lid, _ptr(betas_dev), n, _ptr(out),
                                                 _stream(stream)))
        return out

    # -- simulations ---------------------------------------------------------
    def map_words(self, sims: np.ndarray) -> int:
        ids = np.unique(sims["landscape_id"])
        return max(self.dims[int(i)][1] * ((self.dims[int(i)][0] + 31) // 32) for i in ids)

    def run(self, betas, sims: np.ndarray, seed: int, override: torch.Tensor | None = None,
            want_maps: bool = False, stream=None):
        """fire_run with host parameters/descriptors; returns (results uint8[n,24], maps)."""
        b = np.ascontiguousarray(np.asarray(betas, dtype=np.float64).reshape(-1, 5))
        s = np.ascontiguousarray(sims, dtype=SIM_DTYPE)
        n = len(s)
        res = torch.empty((max(n, 1), 24), dtype=torch.uint8, device=self.device)
        maps, mw = None, 0
        if want_maps and n:
            mw = self.map_words(s)
            maps = torch.empty((n, mw), dtype=torch.int32, device=self.device)
        self._check(self.lib.fire_run(self.ctx, b.ctypes.data, len(b), s.ctypes.data, n,
                                      int(seed) & (2 ** 64 - 1), _ptr(override), _ptr(res),
                                      _ptr(maps), mw, _stream(stream)))
        return res[:n], maps

    def order_sims(self, betas, sims: np.ndarray) -> np.ndarray:
        """fire_order_sims: the longest-expected-first permutation of host descriptors."""
        b = np.ascontiguousarray(np.asarray(betas, dtype=np.float64).reshape(-1, 5))
        s = np.ascontiguousarray(sims, dtype=SIM_DTYPE)
        order = np.empty(max(len(s), 1), dtype=np.int32)
        self._check(self.lib.fire_order_sims(self.ctx, b.ctypes.data, len(b), s.ctypes.data,
                                             len(s), order.ctypes.data))
        return order[:len(s)]

    def run_dense(self, betas, sims: np.ndarray, seed: int, want_maps: bool = False,
                  stream=None):
        """fire_run_dense (per-cell ablation path); returns (results, maps)."""
        b = np.ascontiguousarray(np.asarray(betas, dtype=np.float64).reshape(-1, 5))
        s = np.ascontiguousarray(sims, dtype=SIM_DTYPE)
        n = len(s)
        res = torch.empty((max(n, 1), 24), dtype=torch.uint8, device=self.device)
        maps, mw = None, 0
        if want_maps and n:
            mw = self.map_words(s)
            maps = torch.empty((n, mw), dtype=torch.int32, device=self.device)
        self._check(self.lib.fire_run_dense(self.ctx, b.ctypes.data, len(b), s.ctypes.data, n,
                                            int(seed) & (2 ** 64 - 1), _ptr(res), _ptr(maps), mw,
                                            _stream(stream)))
        return res[:n], maps

    def run_dev(self, betas_dev: torch.Tensor, sims_dev: torch.Tensor, n_sims: int, seed: int,
                out: torch.Tensor, maps: torch.Tensor | None = None, map_words: int = 0,
                override: torch.Tensor | None = None, stream=None):
        """fire_run_dev: every buffer already on the device (no host staging)."""
        n_params = betas_dev.numel() // 5
        self._check(self.lib.fire_run_dev(self.ctx, _ptr(betas_dev), n_params, _ptr(sims_dev),
                                          n_sims, int(seed) & (2 ** 64 - 1), _ptr(override),
                                          _ptr(out), _ptr(maps), map_words, _stream(stream)))

    def run_dev_noalloc(self, betas_dev: torch.Tensor, sims_dev: torch.Tensor, n_sims: int,
                        seed: int, out: torch.Tensor, maps: torch.Tensor | None = None,
                        map_words: int = 0, override: torch.Tensor | None = None, stream=None):
        """fire_run_dev_noalloc: as run_dev, with the library's per-GPU scratch
        array instead of allocated buffers (calls on one GPU must not overlap)."""
        n_params = betas_dev.numel() // 5
        self._check(self.lib.fire_run_dev_noalloc(
            self.ctx, _ptr(betas_dev), n_params, _ptr(sims_dev), n_sims,
            int(seed) & (2 ** 64 - 1), _ptr(override), _ptr(out), _ptr(maps), map_words,
            _stream(stream)))

    def set_sim_timing(self, times: torch.Tensor | None):
        """fire_set_sim_timing: per-simulation (take, finish) device clocks
        into `times` (int64, shape (capacity, 2), on this device) until
        called with None."""
        if times is None:
            self._check(self.lib.fire_set_sim_timing(self.ctx, None, 0))
            return
        if times.dtype != torch.int64 or times.dim() != 2 or times.shape[1] != 2 \
                or not times.is_contiguous():
            raise ValueError("times must be a contiguous int64 tensor of shape (n, 2)")
        self._check(self.lib.fire_set_sim_timing(self.ctx, _ptr(times), times.shape[0]))

    # -- schedule ------------------------------------------------------------
    def set_schedule(self, threads=None, queue_cap=None, table_mode=None, wg_per_cu=None,
                     window=0, wave=0, reset=False):
        """Fix the schedule (window: 0 = whole-lattice bitsets, -1 = built-in
        choice, else the LDS window side in cells; wave: 1 = one simulation
        per wavefront, 0 = one per workgroup of `threads`)."""
        if reset:
            self._check(self.lib.fire_set_schedule(self.ctx, None))
            return
        s = Schedule(int(threads), int(queue_cap), int(table_mode), int(wg_per_cu), int(window),
                     int(wave))
        self._check(self.lib.fire_set_schedule(self.ctx, ctypes.byref(s)))

    BATCH_KINDS = {"replicate": 0, "population": 1, "scattered": 2}

    def set_class_schedule(self, max_cells: int, sched: dict | None, kind=None):
        """Schedule for runs on landscapes of the size class of ``max_cells``
        and batches of `kind`: "replicate" (at most 8 parameter vectors),
        "population" (more, with at least 8 simulations each), "scattered"
        (the rest), or every kind (None)."""
        kinds = (0, 1, 2) if kind is None else (self.BATCH_KINDS[kind],)
        for k in kinds:
            if sched is None:
                self._check(self.lib.fire_set_class_schedule(self.ctx, int(max_cells), k, None))
                continue
            s = Schedule(int(sched["threads"]), int(sched["queue_cap"]),
                         int(sched["table_mode"]), int(sched["wg_per_cu"]),
                         int(sched.get("window", -1)), int(sched.get("wave", -1)))
            self._check(self.lib.fire_set_class_schedule(self.ctx, int(max_cells), k,
                                                         ctypes.byref(s)))

    def get_schedule(self, max_cells: int, n_params: int = 1, n_sims: int = 1 << 20) -> dict:
        """The schedule a batch of n_sims simulations would use."""
        s = Schedule()
        self._check(self.lib.fire_get_schedule(self.ctx, int(max_cells), int(n_params),
                                               int(n_sims), ctypes.byref(s)))
        return s.as_dict()

    # -- GA, ensemble, scan --------------------------------------------------
    @staticmethod
    def ga_cfg(elite=2, pm0=0.2, mut_h=1.0, lo=-30.0, hi=30.0, generations=50) -> GACfg:
        return GACfg(elite, pm0, mut_h, lo, hi, generations)

    def ga_step(self, pop: torch.Tensor, fit: torch.Tensor, cfg: GACfg, gen: int, ga_seed: int,
                mean_fit: torch.Tensor | None = None, stream=None):
        P, G = pop.shape
        R = fit.shape[1]
        self._check(self.lib.fire_ga_step(self.ctx, _ptr(pop), _ptr(fit), _ptr(mean_fit), P, G, R,
                                          ctypes.byref(cfg), int(gen), int(ga_seed) & (2 ** 64 - 1),
                                          _stream(stream)))

    def ga_offspring(self, pop: torch.Tensor, fit: torch.Tensor, cfg: GACfg, gen: int,
                     ga_seed: int, seed_step: int, out_sets: torch.Tensor, stream=None):
        """fire_ga_offspring: out_sets[o] = the offspring fire_ga_step would
        make from (pop, fit) under seed ga_seed + o * seed_step (mod 2^64)."""
        P, G = pop.shape
        R = fit.shape[1]
        S = out_sets.shape[0]
        assert out_sets.shape == (S, P, G) and out_sets.dtype == torch.float64 \
            and out_sets.is_contiguous()
        self._check(self.lib.fire_ga_offspring(self.ctx, _ptr(pop), _ptr(fit), P, G, R,
                                               ctypes.byref(cfg), int(gen),
                                               int(ga_seed) & (2 ** 64 - 1),
                                               int(seed_step) & (2 ** 64 - 1), S, _ptr(out_sets),
                                               _stream(stream)))

    def ga_step_genes(self, pop: torch.Tensor, fit: torch.Tensor, *, elite: int, pm0: float,
                      lo, hi, h, generations: int, gen: int, ga_seed: int,
                      mean_fit: torch.Tensor | None = None, stream=None):
        """GA generation with a box and mutation width per gene."""
        P, G = pop.shape
        R = fit.shape[1]
        arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (G,)))
                for a in (lo, hi, h)]
        self._check(self.lib.fire_ga_step_genes(
            self.ctx, _ptr(pop), _ptr(fit), _ptr(mean_fit), P, G, R, int(elite), float(pm0),
            arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data, int(generations),
            int(gen), int(ga_seed) & (2 ** 64 - 1), _stream(stream)))

    def ga_sims_from_pop(self, pop: torch.Tensor, R: int, lid: int, tid: int, gen: int,
                         sims: torch.Tensor | None = None, betas: torch.Tensor | None = None,
                         stream=None):
        """Device descriptors (uint8 [P*R, 28]) and betas [P, 5] of a generation
        whose genes 5 and 6 are the ignition cell."""
        P, G = pop.shape
        if sims is None:
            sims = torch.empty((P * R, SIM_DTYPE.itemsize), dtype=torch.uint8, device=self.device)
        if betas is None:
            betas = torch.empty((P, 5), dtype=torch.float64, device=self.device)
        self._check(self.lib.fire_ga_sims_from_pop(self.ctx, _ptr(pop), P, G, R, lid, tid,
                                                   int(gen), _ptr(sims), _ptr(betas),
                                                   _stream(stream)))
        return sims, betas

    def ga_run(self, lid: int, tid: int, ign, pop0: np.ndarray, R: int, cfg: GACfg,
               sim_seed: int, ga_seed: int, stream=None):
        p0 = np.ascontiguousarray(pop0, dtype=np.float64)
        P = p0.shape[0]
        gens = int(cfg.generations)
        hist_pop = torch.empty((gens, P, 5), dtype=torch.float64, device=self.device)
        hist_fit = torch.empty((gens, P, R), dtype=torch.float64, device=self.device)
        self._check(self.lib.fire_ga_run(self.ctx, lid, tid, int(ign[0]), int(ign[1]),
                                         p0.ctypes.data, P, R, ctypes.byref(cfg),
                                         int(sim_seed) & (2 ** 64 - 1),
                                         int(ga_seed) & (2 ** 64 - 1), _ptr(hist_pop),
                                         _ptr(hist_fit), _stream(stream)))
        return hist_pop, hist_fit

    def ga_run_ignition(self, lid: int, tid: int, pop0: np.ndarray, R: int, *, elite: int,
                        pm0: float, generations: int, lo, hi, h, sim_seed: int, ga_seed: int,
                        stream=None):
        """GA over (beta[5], x, y) (fire_ga_run_ignition). Returns device
        histories (pop [gens][P][7], fitness [gens][P][R])."""
        p0 = np.ascontiguousarray(pop0, dtype=np.float64)
        P = p0.shape[0]
        assert p0.shape[1] == 7
        arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (7,)))
                for a in (lo, hi, h)]
        hist_pop = torch.empty((generations, P, 7), dtype=torch.float64, device=self.device)
        hist_fit = torch.empty((generations, P, R), dtype=torch.float64, device=self.device)
        self._check(self.lib.fire_ga_run_ignition(
            self.ctx, lid, tid, p0.ctypes.data, P, R, int(elite), float(pm0), int(generations),
            arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data,
            int(sim_seed) & (2 ** 64 - 1), int(ga_seed) & (2 ** 64 - 1), _ptr(hist_pop),
            _ptr(hist_fit), _stream(stream)))
        return hist_pop, hist_fit

    def ensemble(self, params: torch.Tensor, deltas: torch.Tensor, cutoff: float, stream=None):
        N, G = params.shape
        R = deltas.numel() // N
        best = torch.empty(1, dtype=torch.int32, device=self.device)
        n = torch.empty(1, dtype=torch.int32, device=self.device)
        mean = torch.empty(G, dtype=torch.float64, device=self.device)
        sd = torch.empty(G, dtype=torch.float64, device=self.device)
        self._check(self.lib.fire_ensemble(self.ctx, _ptr(params), _ptr(deltas), N, G, R,
                                           float(cutoff), _ptr(best), _ptr(n), _ptr(mean),
                                           _ptr(sd), _stream(stream)))
        return {"best_individual": best, "n_accepted": n, "mean": mean, "sd": sd}

    def scan_reduce(self, deltas: torch.Tensor, cutoff: float, tau: float = 0.1, stream=None):
        C, R = deltas.shape
        outs = [torch.empty(C, dtype=torch.float64, device=self.device) for _ in range(4)]
        self._check(self.lib.fire_scan_reduce(self.ctx, _ptr(deltas), C, R, float(cutoff),
                                              float(tau), *[_ptr(o) for o in outs],
                                              _stream(stream)))
        return dict(zip(("mean", "sd", "accept", "posterior"), outs))
