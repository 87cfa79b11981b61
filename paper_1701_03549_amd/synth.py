"""Seeded synthetic landscapes (inputs only; none of the model's arithmetic).

The paper runs on 801x801 rasters of the northern Patagonian Andes at 30 m
(Methods, "Forest Fire Spread Simulation", and the landscape figure): a
vegetation map (0 non-burnable, 1 forest, 2 shrubland), slope, aspect and a
wind-direction field. Those rasters are not available, so this module builds
stand-ins of the same kind and layout from seeded value noise:

* vegetation (uint8): class-0 blobs where a low-frequency noise field (period
  W/8) is below its 10th percentile (about 10% of the cells); the other cells
  split into classes 1/2/3 by the terciles of an independent noise field;
* elevation (float32, metres): 4-octave value noise (base period W/4,
  persistence 0.5) rescaled to [0, 500];
* slope and aspect (float32, degrees): central differences of the elevation
  with 30 m cells (one-sided at the borders); slope = atan(|grad z|); aspect =
  compass direction (clockwise from north) that the downhill slope faces, 0
  on flat cells;
* wind (float32, compass degrees the wind blows toward): uniform 45 degrees,
  or a smooth field 45 + 60 * (2n - 1) with n a 1-octave value noise of
  period W/2.

Row 0 is north and x grows east. Every generator is a pure function of its
seed (numpy PCG64), so the oracle and the GPU library receive identical
arrays.
"""
from __future__ import annotations

import numpy as np

CELL_M = 30.0


def value_noise(W: int, H: int, period: float, rng: np.random.Generator) -> np.ndarray:
    """Smooth noise in [0, 1]: random lattice values every ``period`` cells,
    blended with a smoothstep-weighted bilinear interpolation."""
    period = max(float(period), 1.0)
    gw = int(np.ceil(W / period)) + 2
    gh = int(np.ceil(H / period)) + 2
    grid = rng.random((gh, gw))
    fx = np.arange(W, dtype=np.float64) / period
    fy = np.arange(H, dtype=np.float64) / period
    ix = np.floor(fx).astype(np.int64)
    iy = np.floor(fy).astype(np.int64)
    tx = fx - ix
    ty = fy - iy
    sx = tx * tx * (3.0 - 2.0 * tx)
    sy = ty * ty * (3.0 - 2.0 * ty)
    g00 = grid[iy[:, None], ix[None, :]]
    g01 = grid[iy[:, None], ix[None, :] + 1]
    g10 = grid[iy[:, None] + 1, ix[None, :]]
    g11 = grid[iy[:, None] + 1, ix[None, :] + 1]
    top = g00 * (1.0 - sx[None, :]) + g01 * sx[None, :]
    bot = g10 * (1.0 - sx[None, :]) + g11 * sx[None, :]
    return top * (1.0 - sy[:, None]) + bot * sy[:, None]


def fbm(W: int, H: int, base_period: float, octaves: int, persistence: float,
        rng: np.random.Generator) -> np.ndarray:
    acc = np.zeros((H, W), dtype=np.float64)
    amp = 1.0
    for o in range(octaves):
        acc += amp * value_noise(W, H, base_period / (2 ** o), rng)
        amp *= persistence
    return acc


def slope_aspect(elev: np.ndarray, cell_m: float = CELL_M):
    """Slope (degrees) and compass aspect (degrees) of an elevation raster."""
    z = np.asarray(elev, dtype=np.float64)
    H, W = z.shape
    dzdx = np.zeros_like(z)
    dzdy = np.zeros_like(z)  # derivative along increasing row (southward)
    if W > 1:
        dzdx[:, 1:-1] = (z[:, 2:] - z[:, :-2]) / (2.0 * cell_m)
        dzdx[:, 0] = (z[:, 1] - z[:, 0]) / cell_m
        dzdx[:, -1] = (z[:, -1] - z[:, -2]) / cell_m
    if H > 1:
        dzdy[1:-1, :] = (z[2:, :] - z[:-2, :]) / (2.0 * cell_m)
        dzdy[0, :] = (z[1, :] - z[0, :]) / cell_m
        dzdy[-1, :] = (z[-1, :] - z[-2, :]) / cell_m
    grad = np.hypot(dzdx, dzdy)
    slope = np.degrees(np.arctan(grad))
    # downhill direction: east component -dz/dx, north component +dz/dy(row)
    aspect = np.degrees(np.arctan2(-dzdx, dzdy)) % 360.0
    aspect = np.where(grad > 0.0, aspect, 0.0)
    return slope.astype(np.float32), aspect.astype(np.float32)


def make_landscape(W: int, H: int, seed: int, wind: str = "uniform",
                   wind_deg: float = 45.0) -> dict:
    """A seeded synthetic landscape of W x H cells at 30 m."""
    rng = np.random.default_rng(seed)
    # vegetation
    blobs = value_noise(W, H, max(W / 8.0, 2.0), rng)
    cut = np.quantile(blobs, 0.10)
    classes = value_noise(W, H, max(W / 8.0, 2.0), rng)
    t1, t2 = np.quantile(classes, [1.0 / 3.0, 2.0 / 3.0])
    veg = np.where(classes < t1, 1, np.where(classes < t2, 2, 3)).astype(np.uint8)
    veg[blobs < cut] = 0
    # elevation
    e = fbm(W, H, max(W / 4.0, 2.0), 4, 0.5, rng)
    e = (e - e.min()) / max(e.max() - e.min(), 1e-12) * 500.0
    elev = e.astype(np.float32)
    slope, aspect = slope_aspect(elev)
    # wind
    if wind == "uniform":
        wind_to = np.full((H, W), wind_deg, dtype=np.float32)
    elif wind == "smooth":
        n = value_noise(W, H, max(W / 2.0, 2.0), rng)
        wind_to = ((wind_deg + 60.0 * (2.0 * n - 1.0)) % 360.0).astype(np.float32)
    else:
        raise ValueError(f"unknown wind mode {wind!r}")
    return {"veg": veg, "elev_m": elev, "slope_deg": slope, "aspect_deg": aspect,
            "wind_to_deg": wind_to, "cell_m": CELL_M, "seed": seed}


def uniform_landscape(W: int, H: int, veg_class: int = 2, wind_deg: float = 45.0) -> dict:
    """A flat landscape of one vegetation class (test fixture)."""
    return {"veg": np.full((H, W), veg_class, dtype=np.uint8),
            "elev_m": np.zeros((H, W), dtype=np.float32),
            "slope_deg": np.zeros((H, W), dtype=np.float32),
            "aspect_deg": np.zeros((H, W), dtype=np.float32),
            "wind_to_deg": np.full((H, W), wind_deg, dtype=np.float32),
            "cell_m": CELL_M, "seed": None}


def random_small_landscape(W: int, H: int, seed: int, p_blocked: float = 0.15) -> dict:
    """Unstructured random landscape for property tests on tiny lattices."""
    rng = np.random.default_rng(seed)
    veg = rng.integers(1, 4, size=(H, W)).astype(np.uint8)
    veg[rng.random((H, W)) < p_blocked] = 0
    elev = (rng.random((H, W)) * 100.0).astype(np.float32)
    slope = (rng.random((H, W)) * 30.0).astype(np.float32)
    aspect = (rng.random((H, W)) * 360.0).astype(np.float32)
    wind = (rng.random((H, W)) * 360.0).astype(np.float32)
    return {"veg": veg, "elev_m": elev, "slope_deg": slope, "aspect_deg": aspect,
            "wind_to_deg": wind, "cell_m": CELL_M, "seed": seed}


def pack_bits(mask: np.ndarray) -> np.ndarray:
    """Boolean [H][W] -> uint32 [H][ceil(W/32)], cell x is bit x%32 of word x//32."""
    m = np.asarray(mask, dtype=bool)
    H, W = m.shape
    wpr = (W + 31) // 32
    pad = np.zeros((H, wpr * 32), dtype=bool)
    pad[:, :W] = m
    b = pad.reshape(H, wpr, 32).astype(np.uint64)
    weights = (np.uint64(1) << np.arange(32, dtype=np.uint64))
    return (b * weights).sum(axis=2).astype(np.uint32)


def unpack_bits(bits: np.ndarray, W: int) -> np.ndarray:
    """uint32 [H][ceil(W/32)] -> boolean [H][W]."""
    b = np.asarray(bits, dtype=np.uint32)
    H, wpr = b.shape
    shifts = np.arange(32, dtype=np.uint32)
    full = ((b[:, :, None] >> shifts[None, None, :]) & 1).astype(bool).reshape(H, wpr * 32)
    return full[:, :W]


def nearest_burnable(veg: np.ndarray, x: int, y: int):
    """The burnable cell closest (Euclidean, ties by row then column) to (x, y);
    the workloads' "ignition at the centre" uses this so that a non-burnable
    blob at the exact centre does not leave every replicate empty."""
    v = np.asarray(veg)
    ys, xs = np.nonzero(v != 0)
    d2 = (xs - x) ** 2 + (ys - y) ** 2
    k = np.lexsort((xs, ys, d2))[0]
    return int(xs[k]), int(ys[k])


def nearest_of_class(veg: np.ndarray, cls: int, x: int, y: int):
    """The cell of vegetation class ``cls`` closest to (x, y) (Euclidean, ties
    by row then column)."""
    v = np.asarray(veg)
    ys, xs = np.nonzero(v == cls)
    d2 = (xs - x) ** 2 + (ys - y) ** 2
    k = np.lexsort((xs, ys, d2))[0]
    return int(xs[k]), int(ys[k])


def ignition_site(ls: dict, x=None, y=None):
    """Reference ignition of the workloads: the burnable cell nearest (x, y)
    (default: the centre) on a slope steeper than 5 degrees facing within 45
    degrees of north-west, the driest exposure in the paper's study area; the
    reference fires of the benchmarks start there so that they stay on their
    hillside, as the paper's reference fire stays away from the lattice edge."""
    veg = np.asarray(ls["veg"])
    H, W = veg.shape
    x = W // 2 if x is None else x
    y = H // 2 if y is None else y
    dev = (np.asarray(ls["aspect_deg"], dtype=np.float64) - 315.0 + 180.0) % 360.0 - 180.0
    ok = (veg != 0) & (np.asarray(ls["slope_deg"]) > 5.0) & (np.abs(dev) <= 45.0)
    if not ok.any():
        return nearest_burnable(veg, x, y)
    ys, xs = np.nonzero(ok)
    d2 = (xs - x) ** 2 + (ys - y) ** 2
    k = np.lexsort((xs, ys, d2))[0]
    return int(xs[k]), int(ys[k])


# ---------------------------------------------------------------------------
# The ignition-scan workload: 1024 x 1024, landscape seed 103, smooth wind.
# Slopes on this landscape are gentle (6% of cells steeper than 5 degrees),
# so the calibration vector, whose fires are driven by the aspect term,
# burns about a hundred cells there. The scan instead uses a vector whose
# fires are driven by forest and wind: forest burns (logit -1 + 1.0 omega +
# slope term), other classes barely do (logit -2.5 + ...), so a fire from the
# forest cell nearest the centre fills part of its forest stand (median 2.6%
# of the lattice in an oracle pilot of 100 replicates, none reaching the
# border) and stops where the stand ends.
SCAN_SIZE = (1024, 1024)
SCAN_SEED = 103
SCAN_BETA = (-2.5, 1.5, 0.0, 1.0, 1.0)


def scan_landscape() -> dict:
    W, H = SCAN_SIZE
    return make_landscape(W, H, SCAN_SEED, wind="smooth")


def scan_ignition(ls: dict):
    """The true ignition of the scan workload: the forest cell (class 1)
    nearest the centre."""
    H, W = np.asarray(ls["veg"]).shape
    return nearest_of_class(ls["veg"], 1, W // 2, H // 2)
