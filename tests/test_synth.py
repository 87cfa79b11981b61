"""Input generators: determinism, layout and the slope/aspect conventions."""
import numpy as np

from paper_1701_03549_amd import synth


def test_deterministic_and_ranges():
    a = synth.make_landscape(96, 64, 101)
    b = synth.make_landscape(96, 64, 101)
    for k in ("veg", "elev_m", "slope_deg", "aspect_deg", "wind_to_deg"):
        assert np.array_equal(a[k], b[k])
        assert a[k].shape == (64, 96)
    assert a["veg"].dtype == np.uint8 and a["elev_m"].dtype == np.float32
    assert set(np.unique(a["veg"])) <= {0, 1, 2, 3}
    assert 0.08 <= np.mean(a["veg"] == 0) <= 0.12
    assert a["elev_m"].min() == 0.0 and abs(a["elev_m"].max() - 500.0) < 1e-3
    assert np.all(a["wind_to_deg"] == 45.0)
    s = synth.make_landscape(128, 128, 103, wind="smooth")
    assert np.all(s["wind_to_deg"] >= 0) and np.all(s["wind_to_deg"] < 360)
    assert s["wind_to_deg"].std() > 5


def test_slope_aspect_of_planes():
    x = np.arange(20, dtype=np.float64)[None, :].repeat(10, 0)
    y = np.arange(10, dtype=np.float64)[:, None].repeat(20, 1)
    # rising to the east by 30 m per cell: 45 degrees, faces west (270)
    s, a = synth.slope_aspect(x * 30.0)
    assert np.allclose(s, 45.0) and np.allclose(a, 270.0)
    # rising to the south (row grows): faces north (0)
    s, a = synth.slope_aspect(y * 15.0)
    assert np.allclose(s, np.degrees(np.arctan(0.5))) and np.allclose(a % 360, 0.0)
    # rising to the north-west: faces south-east (135)
    s, a = synth.slope_aspect(-(x + y) * 30.0)
    assert np.allclose(a, 135.0)
    s, a = synth.slope_aspect(np.zeros((4, 4)))
    assert np.all(s == 0) and np.all(a == 0)


def test_pack_roundtrip():
    rng = np.random.default_rng(0)
    for W in (1, 31, 32, 33, 100):
        m = rng.random((7, W)) < 0.5
        p = synth.pack_bits(m)
        assert p.shape == (7, (W + 31) // 32)
        assert np.array_equal(synth.unpack_bits(p, W), m)
        assert p[0, 0] & 1 == m[0, 0]
