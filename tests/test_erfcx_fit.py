"""The erfcx series the pair kernels use for erfc (csrc/erfcx_fit.h),
evaluated here on the host in the kernels' own steps and precision, against
scipy's erfcx and erfc (no GPU)."""
import os
import re

import numpy as np
from scipy.special import erfc, erfcx

HEADER = os.path.join(os.path.dirname(os.path.abspath(__file__)), os.pardir,
                      "paper_2201_00804_amd", "csrc", "erfcx_fit.h")


def _fit(name):
    text = open(HEADER).read()
    deg = int(re.search(rf"kErfcxDeg{name} = (\d+);", text).group(1))
    p = float(re.search(rf"kErfcxP{name} = ([-+0-9.eE]+)f?;", text).group(1))
    t0 = float(re.search(rf"kErfcxT0{name} = ([-+0-9.eE]+)f?;", text).group(1))
    body = re.search(rf"kErfcxC{name}\[\d+\] = \{{(.*?)\}};", text, re.S).group(1)
    c = [float(v.rstrip("f")) for v in body.replace(",", " ").split()]
    xmax = float(re.search(r"kErfcxMax = ([0-9.]+);", text).group(1))
    assert len(c) == deg + 1
    return p, t0, np.array(c), xmax


def _series(x, p, t0, c, dt):
    """The kernels' evaluation: t = 1/(1 + p x), u, Clenshaw, all in dt."""
    x = np.minimum(x.astype(dt), dt(6.0))
    t = (dt(1) / (dt(1) + dt(p) * x)).astype(dt)
    u = ((t - dt(t0)) * dt(2.0 / (1.0 - t0)) - dt(1)).astype(dt)
    cc = c.astype(dt)
    b1 = np.zeros_like(u)
    b2 = np.zeros_like(u)
    for k in range(len(c) - 1, 0, -1):
        b1, b2 = (dt(2) * u * b1 + (cc[k] - b2)).astype(dt), b1
    return (u * b1 + (cc[0] - b2)).astype(dt)


def test_fp64_series():
    p, t0, c, xmax = _fit("F64")
    assert xmax == 6.0
    x = np.linspace(0.0, xmax, 200001)
    rel = np.abs(_series(x, p, t0, c, np.float64) / erfcx(x) - 1.0)
    assert rel.max() < 3e-14, rel.max()
    # erfc itself through the exp factor, over the Ewald range
    xs = np.linspace(0.05, 5.0, 20001)
    e = np.exp(-xs * xs) * _series(xs, p, t0, c, np.float64)
    assert np.abs(e / erfc(xs) - 1.0).max() < 5e-14


def test_fp32_series():
    p, t0, c, xmax = _fit("F32")
    x = np.linspace(0.0, xmax, 200001).astype(np.float32)
    ref = erfcx(x.astype(np.float64))
    rel = np.abs(_series(x, p, t0, c, np.float32).astype(np.float64) / ref - 1.0)
    assert rel.max() < 1.5e-6, rel.max()


def test_clamp_beyond_range():
    """Past x = 6 the series is taken at 6: erfc is below 2e-17 there, and the
    clamped value stays within a factor x/6 of it."""
    p, t0, c, _ = _fit("F64")
    x = np.array([6.0, 7.0, 9.0, 12.0])
    e = np.exp(-x * x) * _series(x, p, t0, c, np.float64)
    assert np.all(e <= 2.2e-17)
    assert np.all(e >= erfc(x) * 0.99) and np.all(e <= erfc(x) * x / 6.0 * 1.01)
