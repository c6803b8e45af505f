"""The gradient angle of the orientation and descriptor kernels is an
octant-reduced odd polynomial (no library arctangent).  Its coefficients are
read from the kernel source and evaluated here in float32 exactly as the
kernel does (Horner with fused multiply-adds emulated in float64 then
rounded), against numpy's arctan2 over all quadrants."""
import importlib.util
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1705_09776_amd", "csrc", "describe.hip")


def _coeffs():
    body = open(SRC).read()
    body = body[body.index("float angle_2pi("):]
    body = body[:body.index("return r")]
    first = re.search(r"float p = (-?[0-9.e-]+)f;", body).group(1)
    rest = re.findall(r"p = fmaf\(p, s, (-?[0-9.e-]+)f\);", body)
    return [np.float32(first)] + [np.float32(c) for c in rest]


def _angle(y, x):
    f = np.float32
    ax, ay = np.abs(x), np.abs(y)
    mx = np.maximum(np.maximum(ax, ay), f(1.17549435e-38))
    mn = np.minimum(ax, ay)
    t = (mn / mx).astype(np.float32)
    s = (t * t).astype(np.float32)
    c = _coeffs()
    p = np.full_like(t, c[0])
    for cc in c[1:]:
        p = (p.astype(np.float64) * s + cc).astype(np.float32)
    r = (p * t).astype(np.float32)
    r = np.where(ay > ax, f(1.5707963267948966) - r, r).astype(np.float32)
    r = np.where(x < 0, f(3.141592653589793) - r, r).astype(np.float32)
    return np.where(y < 0, f(2 * np.pi) - r, r).astype(np.float32)


def test_polynomial_on_unit_interval():
    c = _coeffs()
    assert len(c) == 6
    t = np.linspace(0, 1, 100001)
    p = np.polyval(np.array(c, dtype=np.float64), t * t) * t   # c runs from the highest power down
    assert np.abs(p - np.arctan(t)).max() < 2e-6


def test_angle_all_quadrants():
    rng = np.random.default_rng(0)
    x = rng.normal(size=200000).astype(np.float32) * 50
    y = rng.normal(size=200000).astype(np.float32) * 50
    x[:4] = [1, 0, -1, 0]
    y[:4] = [0, 1, 0, -1]
    got = _angle(y, x).astype(np.float64)
    ref = np.mod(np.arctan2(y.astype(np.float64), x.astype(np.float64)), 2 * np.pi)
    d = np.abs(got - ref)
    d = np.minimum(d, 2 * np.pi - d)
    # the polynomial's 1.7e-6, plus one fp32 ulp at 2 pi (4.8e-7) from the
    # reflections
    assert d.max() < 2.5e-6
    # 2 pi itself only by rounding (the histograms take it as bin 0)
    assert np.all((got >= 0) & (got <= np.float32(2 * np.pi)))
    assert _angle(np.float32([0]), np.float32([0]))[0] == 0


def test_coefficients_reproduced_by_the_fit_script():
    """The kernel's coefficients are what the committed fitting script
    (Lawson minimax fit, float64, rounded to float32) writes -- within one
    float32 ulp, so a last-bit change of a library's least-squares solver
    does not matter."""
    path = os.path.join(ROOT, "paper_1705_09776_amd", "csrc", "fit_atan_poly.py")
    spec = importlib.util.spec_from_file_location("fit_atan_poly", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    fitted = mod.fit()
    src = np.array(_coeffs(), dtype=np.float32)
    assert fitted.shape == src.shape
    assert np.all(np.abs(fitted - src) <= np.spacing(np.abs(src)))
    assert mod.max_error(src) < 2e-6
