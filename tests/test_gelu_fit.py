"""The closed-form gelu of the inference kernel (gelu_fit in vx_mlp.hip) against the definition
x Phi(x) = x (1 + erf(x / sqrt 2)) / 2: the error bound its comments, the header and the design notes
state (below 3e-5 everywhere). The constants are read from the kernel source, so the check follows
the code; the formula is evaluated in float32 as the kernel does (exp2 and reciprocal exact here,
the hardware's are within an ulp or two)."""
import os
import re

import numpy as np
from scipy.special import erf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def fit_constants():
    src = open(os.path.join(ROOT, "paper_1911_12070_amd", "csrc", "vx_mlp.hip")).read()
    body = src[src.index("float gelu_fit(float x)"):]
    body = body[:body.index("}")]
    m = re.search(r"fmaf\(fmaf\(t, ([-+0-9.e]+)f, ([-+0-9.e]+)f\), t, ([-+0-9.e]+)f\)", body)
    assert m, "gelu_fit's polynomial not found"
    clamp = re.search(r"fmed3f\(x, (-?[0-9.]+)f, ([0-9.]+)f\)", body)
    assert clamp
    return [np.float32(v) for v in m.groups()], float(clamp.group(1)), float(clamp.group(2))


def gelu_fit(x, c2, c1, c0, lo, hi):
    x = x.astype(np.float32)
    xc = np.clip(x, np.float32(lo), np.float32(hi))
    t = xc * xc
    q = (t * c2 + c1) * t + c0
    with np.errstate(over="ignore"):
        return x / (np.float32(1) + np.exp2(xc * q))


def test_gelu_fit_error_bound():
    (c2, c1, c0), lo, hi = fit_constants()
    assert (lo, hi) == (-8.0, 8.0)
    x = np.concatenate([np.linspace(-40, 40, 800_001), [-1e30, -1e6, 1e6, 1e30, 0.0]])
    exact = x * 0.5 * (1.0 + erf(x / np.sqrt(2.0)))
    got = gelu_fit(x, c2, c1, c0, lo, hi).astype(np.float64)
    err = np.abs(got - exact)
    small = np.abs(x) < 1e3
    assert err[small].max() < 3e-5, (err[small].max(), x[small][err[small].argmax()])
    # far outside the clamp: x itself above, 0 below (relative to the value's size)
    big = ~small
    assert np.all(np.abs(got[big] - np.maximum(x[big], 0.0)) <= 1e-6 * np.abs(x[big]))
    # the fit is the sigmoid of an odd function of x: gelu(x) - gelu(-x) = x
    y = np.linspace(0, 8, 10_001)
    d = gelu_fit(y, c2, c1, c0, lo, hi).astype(np.float64) - gelu_fit(-y, c2, c1, c0, lo, hi).astype(np.float64)
    assert np.abs(d - y).max() < 1e-5
