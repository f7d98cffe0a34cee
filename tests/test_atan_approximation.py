"""Error bound of the kernels' fast_atan2 (the azimuth of a predicted point,
the centre of its search window).

The kernel evaluates atan on [0, 1] by an odd polynomial of degree 15 (eight
coefficients in t^2), after reducing the argument to one octant.  This test
reads the coefficients from the kernel source, (1) refits the polynomial by
weighted least squares on [0, 1] and checks that the source's coefficients
do as well as that fit, and (2) evaluates the function as the kernel does,
in float32 with single-rounded multiply-adds and a reciprocal within one ulp,
over a dense grid of directions, against numpy's double-precision arctan2.
The window pads the azimuth by 1e-5 rad, so the bound that matters is far
below that; the test requires 4e-7 rad (the float32 rounding of results
near pi, 1.2e-7 each, dominates).
"""
import math
import os
import re

import numpy as np

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1702_06359_amd", "csrc",
                   "mkf_device.hpp")


def kernel_coefficients():
    src = open(SRC).read()
    body = src[src.index("float fast_atan2("):]
    body = body[:body.index("return copysignf")]
    # r = fmaf(v, c_hi, c_next) then r = fmaf(v, r, c) ...: the constants in order, highest power first
    nums = [float(x) for x in re.findall(r"fmaf\(v, (?:r, )?(-?[0-9.]+)f(?:, (-?[0-9.]+)f)?\)", body)
            for x in x if x]
    return np.array(nums[::-1])          # ascending powers of v = t^2


def fma32(a, b, c):
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def atan_poly32(t, coef):
    """r = c7; r = r v + c_k ...; atan ~ t r, all in float32 as the kernel does."""
    v = (t * t).astype(np.float32)
    c = coef.astype(np.float32)
    r = fma32(v, np.full_like(v, c[7]), np.full_like(v, c[6]))
    for k in range(5, -1, -1):
        r = fma32(v, r, np.full_like(v, c[k]))
    return (t * r).astype(np.float32)


def fast_atan2_32(y, x, coef, rcp_ulps=0):
    ax, ay = np.abs(x), np.abs(y)
    mx, mn = np.maximum(ax, ay), np.minimum(ax, ay)
    inv = (1.0 / mx.astype(np.float64)).astype(np.float32)
    if rcp_ulps:
        inv = np.nextafter(inv, np.float32(np.inf) if rcp_ulps > 0 else np.float32(0))
    t = (mn * inv).astype(np.float32)
    a = atan_poly32(t, coef)
    a = np.where(ay > ax, (np.float32(1.57079632679) - a).astype(np.float32), a)
    a = np.where(x < 0, (np.float32(3.14159265359) - a).astype(np.float32), a)
    return np.copysign(a, y)


def test_coefficients_are_a_least_squares_fit_of_atan():
    coef = kernel_coefficients()
    assert coef.shape == (8,)
    t = np.linspace(0.0, 1.0, 200001)
    # odd basis t, t^3, ..., t^15, fitted to atan(t)
    A = np.stack([t ** (2 * k + 1) for k in range(8)], 1)
    fit, *_ = np.linalg.lstsq(A, np.arctan(t), rcond=None)
    err_src = np.abs(A @ coef - np.arctan(t)).max()
    err_fit = np.abs(A @ fit - np.arctan(t)).max()
    assert err_src < 1.2e-7 and err_src < 3 * err_fit, (err_src, err_fit)


def test_fast_atan2_error_bound_in_float32():
    coef = kernel_coefficients()
    ang = np.linspace(-math.pi, math.pi, 2_000_001)
    worst = 0.0
    for r in (4.0, 40.0, 0.013, 1e3):
        x = (r * np.cos(ang)).astype(np.float32)
        y = (r * np.sin(ang)).astype(np.float32)
        ref = np.arctan2(y.astype(np.float64), x.astype(np.float64))
        for ulps in (0, 1, -1):
            got = fast_atan2_32(y, x, coef, ulps).astype(np.float64)
            d = np.abs(np.remainder(got - ref + math.pi, 2 * math.pi) - math.pi)
            worst = max(worst, float(d.max()))
    print(f"fast_atan2 worst error {worst:.3e} rad")
    assert worst < 4e-7
