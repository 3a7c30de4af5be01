"""Accuracy of the float cosine of the fixed-width-row engine (cos x = -sin(|x| - pi/2) with a
degree-9 odd polynomial) on wrapped angles |x| <= pi_f, pinned against the float64 cosine.

The coefficients are read from the kernel source, so the pin checks the constants the kernel
uses.  The float32 evaluation is emulated: every operation rounded to float32, each fused
multiply-add formed exactly in float64 and rounded once to float32 (float32 products are exact
in float64; the sum rounds at most twice, which moves the result by at most one float32 ulp in
rare halfway cases).  Bar: 2 ulp of the result, and 1.1e-7 absolute near the zeros of the
cosine, where the representation of x itself (ulp(pi/2) / 2 = 6e-8) already limits any float
evaluation."""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2312_05837_amd", "csrc", "kernels_ds.hip")


def _constants():
    src = open(SRC).read()
    c = {}
    for name in ("WCOS_S1", "WCOS_S2", "WCOS_S3", "WCOS_S4"):
        c[name] = np.float32(float(re.search(name + r"\s*=\s*([-+0-9.e]+)f", src).group(1)))
    body = src[src.index("__device__ inline float wrapped_cos(float x)"):]
    body = body[:body.index("}")]
    hi, lo = re.findall(r"([-+]?[0-9.]+e?[-+0-9]*)f", body)[:2]
    return c, np.float32(float(hi)), np.float32(float(lo))


def _fma(a, b, c):
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64)).astype(np.float32)


def wrapped_cos(x):
    c, hi, lo = _constants()
    x = np.asarray(x, np.float32)
    f = ((np.abs(x) - hi).astype(np.float32) - lo).astype(np.float32)
    z = (f * f).astype(np.float32)
    p = _fma(z, c["WCOS_S4"], c["WCOS_S3"])
    p = _fma(z, p, c["WCOS_S2"])
    p = _fma(z, p, c["WCOS_S1"])
    return _fma((-f * z).astype(np.float32), p, -f)


def test_pi_over_two_split():
    _, hi, lo = _constants()
    assert abs(float(hi) + float(lo) - np.pi / 2) < 4e-15


def _check(x):
    got = wrapped_cos(x).astype(np.float64)
    ref = np.cos(x.astype(np.float64))
    err = np.abs(got - ref)
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    small = np.abs(ref) < 1e-3
    assert np.all(err[~small] <= 2.0 * ulp[~small]), (err[~small] / ulp[~small]).max()
    assert not small.any() or err[small].max() <= 1.1e-7


def test_cos_on_random_wrapped_angles():
    pi_up = float(np.nextafter(np.float32(np.pi), np.float32(4)))
    x = np.random.default_rng(5837).uniform(-pi_up, pi_up, 5_000_000).astype(np.float32)
    _check(x)


def test_cos_around_zeros_extrema_and_the_wrap_ends():
    for centre in (0.0, np.pi / 2, -np.pi / 2, np.pi, -np.pi):
        c = np.float32(centre).view(np.int32)
        x = (c + np.arange(-300000, 300001, dtype=np.int64)).astype(np.int32).view(np.float32)
        x = x[np.isfinite(x) & (np.abs(x) <= np.nextafter(np.float32(np.pi), np.float32(4)))]
        _check(x)
