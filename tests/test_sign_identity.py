"""The persistent engine decides the next vertex of a wrapped angle x (|x| <= pi plus a rounding
error) as (x < 0) xor (|x| >= pi_f), pi_f the float just above pi, instead of evaluating the sine.
This pins that identity against the sign of the float64 sine (exact in sign for float32 inputs:
the smallest |sin x| away from 0 is |sin pi_f| ~ 8.7e-8) on every float32 within 2^20 ulps of
0, +-pi/2 and +-pi and on 10^7 random angles in [-4, 4]."""
import numpy as np

PI_F = np.float32(np.pi)


def wrapped_sin_neg(x):
    return (x < 0) != (np.abs(x) >= PI_F)


def _window(center, ulps):
    c = np.float32(center).view(np.int32)
    bits = np.arange(int(c) - ulps, int(c) + ulps + 1, dtype=np.int64).astype(np.int32)
    x = bits.view(np.float32)
    return x[np.isfinite(x)]


def test_pi_f_is_above_pi():
    assert float(PI_F) > np.pi and float(np.nextafter(PI_F, np.float32(0))) < np.pi


def test_identity_near_every_sign_change_and_quadrant_boundary():
    xs = [_window(c, 1 << 20) for c in (np.pi, -np.pi, np.pi / 2, -np.pi / 2)]
    zero = np.arange(0, 1 << 21, dtype=np.int32).view(np.float32)  # +0 and the smallest positives
    xs += [zero, -zero]
    for x in xs:
        ref = np.sin(x.astype(np.float64)) < 0
        assert np.array_equal(wrapped_sin_neg(x), ref)


def test_identity_on_random_angles():
    rng = np.random.default_rng(2312)
    x = rng.uniform(-4.0, 4.0, 10_000_000).astype(np.float32)
    assert np.array_equal(wrapped_sin_neg(x), np.sin(x.astype(np.float64)) < 0)
