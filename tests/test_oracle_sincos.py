"""Pins for the oracle's FP32 sin/cos of 2*pi*u (Cephes-style, Sec. 3.2.3):
within 2 ulp of libm's FP64 sin/cos, exact at the quarter turns."""
import numpy as np

import oracle as O


def _ulp32(x):
    x = np.float32(abs(x))
    return float(np.spacing(x)) if x > 0 else float(np.spacing(np.float32(0)))


def test_quarter_turns_exact():
    assert O.sincos2pi(0.0) == (0.0, 1.0)
    assert O.sincos2pi(0.25) == (1.0, 0.0) or O.sincos2pi(0.25) == (1.0, -0.0)
    s, c = O.sincos2pi(0.5)
    assert abs(s) == 0.0 and c == -1.0
    s, c = O.sincos2pi(0.75)
    assert s == -1.0 and abs(c) == 0.0


def test_within_two_ulp_of_fp64():
    rng = np.random.default_rng(1)
    us = np.concatenate([rng.random(20000, dtype=np.float32),
                         (np.arange(4096, dtype=np.float32) / 4096.0),
                         np.float32([1e-7, 0.125, 0.375, 0.999999, 0.2499999, 0.2500001])])
    worst = 0.0
    for u in us:
        s, c = O.sincos2pi(float(u))
        rs, rc = np.sin(2 * np.pi * np.float64(u)), np.cos(2 * np.pi * np.float64(u))
        # error in units of the FP32 ulp of the result (absolute floor near zero:
        # the ulp of the largest term, 2^-24, since the argument itself carries
        # an FP32 rounding of 2*pi*u)
        es = abs(s - rs) / max(_ulp32(rs), 2.0 ** -26)
        ec = abs(c - rc) / max(_ulp32(rc), 2.0 ** -26)
        worst = max(worst, es, ec)
    assert worst <= 2.0, worst


def test_pythagoras_and_symmetry():
    for u in np.linspace(0, 1, 777, endpoint=False, dtype=np.float32):
        s, c = O.sincos2pi(float(u))
        assert abs(s * s + c * c - 1.0) < 4e-7
        s2, c2 = O.sincos2pi(float(np.float32(-u)))
        assert s2 == -s and c2 == c
