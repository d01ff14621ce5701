"""Pins of the tracker's own sine, cosine and logarithm (series evaluations
that both implementations follow step by step): agreement with the C
library within the stated ulps over the ranges the maps use, exact special
values, and the identities that a wrong coefficient, sign or quadrant breaks."""
import math

import numpy as np

import oracle


def _ulps(a, b):
    return abs(a - b) / math.ulp(b) if b != 0 else abs(a - b) / math.ulp(0.0)


def test_sin_cos_against_libm():
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.uniform(-40, 40, 40000), rng.uniform(-1e-3, 1e-3, 2000),
                         (np.arange(-64, 65) * math.pi / 4)])
    assert max(_ulps(oracle.xsin(x), math.sin(x)) for x in xs) <= 1.0
    assert max(_ulps(oracle.xcos(x), math.cos(x)) for x in xs) <= 1.0


def test_log_against_libm():
    rng = np.random.default_rng(4)
    xs = np.concatenate([rng.random(40000), (np.arange(1, 2000) + 0.5) * 2.0 ** -52,
                         10.0 ** rng.uniform(-300, 300, 4000), 1 + rng.uniform(-1e-6, 1e-6, 2000)])
    assert max(_ulps(oracle.xlog(x), math.log(x)) for x in xs) <= 2.0


def test_special_values_and_identities():
    assert oracle.xsin(0.0) == 0.0 and oracle.xcos(0.0) == 1.0 and oracle.xlog(1.0) == 0.0
    for k in range(-20, 21):
        assert abs(oracle.xlog(2.0 ** k) - k * math.log(2)) <= 2 * math.ulp(max(abs(k), 1) * 0.7)
    rng = np.random.default_rng(5)
    for x in rng.uniform(-10, 10, 2000):
        s, c = oracle.xsin(x), oracle.xcos(x)
        assert abs(s * s + c * c - 1) < 4e-16
        assert oracle.xsin(-x) == -s and oracle.xcos(-x) == c          # odd / even
        assert abs(oracle.xsin(x + math.pi / 2) - c) < 4e-15           # quarter shift
    for x in rng.uniform(1e-3, 1, 2000):
        assert abs(oracle.xlog(x) + oracle.xlog(1 / x)) < 4e-15        # log(1/x) = -log x
