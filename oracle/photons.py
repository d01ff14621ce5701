"""Universal synchrotron photon spectrum for the photon-by-photon radiation
model (test infrastructure: the oracle's own computation).

Paper section "Synchrotron radiation models and compensation": besides the
mean energy loss, the quantum model emits individual photons.  For a particle
of Lorentz factor gamma bending with curvature h, a photon's energy is
x u_c with u_c = (3/2) hbar_c gamma^3 h, and x follows the photon-number
density n(x) = 3/(5 pi) int_x^inf K_{5/3}(t) dt (normalised to one photon).
With K_nu(t) = int_0^inf exp(-t cosh a) cosh(nu a) da the density, the
tail Q(x) = P(X > x) and the head F(x) = 1 - Q(x) become single integrals
over a:
    n(x) = 3/(5 pi) int_0^inf exp(-x cosh a) cosh(5a/3) / cosh a   da
    Q(x) = 3/(5 pi) int_0^inf exp(-x cosh a) cosh(5a/3) / cosh^2 a da
    F(x) = 3/(5 pi) int_0^inf (1 - exp(-x cosh a)) cosh(5a/3) / cosh^2 a da
They are evaluated here by the trapezoidal rule with step 1/16 on [0, 120]
(even integrands analytic in |Im a| < pi/2: the rule converges
geometrically) with exactly rounded summation (math.fsum).

The sampling table: g_i = x^(1/3) with Q(x) = exp(-s_i), s_i = i/64,
i = 0 .. 2432, each rounded to single precision; a photon's x is g^3 with g
interpolated linearly at s = -ln u.  Each g_i is found by Newton's method in
y = x^(1/3), on F(y^3) = 1 - exp(-s) for s <= ln 2 and on ln Q(y^3) = -s
beyond, starting from the previous node's root.
"""
from __future__ import annotations

import math

import numpy as np

NODES = 2433
STEP_INV = 64.0

_A = np.arange(0.0, 120.0 + 1e-9, 1.0 / 16.0)
_W = np.full(len(_A), 1.0 / 16.0)
_W[0] = 1.0 / 32.0
_CH = np.cosh(_A)
_B = _W * np.cosh(5.0 * _A / 3.0) / (_CH * _CH)
_NORM = 3.0 / (5.0 * math.pi)


def tail(x: float) -> float:
    """Q(x): probability that a photon's energy exceeds x u_c."""
    return _NORM * math.fsum(_B * np.exp(-x * _CH))


def head(x: float) -> float:
    """F(x) = 1 - Q(x), accurate for small x."""
    return _NORM * math.fsum(_B * -np.expm1(-x * _CH))


def density(x: float) -> float:
    """n(x), the photon-number density (x > 0)."""
    return _NORM * math.fsum(_B * _CH * np.exp(-x * _CH))


def _root(s: float, y: float) -> float:
    last = math.inf
    for _ in range(60):
        x = y * y * y
        if s <= math.log(2.0):
            phi = head(x) + math.expm1(-s)
            dphi = density(x) * 3.0 * y * y
        else:
            q = tail(x)
            phi = math.log(q) + s
            dphi = -density(x) / q * 3.0 * y * y
        yn = y - phi / dphi
        if yn <= 0.0:
            yn = 0.5 * y
        size = abs(yn - y)
        y = yn
        if size <= 1e-17 * y or size >= last:
            break
        last = size
    return y


_TABLE = None


def table() -> np.ndarray:
    """The sampling table g_0 .. g_2432 (float64 array of single-precision
    values), computed once per process."""
    global _TABLE
    if _TABLE is None:
        g = np.zeros(NODES)
        y = 0.0
        for i in range(1, NODES):
            s = i / STEP_INV
            # the small-x law F(x) ~ 1.2315 x^(1/3) starts the first node
            y = _root(s, s / 1.2315 if i == 1 else y)
            g[i] = y
        _TABLE = g.astype(np.float32).astype(np.float64)
    return _TABLE


def photon_x(s) -> np.ndarray:
    """x at s = -ln u from the table (linear interpolation of g, then g^3),
    vectorised for statistics; the tracking code evaluates the same
    interpolation with a fused multiply-add."""
    g = table()
    v = np.asarray(s, dtype=np.float64) * STEP_INV
    i = np.minimum(v.astype(np.int64), NODES - 2)
    f = v - i
    gv = g[i] + f * (g[i + 1] - g[i])
    return gv * gv * gv
