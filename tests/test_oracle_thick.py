"""Pins of the thick-element slicing (drift-kick-drift slices with the kicks
at the slice midpoints, a second-order symplectic splitting): the sliced
linear maps converge to the exact thick quadrupole and sector-bend matrices
at second order in the slice length, stay symplectic, and a quadrupole of
zero gradient is a drift."""
import math

import numpy as np
import pytest

from paper_2310_00317_amd import inputs as I

REF = I.PROTON_450GEV


def quad_exact(k, L):
    if k > 0:
        w = math.sqrt(k)
        return np.array([[math.cos(w * L), math.sin(w * L) / w], [-w * math.sin(w * L), math.cos(w * L)]])
    w = math.sqrt(-k)
    return np.array([[math.cosh(w * L), math.sinh(w * L) / w], [w * math.sinh(w * L), math.cosh(w * L)]])


def jac(oracle_mod, el):
    return oracle_mod.jacobian(el, REF, h=np.array([1e-8, 1e-10, 1e-8, 1e-10, 1e-7, 1e-9]))


def test_expansion_layout(oracle_mod):
    el = oracle_mod.expand_thick(I.line([I.marker(), I.quadrupole(2.0, 0.3, 0.01, slices=3)]))
    assert list(el["type"]) == [I.MARKER, I.DRIFT, I.MULTIPOLE, I.DRIFT, I.MULTIPOLE, I.DRIFT,
                                I.MULTIPOLE, I.DRIFT]
    d = 2.0 / 3.0
    assert np.allclose(el["length"][[1, 3, 5, 7]], [d / 2, d, d, d / 2], rtol=0, atol=1e-16)
    assert abs(el["length"][1::2].sum() - 2.0) < 1e-15
    assert np.allclose(el["knl"][[2, 4, 6], 1], 0.3 * d) and np.allclose(el["ksl"][[2, 4, 6], 1], 0.01 * d)


@pytest.mark.parametrize("k", [0.4, -0.25])
def test_thick_quadrupole_converges_at_second_order(oracle_mod, k):
    L = 2.0
    errs = []
    for n in (8, 16, 32):
        J = jac(oracle_mod, I.line([I.quadrupole(L, k, slices=n)]))
        ex, ey = quad_exact(k, L), quad_exact(-k, L)
        errs.append(max(np.max(np.abs(J[:2, :2] - ex)), np.max(np.abs(J[2:4, 2:4] - ey))))
        assert oracle_mod.symplectic_error(J) < 1e-7
        assert np.max(np.abs(J[:2, 2:4])) < 1e-9  # no coupling without skew gradient
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4
    assert errs[2] < 2e-3 * abs(k) * L * L


def test_sector_bend_converges_at_second_order(oracle_mod):
    L, theta = 3.0, 0.1
    h = theta / L
    exact = np.array([[math.cos(h * L), math.sin(h * L) / h], [-h * math.sin(h * L), math.cos(h * L)]])
    disp = np.array([(1 - math.cos(h * L)) / h, math.sin(h * L)])
    errs = []
    for n in (8, 16, 32):
        J = jac(oracle_mod, I.line([I.sbend(L, theta, slices=n)]))
        # momentum column: pzeta = ptau / beta0 and d delta / d pzeta = 1 at delta = 0
        errs.append(max(np.max(np.abs(J[:2, :2] - exact)), np.max(np.abs(J[:2, 5] - disp))))
        assert np.allclose(J[2:4, 2:4], [[1.0, L], [0.0, 1.0]], atol=1e-9)  # vertical: a drift
        assert oracle_mod.symplectic_error(J) < 1e-7
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


def test_zero_gradient_quadrupole_is_a_drift(oracle_mod):
    c = np.array([[1e-3, 2e-4, -5e-4, 1e-4, 0.01, 1e-4]])
    a = oracle_mod.init(c, REF)
    oracle_mod.track(I.line([I.quadrupole(4.0, 0.0, slices=5)]), REF, a, 1)
    b = oracle_mod.init(c, REF)
    oracle_mod.track(I.line([I.drift(4.0)]), REF, b, 1)
    for f in ("x", "px", "y", "py", "zeta"):
        assert abs(getattr(a, f)[0] - getattr(b, f)[0]) <= 1e-15 * max(1e-3, abs(getattr(b, f)[0]))
