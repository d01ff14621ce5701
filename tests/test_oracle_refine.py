"""Pins of the oracle's loss-location refinement (backtracking plus a
polygon-interpolated aperture, paper section on beam-loss localisation and
its aperture figure) against closed forms, invariances and an independent
brute-force scan.

The paper gives the method in one sentence; the reading under test (rays at
angles 2 pi k / M from each aperture's origin, vertices interpolated
linearly in s between the previous aperture and the one that caught the
particle, sub-steps of ds then bisection) is stated with the oracle.
"""
import math

import numpy as np
import pytest

from paper_2310_00317_amd import inputs as I

REF = I.PROTON_450GEV


def lost_once(oracle_mod, elements, coords):
    el = I.line(elements)
    p = oracle_mod.init(np.atleast_2d(coords), REF)
    oracle_mod.track(el, REF, p, 1)
    return el, p


def pz_of(px, py, delta=0.0):
    return math.sqrt((1.0 + delta) ** 2 - px * px - py * py)


def test_straight_exit_through_square(oracle_mod):
    a, L, x0, y0, px = 0.01, 10.0, 0.005, 0.002, 1e-3
    el, p = lost_once(oracle_mod, [I.ap_rect(-a, a, -a, a), I.drift(L), I.ap_rect(-a, a, -a, a)],
                      [x0, px, y0, 0.0, 0.0, 0.0])
    assert p.state[0] == 0 and p.at_element[0] == 2
    s, x, y = oracle_mod.refine_losses(el, REF, p, n_vertices=8, ds=0.01, n_bisect=40)
    s_star = (a - x0) * pz_of(px, 0.0) / px
    assert abs(s[0] - s_star) < 1e-9
    assert abs(x[0] - a) < 1e-9 and abs(y[0] - y0) < 1e-12
    # without bisection: the end of the first sub-step past the crossing
    s0, _, _ = oracle_mod.refine_losses(el, REF, p, n_vertices=8, ds=0.01, n_bisect=0)
    assert s_star <= s0[0] < s_star + 0.01 + 1e-12


def test_tapered_square_closed_form(oracle_mod):
    a1, a2, L, x0 = 0.02, 0.01, 10.0, 0.0125  # off the midpoint: w* = 0.75
    el, p = lost_once(oracle_mod, [I.ap_rect(-a1, a1, -a1, a1), I.drift(L),
                                   I.ap_rect(-a2, a2, -a2, a2)],
                      [x0, 0.0, 0.001, 0.0, 0.0, 0.0])
    assert p.state[0] == 0 and p.at_element[0] == 2
    s, x, _ = oracle_mod.refine_losses(el, REF, p, n_vertices=16, ds=0.05, n_bisect=40)
    # the right side moves as a1 + (a2 - a1) s / L and meets x0 at L (x0-a1)/(a2-a1)
    assert abs(s[0] - L * (x0 - a1) / (a2 - a1)) < 1e-9
    assert abs(x[0] - x0) < 1e-15


def test_shifted_aperture_closed_form(oracle_mod):
    a, dx, L, x0 = 0.01, 0.004, 10.0, -0.009  # w* = 0.25
    el, p = lost_once(oracle_mod, [I.ap_rect(-a, a, -a, a), I.drift(L), I.xyshift(dx, 0.0),
                                   I.ap_rect(-a, a, -a, a), I.xyshift(-dx, 0.0)],
                      [x0, 0.0, 0.0005, 0.0, 0.0, 0.0])
    assert p.state[0] == 0 and p.at_element[0] == 3
    s, x, _ = oracle_mod.refine_losses(el, REF, p, n_vertices=8, ds=0.1, n_bisect=40)
    # left side of the shifted square in the line frame: -a + w dx
    assert abs(s[0] - L * (x0 + a) / dx) < 1e-9
    assert abs(x[0] - x0) < 1e-15


def test_drift_lengths_and_kicks_between_apertures(oracle_mod):
    # two drifts with a thin quadrupole between them: the path bends at the
    # quadrupole; crossing of the exit square computed from the kinked line
    a, L1, L2, x0, px0, k1 = 0.01, 3.0, 4.0, 0.004, 5e-4, 0.2
    el, p = lost_once(oracle_mod, [I.ap_rect(-a, a, -a, a), I.drift(L1), I.multipole(knl=[0.0, -k1]),
                                   I.drift(L2), I.ap_rect(-a, a, -a, a)],
                      [x0, px0, 0.0003, 0.0, 0.0, 0.0])
    assert p.state[0] == 0 and p.at_element[0] == 4
    s, x, _ = oracle_mod.refine_losses(el, REF, p, n_vertices=8, ds=0.01, n_bisect=40)
    x1 = x0 + px0 * L1 / pz_of(px0, 0.0)
    assert x1 < a  # still inside at the quadrupole
    y0 = 0.0003
    px1 = px0 + k1 * x1  # knl1 = -k1: dpx = -knl1 x = +k1 x
    py1 = -k1 * y0       # and dpy = +knl1 y = -k1 y
    s_star = L1 + (a - x1) * pz_of(px1, py1) / px1
    assert abs(s[0] - s_star) < 1e-9
    assert abs(x[0] - a) < 1e-9


@pytest.mark.parametrize("theta", [0.3, -1.1, 2.5])
def test_rotated_and_shifted_frame_invariance(oracle_mod, theta):
    # the same problem seen through a rotated and shifted line frame: the
    # refined s is unchanged and the loss point transforms with the frame
    r1, r2, L = 0.012, 0.009, 8.0
    u0 = np.array([0.003, 1e-3, -0.002, -8e-4, 0.0, 1e-4])
    base = [I.ap_ellipse(r1, 0.8 * r1), I.drift(L), I.ap_ellipse(r2, 1.1 * r2)]
    el_u, p_u = lost_once(oracle_mod, base, u0)
    assert p_u.state[0] == 0
    s_u, x_u, y_u = oracle_mod.refine_losses(el_u, REF, p_u, n_vertices=64, ds=0.02, n_bisect=40)
    d = (0.001, -0.0005)
    c, sn = math.cos(theta), math.sin(theta)
    # line coordinates whose rotated then shifted image is u0
    def back(x, y):
        x, y = x + d[0], y + d[1]
        return c * x - sn * y, sn * x + c * y
    vx, vy = back(u0[0], u0[2])
    vpx, vpy = c * u0[1] - sn * u0[3], sn * u0[1] + c * u0[3]
    el_r, p_r = lost_once(oracle_mod, [I.srotation(theta), I.xyshift(*d)] + base
                          + [I.xyshift(-d[0], -d[1]), I.srotation(-theta)],
                          [vx, vpx, vy, vpy, 0.0, 1e-4])
    assert p_r.state[0] == 0 and p_r.at_element[0] == p_u.at_element[0] + 2
    s_r, x_r, y_r = oracle_mod.refine_losses(el_r, REF, p_r, n_vertices=64, ds=0.02, n_bisect=40)
    assert abs(s_r[0] - s_u[0]) < 1e-9
    ex, ey = back(x_u[0], y_u[0])
    assert abs(x_r[0] - ex) < 1e-11 and abs(y_r[0] - ey) < 1e-11


# ----------------------------------------------------------- brute force
def _radius(kind, prm, ang):
    c, s = np.cos(ang), np.sin(ang)
    if kind == "circle":
        return np.full_like(ang, prm[0])
    if kind == "ellipse":
        return 1.0 / np.sqrt(c * c / prm[0] ** 2 + s * s / prm[1] ** 2)
    xmin, xmax, ymin, ymax = prm
    with np.errstate(divide="ignore"):
        cand = np.stack([np.where(c > 0, xmax / c, np.inf), np.where(c < 0, xmin / c, np.inf),
                         np.where(s > 0, ymax / s, np.inf), np.where(s < 0, ymin / s, np.inf)])
    return cand.min(axis=0)


def _inside(px, py, vx, vy):
    # even-odd rule, vectorised over the edges
    xi, yi, xj, yj = vx, vy, np.roll(vx, -1), np.roll(vy, -1)
    straddle = (yi > py) != (yj > py)
    with np.errstate(divide="ignore", invalid="ignore"):
        xc = xi + (py - yi) * (xj - xi) / (yj - yi)
    return bool(np.count_nonzero(straddle & (px < xc)) % 2)


SHAPES = {
    "circle": (I.ap_circle, lambda r: (r.uniform(0.008, 0.012),)),
    "ellipse": (I.ap_ellipse, lambda r: (r.uniform(0.008, 0.014), r.uniform(0.006, 0.012))),
    "rect": (I.ap_rect, lambda r: (-r.uniform(0.006, 0.012), r.uniform(0.006, 0.012),
                                    -r.uniform(0.006, 0.012), r.uniform(0.006, 0.012))),
}


@pytest.mark.parametrize("case", range(12))
def test_brute_force_scan_drift_only(oracle_mod, case):
    rng = np.random.default_rng(900 + case)
    kinds = list(SHAPES)
    ka, kb = kinds[case % 3], kinds[(case // 3) % 3]
    pa, pb = SHAPES[ka][1](rng), SHAPES[kb][1](rng)
    L, M = float(rng.uniform(2.0, 9.0)), 32
    for _ in range(200):
        u = np.array([rng.uniform(-0.005, 0.005), rng.normal(0, 2e-3), rng.uniform(-0.005, 0.005),
                      rng.normal(0, 2e-3), 0.0, 0.0])
        el, p = lost_once(oracle_mod, [SHAPES[ka][0](*pa), I.drift(L), SHAPES[kb][0](*pb)], u)
        if p.state[0] == 0 and p.at_element[0] == 2:
            break
    else:
        pytest.skip("no particle lost at the second aperture")
    s, x, y = oracle_mod.refine_losses(el, REF, p, n_vertices=M, ds=0.05, n_bisect=40)
    # straight line back from the stored loss coordinates
    pz = pz_of(u[1], u[3])
    xL, yL = p.x[0], p.y[0]
    ang = 2.0 * np.pi * np.arange(M) / M
    ra, rb = _radius(ka, pa, ang), _radius(kb, pb, ang)
    va = (ra * np.cos(ang), ra * np.sin(ang))
    vb = (rb * np.cos(ang), rb * np.sin(ang))
    h = 1e-4
    grid = np.arange(h, L + h / 2, h)
    first = L
    for sv in grid:
        w = sv / L
        bx, by = xL - u[1] / pz * (L - sv), yL - u[3] / pz * (L - sv)
        vx = va[0] + w * (vb[0] - va[0])
        vy = va[1] + w * (vb[1] - va[1])
        if not _inside(bx, by, vx, vy):
            first = sv
            break
    # the oracle finds the first sub-step of 0.05 m whose end is outside, then
    # bisects it; when the path leaves and re-enters within one sub-step the
    # two may differ, which these smooth shapes do not produce
    assert first - h - 1e-9 <= s[0] <= first + 1e-9
    assert 0.0 <= s[0] <= L
