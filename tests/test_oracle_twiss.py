"""Pins of the oracle's optics by tracking (closed orbit by Newton's method,
central-difference Jacobian, uncoupled normal form, propagation through the
line; paper section "Twiss module") against thin-lens closed forms, the
drift propagation law, the closed orbit of a single kick, and dispersion
taken as the momentum derivative of closed orbits found independently."""
import math

import numpy as np
import pytest

from paper_2310_00317_amd import inputs as I

EREF = I.ELECTRON_45GEV6

REF = I.PROTON_450GEV


def fodo_closed_form():
    f, L = I.CFG1_F, I.CFG1_HALF
    mu = math.acos(1.0 - L * L / (2.0 * f * f))
    bmax = 2.0 * L * (1.0 + math.sin(mu / 2)) / math.sin(mu)
    bmin = 2.0 * L * (1.0 - math.sin(mu / 2)) / math.sin(mu)
    return f, L, mu, bmax, bmin


@pytest.mark.parametrize("sext", [False, True])
def test_fodo_ring_thin_lens_closed_forms(oracle_mod, sext):
    el = I.cfg1_lattice(rf_on=False, sextupoles=sext)
    tw = oracle_mod.twiss(el, REF, h=1e-10)
    f, L, mu, bmax, bmin = fodo_closed_form()
    assert tw["iterations"] == 0 and tw["residual"] == 0.0  # the orbit is the axis
    assert abs(tw["qx"] - 100 * mu / (2 * math.pi)) < 1e-9
    assert abs(tw["qy"] - 100 * mu / (2 * math.pi)) < 1e-9
    qf, qd = 1 + 8 * np.arange(100), 5 + 8 * np.arange(100)
    for b, a, m, big, small in (("betx", "alfx", "mux", qf, qd), ("bety", "alfy", "muy", qd, qf)):
        assert np.allclose(tw[b][big], bmax, rtol=1e-9, atol=0)
        assert np.allclose(tw[b][small], bmin, rtol=1e-9, atol=0)
        # entry of a thin focusing lens of the symmetric cell: alpha = -beta / (2 f)
        assert np.allclose(tw[a][big], -bmax / (2 * f), rtol=1e-8, atol=0)
        assert np.allclose(np.diff(tw[m][qf]), mu, rtol=0, atol=1e-10)
    assert np.allclose(tw["dx"], 0.0, atol=1e-9) and np.allclose(tw["dy"], 0.0, atol=1e-9)


def test_drift_propagation_law(oracle_mod):
    el = I.cfg1_lattice(rf_on=False)
    tw = oracle_mod.twiss(el, REF, h=1e-10)
    drifts = np.nonzero(el["type"] == I.DRIFT)[0]
    for p in ("x", "y"):
        b, a = tw["bet" + p], tw["alf" + p]
        g = (1 + a * a) / b
        L = el["length"][drifts]
        e = drifts
        assert np.allclose(b[e + 1], b[e] - 2 * a[e] * L + g[e] * L * L, rtol=1e-9)
        assert np.allclose(a[e + 1], a[e] - g[e] * L, rtol=1e-9, atol=1e-9)
        # phase advance through a drift: atan of L / (beta - alpha L)
        dmu = np.arctan2(L, b[e] - a[e] * L)
        assert np.allclose(tw["mu" + p][e + 1] - tw["mu" + p][e], dmu, atol=1e-10)


def test_single_kick_closed_orbit(oracle_mod):
    # near the integer tune the orbit is 40x the kick's local amplitude; a
    # small kick keeps the exact drift's nonlinearity out of the comparison
    theta = 1e-8
    base = list(I.cfg1_lattice(rf_on=False, sextupoles=False))
    k = 41  # a corrector after the drift ending cell 5
    el = I.line(base[:k] + [I.multipole(knl=[-theta])] + base[k:])
    tw0 = oracle_mod.twiss(I.line(base), REF, h=1e-10)
    tw = oracle_mod.twiss(el, REF, h=1e-10)
    assert tw["iterations"] >= 1 and tw["residual"] < 1e-15
    Q = tw0["qx"]
    # rows of the kicked ring without the corrector map onto the plain ring
    rows = np.r_[np.arange(0, k + 1), np.arange(k + 2, len(el) + 1)]
    bk, mk = tw0["betx"][k], tw0["mux"][k]
    b, m = tw0["betx"], tw0["mux"]
    xco = theta * np.sqrt(b * bk) * np.cos(math.pi * Q - np.abs(m - mk)) / (2 * math.sin(math.pi * Q))
    got = tw["x"][rows]
    assert np.max(np.abs(got - xco)) < 1e-7 * np.max(np.abs(xco))
    assert np.max(np.abs(tw["y"])) == 0.0


def bend_ring(n_cells=20, theta=0.05, k=0.04, L=10.0):
    cell = [I.multipole(knl=[0.0, k]), I.multipole(knl=[theta], hxl=theta, length=2.0), I.drift(L),
            I.multipole(knl=[0.0, -k]), I.multipole(knl=[theta], hxl=theta, length=2.0),
            I.drift(L)]
    return I.line(cell * n_cells)


def test_dispersion_is_the_momentum_derivative_of_the_closed_orbit(oracle_mod):
    el = bend_ring()
    tw = oracle_mod.twiss(el, REF, h=1e-9, hd=1e-8)
    eps = 1e-6
    tp = oracle_mod.twiss(el, REF, delta0=eps, h=1e-9)
    tm = oracle_mod.twiss(el, REF, delta0=-eps, h=1e-9)
    for c, d in (("x", "dx"), ("px", "dpx")):
        fd = (tp[c] - tm[c]) / (2 * eps)
        assert np.max(np.abs(fd - tw[d])) < 1e-6 * np.max(np.abs(tw[d]))
    assert np.max(np.abs(tw["dx"])) > 1.0  # the bends make it sizeable
    assert np.allclose(tw["dy"], 0.0, atol=1e-9)


def test_natural_chromaticity_thin_fodo(oracle_mod):
    # thin quadrupoles, kicks independent of delta, drifts advancing px/(1+delta):
    # the effective focusing is K/(1+delta), so xi = -(1/4 pi) sum beta_i K_i L_i
    el = I.cfg1_lattice(rf_on=False, sextupoles=False)
    f, L, mu, bmax, bmin = fodo_closed_form()
    xi = -100.0 * (bmax - bmin) / (4.0 * math.pi * f)
    cx, cy = oracle_mod.chromaticity(el, REF, eps=1e-7, h=1e-10, hd=1e-9)
    assert abs(cx - xi) < 1e-4 * abs(xi) and abs(cy - xi) < 1e-4 * abs(xi)
    # sextupoles at the quadrupoles do nothing at zero dispersion
    cx2, _ = oracle_mod.chromaticity(I.cfg1_lattice(rf_on=False), REF, eps=1e-7, h=1e-10, hd=1e-9)
    assert abs(cx2 - cx) < 1e-4 * abs(xi)


def coupled_bend_ring():
    cell = [I.multipole(knl=[0.0, 0.04]), I.multipole(knl=[0.05], hxl=0.05, length=2.0), I.drift(10.0),
            I.multipole(knl=[0.0, -0.04]), I.multipole(knl=[0.05], hxl=0.05, length=2.0), I.drift(10.0)]
    return I.line(cell * 20)


def test_coupled_optics_uncoupled_limit(oracle_mod):
    el = coupled_bend_ring()
    t = oracle_mod.twiss(el, REF, h=1e-6, hd=1e-6)
    c = oracle_mod.twiss_coupled(el, REF, h=1e-6, hd=1e-6)
    assert abs(c["q1"] - t["qx"]) < 1e-8 and abs(c["q2"] - t["qy"]) < 1e-8
    assert np.allclose(c["betx1"], t["betx"], rtol=1e-7) and np.allclose(c["bety2"], t["bety"], rtol=1e-7)
    assert np.allclose(c["mu1"], t["mux"], atol=1e-7) and np.allclose(c["mu2"], t["muy"], atol=1e-7)
    assert np.max(c["bety1"]) < 1e-12 and np.max(c["betx2"]) < 1e-12


@pytest.mark.parametrize("theta", [0.3, 1.2])
def test_coupled_optics_in_a_rotated_frame(oracle_mod, theta):
    # the same ring seen through a frame rotated by theta: the modes are the
    # uncoupled ones, mixed at the line start as cos^2 / sin^2 of theta
    el = coupled_bend_ring()
    t = oracle_mod.twiss(el, REF, h=1e-6, hd=1e-6)
    rot = I.line([I.srotation(theta)] + list(el) + [I.srotation(-theta)])
    c = oracle_mod.twiss_coupled(rot, REF, h=1e-6, hd=1e-6)
    assert abs(c["q1"] - t["qx"]) < 1e-8 and abs(c["q2"] - t["qy"]) < 1e-8
    cs, sn = math.cos(theta) ** 2, math.sin(theta) ** 2
    b0x, b0y = t["betx"][0], t["bety"][0]
    assert abs(c["betx1"][0] - cs * b0x) < 1e-7 * b0x and abs(c["bety1"][0] - sn * b0x) < 1e-7 * b0x
    assert abs(c["betx2"][0] - sn * b0y) < 1e-7 * b0y and abs(c["bety2"][0] - cs * b0y) < 1e-7 * b0y
    # inside the rotated frame the motion is uncoupled again
    assert np.allclose(c["betx1"][1:-1], t["betx"], rtol=1e-7)
    assert np.allclose(c["bety2"][1:-1], t["bety"], rtol=1e-7)
    assert np.max(c["bety1"][1:-1]) < 1e-9 * b0x


def test_open_line_optics_drift_closed_form(oracle_mod):
    b0, a0, d0, dp0 = 12.0, -1.5, 0.7, 0.02
    el = I.line([I.drift(3.0), I.marker(), I.drift(4.5)])
    t = oracle_mod.twiss_open(el, REF, [0, 0, 0, 0, b0, a0, 20.0, 0.5, d0, dp0, 0.0, 0.0], h=1e-9)
    g0 = (1 + a0 * a0) / b0
    for k, s in enumerate(t["s"]):
        assert abs(t["betx"][k] - (b0 - 2 * a0 * s + g0 * s * s)) < 1e-9 * b0
        assert abs(t["alfx"][k] - (a0 - g0 * s)) < 1e-9
        assert abs(t["dx"][k] - (d0 + dp0 * s)) < 1e-9 and abs(t["dpx"][k] - dp0) < 1e-12


def test_open_line_from_periodic_conditions_reproduces_the_ring(oracle_mod):
    el = coupled_bend_ring()
    t = oracle_mod.twiss(el, REF, h=1e-6, hd=1e-6)
    init = [t["x"][0], t["px"][0], t["y"][0], t["py"][0], t["betx"][0], t["alfx"][0],
            t["bety"][0], t["alfy"][0], t["dx"][0], t["dpx"][0], t["dy"][0], t["dpy"][0]]
    o = oracle_mod.twiss_open(el, REF, init, h=1e-6, hd=1e-6)
    for c in ("betx", "alfx", "mux", "bety", "alfy", "muy", "dx", "dpx"):
        assert np.max(np.abs(o[c] - t[c])) < 1e-9 * max(1.0, np.max(np.abs(t[c]))), c


# ------------------------------------------------------------ 6D normal form
def _symp_norm(v):
    # v^H S v / 2i summed over the three planes
    return sum(float(np.imag(np.conj(v[2 * p]) * v[2 * p + 1])) for p in range(3))


def test_6d_normal_form_reproduces_the_fodo_closed_forms(oracle_mod):
    """FODO ring with its RF cavity, no radiation: the transverse tunes and
    the synchrotron tune of the thin-lens closed forms, no damping, the
    closed orbit on the axis, and |v_x|^2 = beta_x of the transverse optics."""
    el = I.cfg1_lattice()
    nf = oracle_mod.normal_form_6d(el, I.PROTON_450GEV)
    assert np.all(np.abs(nf["co"]) < 1e-15)
    assert abs(nf["q"][0] - 0.99580450867910) < 1e-10     # Q = 24.9958045086791
    assert abs(nf["q"][1] - 0.99580450867910) < 1e-10
    assert abs(nf["q"][2] - 3.5084512757054226e-4) < 1e-10
    assert np.all(np.abs(nf["damping"]) < 1e-12)
    # the line starts at the RF cavity, next to the QF: the thin-lens closed
    # forms L_c (1 +- sin(mu/2)) / sin mu, 170.70136... m and 29.29864... m
    assert abs(abs(nf["v"][0][0]) ** 2 / 170.70136339712423 - 1) < 1e-9
    assert abs(abs(nf["v"][1][2]) ** 2 / 29.298643551925238 - 1) < 1e-9
    for k in range(3):
        assert abs(_symp_norm(nf["v"][k]) - 1) < 1e-12
        assert abs(nf["v"][k][2 * k].imag) == 0.0 and nf["v"][k][2 * k].real > 0
    # symplectic orthogonality of different modes: v_j^T S v_k = 0
    S = oracle_mod.S6
    for j in range(3):
        for k in range(3):
            if j != k:
                assert abs(nf["v"][j] @ S @ nf["v"][k]) < 1e-9


def test_6d_damping_partition_numbers_and_robinson_sum(oracle_mod):
    """Electron ring with the mean energy loss: the damping decrement of mode
    k per turn is J_k U0 / (2 E0); flat ring J_y = 1, separated-function
    thin bends J_x = 1 and J_z = 2, their sum 4 (Robinson); the decrements
    and the determinant of the one-turn map agree exactly
    (det J = prod |lambda|^2)."""
    el = I.cfg5_lattice(100, n_rf=4, apertures=False, sextupoles=False)
    nf = oracle_mod.normal_form_6d(el, EREF, radiation=1)
    u0 = I.CFG5_U0_OVER_E0[100]
    jk = nf["damping"] / (u0 / 2.0)
    assert abs(jk[1] - 1.0) < 2e-3
    assert abs(jk[0] - 1.0) < 2e-3 and abs(jk[2] - 2.0) < 2e-3
    assert abs(jk.sum() - 4.0) < 2e-3
    assert abs(2.0 * nf["damping"].sum() + math.log(np.linalg.det(nf["J"]))) < 1e-10
    # the closed orbit is a fixed point of the damped map
    u = oracle_mod.one_turn(el, EREF, nf["co"], 1, radiation=1)
    assert np.max(np.abs(u - nf["co"])) < 1e-14
    nf0 = oracle_mod.normal_form_6d(el, EREF, radiation=0)
    # without radiation the map is symplectic: no damping beyond the
    # central differences' truncation
    assert np.all(np.abs(nf0["damping"]) < 1e-7)


def test_matched_gaussian_is_invariant_under_the_map(oracle_mod):
    """The covariance sum_k eps_k (Re v_k Re v_k^T + Im v_k Im v_k^T) of the
    matched ensemble is carried into itself by the one-turn map, and the
    sample covariance of a generated ensemble agrees with it."""
    el = I.cfg1_lattice()
    nf = oracle_mod.normal_form_6d(el, I.PROTON_450GEV)
    eps = [3e-9, 1e-9, 2e-5]
    sig = np.zeros((6, 6))
    for k in range(3):
        a, b = nf["v"][k].real, nf["v"][k].imag
        sig += eps[k] * (np.outer(a, a) + np.outer(b, b))
    J = nf["J"]
    assert np.max(np.abs(J @ sig @ J.T - sig)) < 1e-8 * np.max(np.abs(sig))
    g = np.random.default_rng(3).normal(size=(200000, 6))
    c = oracle_mod.matched_gaussian(nf, I.PROTON_450GEV, eps, g)
    b0, _ = oracle_mod.reference(I.PROTON_450GEV)
    u = c.copy()
    # back to pzeta = ptau / beta0 for the comparison
    d = c[:, 5]
    u[:, 5] = (d * (2.0 + d)) / (1.0 / b0 + np.sqrt(1.0 / b0 ** 2 + d * (2.0 + d))) / b0
    cov = np.cov(u.T)
    for i in range(6):
        assert abs(cov[i, i] / sig[i, i] - 1) < 0.02, i
