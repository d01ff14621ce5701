"""Pins of the early-turn feature reference (oracle/features.py) against a
pure rotation and the linear thin FODO ring, where the tune has a closed form
and the actions are invariant."""
import math

import numpy as np

from paper_2310_00317_amd import inputs as I


def test_tune_estimator_pure_rotation():
    from oracle import features as F
    n = np.arange(F.WINDOW)
    for q in (0.9958045086791, 0.31, 0.0123, 0.5):
        u = np.cos(2 * math.pi * q * n + 0.3)
        pu = -np.sin(2 * math.pi * q * n + 0.3)
        est = F.tune_fft(u[None], pu[None])[0]
        d = min(abs(est - q), 1 - abs(est - q))
        assert d < 2e-5, (q, est)
    # the sign convention: rotation the other way gives 1 - q
    q = 0.2
    est = F.tune_fft(np.cos(2 * math.pi * q * n)[None], np.sin(2 * math.pi * q * n)[None])[0]
    assert abs(est - (1 - q)) < 2e-5


def test_features_on_linear_fodo(oracle_mod):
    from oracle import features as F
    el = I.cfg1_lattice(sextupoles=False, rf_on=False)
    k = 1 / I.CFG1_F
    tw = I.cell_twiss_at_qf_entry(k, -k, I.CFG1_HALF)
    emit = 1e-8
    c, r, th = I.polar_grid(4, 3, 6.0, tw, emit, delta=0.0)
    c = c[np.r_[1:4, 5:8, 9:12]]                       # skip the particles at the origin
    rec, p = F.record(el, I.PROTON_450GEV, c, nthreads=1)
    f = F.features(rec, tw, emit, I.CFG1_APERTURE)
    mu = math.acos(1 - I.CFG1_HALF ** 2 / (2 * I.CFG1_F ** 2))
    qfrac = (100 * mu / (2 * math.pi)) % 1.0
    amp = np.hypot(np.cos(th[np.r_[1:4, 5:8, 9:12]]), np.sin(th[np.r_[1:4, 5:8, 9:12]]))
    rr = r[np.r_[1:4, 5:8, 9:12]]
    assert np.allclose(f[:, 2], rr, rtol=1e-12)
    assert np.allclose(f[:, 0], rr * np.cos(th[np.r_[1:4, 5:8, 9:12]]), rtol=1e-12, atol=1e-12)
    for j in (4, 5, 6, 7):
        assert np.all(np.abs(f[:, j] - qfrac) < 2e-5), (j, f[:, j], qfrac)
    assert np.all(f[:, 8] < -6) and np.all(f[:, 9] < -6)     # no tune diffusion
    # invariant actions (up to the exact drift's tiny nonlinearity)
    assert np.all(np.abs(f[:, 10:14]) < 1e-6)
    assert np.all(np.abs(f[:, 15] - 1) < 1e-6)
    xmax = np.max(np.hypot(rec[:, 0], rec[:, 2]), axis=0)
    assert np.allclose(f[:, 14], xmax / I.CFG1_APERTURE)
    assert amp.shape == rr.shape


def test_features_flag_a_nonlinear_orbit(oracle_mod):
    """On the sextupole lattice a particle near the dynamic aperture shows
    tune diffusion and action drift orders of magnitude above a core one."""
    from oracle import features as F
    el = I.cfg1_lattice()
    k = 1 / I.CFG1_F
    tw = I.cell_twiss_at_qf_entry(k, -k, I.CFG1_HALF)
    c, r, th = I.polar_grid(2, 1, 16.0, tw, 1e-8, delta=2.7e-4)
    c[0] = I.polar_grid(2, 1, 2.0, tw, 1e-8, delta=2.7e-4)[0][1]
    rec, p = F.record(el, I.PROTON_450GEV, c, nthreads=1)
    f = F.features(rec, tw, 1e-8, I.CFG1_APERTURE)
    assert f[1, 8] > f[0, 8] + 1.0 or f[1, 12] > 10 * f[0, 12]
