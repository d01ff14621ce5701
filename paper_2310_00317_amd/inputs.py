"""Seeded synthetic inputs: lattices and particle ensembles.

This module only *describes* inputs.  It builds element-description records
(the beam line as an ordered sequence of element objects, paper section
"Lattice modelling and single particle tracking") and draws seeded initial
coordinates.  It holds none of the tracking arithmetic: no map, no derived
particle variable, no normal form.  Both the HIP path and the CPU oracle
consume what it returns, so it must stay free of anything either of them
computes.

The one piece of optics here is lattice *design*: thin-lens 2x2 cell matrices
used to pick quadrupole strengths for a target phase advance and to place a
grid in units of the beam size.  That is a closed-form recipe for choosing
inputs, not the method under test.

Layout of an element record (``ELEMENT_DTYPE``, 248 bytes, C-compatible with
``xtm_element_desc`` in ``include/xtm.h``):

    int32 type, int32 order, double length, double knl[11], double ksl[11],
    double hxl, double p[6]

``p`` meaning by type: RF (V [V], f [Hz], lag [deg]); XYShift (dx, dy [m]);
SRotation (angle [rad]); circle (r); ellipse (a, b); rect (xmin, xmax, ymin,
ymax).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# ---------------------------------------------------------------- constants
# CODATA 2018 values, stored as data so every consumer reads identical doubles.
CLIGHT = 299792458.0                 # m/s
PROTON_MASS_EV = 938.27208816e6      # eV
ELECTRON_MASS_EV = 0.51099895000e6   # eV
R_ELECTRON = 2.8179403262e-15        # classical electron radius [m]
HBAR_C_EVM = 197.3269804e-9          # hbar*c [eV m]

MAX_ORDER = 10

# element type codes (same numbering as include/xtm.h)
DRIFT = 1
DRIFT_EXPANDED = 2
MULTIPOLE = 3
RF = 4
XYSHIFT = 5
SROTATION = 6
AP_CIRCLE = 7
AP_ELLIPSE = 8
AP_RECT = 9
MARKER = 10
QUADRUPOLE = 11
SBEND = 12

TYPE_NAMES = {DRIFT: "drift", DRIFT_EXPANDED: "drift_expanded",
              MULTIPOLE: "multipole", RF: "rf", XYSHIFT: "xyshift",
              SROTATION: "srotation", AP_CIRCLE: "ap_circle",
              AP_ELLIPSE: "ap_ellipse", AP_RECT: "ap_rect", MARKER: "marker",
              QUADRUPOLE: "quadrupole", SBEND: "sbend"}

ELEMENT_DTYPE = np.dtype([
    ("type", "<i4"), ("order", "<i4"), ("length", "<f8"),
    ("knl", "<f8", (MAX_ORDER + 1,)), ("ksl", "<f8", (MAX_ORDER + 1,)),
    ("hxl", "<f8"), ("p", "<f8", (6,)),
], align=True)
assert ELEMENT_DTYPE.itemsize == 248

# recorded particle coordinate order of every (n, 6) array in this project
COORDS = ("x", "px", "y", "py", "zeta", "delta")


@dataclass(frozen=True)
class Reference:
    """Reference particle: rest mass [eV], charge [e], momentum p0c [eV]."""
    mass0_eV: float
    charge0: float
    p0c_eV: float

    def as_array(self) -> np.ndarray:
        return np.array([self.mass0_eV, self.charge0, self.p0c_eV], dtype="<f8")


PROTON_450GEV = Reference(PROTON_MASS_EV, 1.0, 450e9)
ELECTRON_45GEV6 = Reference(ELECTRON_MASS_EV, -1.0, 45.6e9)


# ------------------------------------------------------ element constructors
def _blank() -> np.ndarray:
    return np.zeros((), dtype=ELEMENT_DTYPE)


def drift(length: float, expanded: bool = False) -> np.ndarray:
    e = _blank()
    e["type"] = DRIFT_EXPANDED if expanded else DRIFT
    e["length"] = length
    return e


def multipole(knl=(), ksl=(), hxl: float = 0.0, length: float = 0.0,
              order: int | None = None) -> np.ndarray:
    """Thin multipole; ``knl[n]``/``ksl[n]`` integrated normal/skew strength of
    MAD index n [m^-n]; ``length`` is the radiation (and weak-focusing) length."""
    e = _blank()
    e["type"] = MULTIPOLE
    knl = list(knl)
    ksl = list(ksl)
    if order is None:
        order = max(len(knl), len(ksl), 1) - 1
    assert 0 <= order <= MAX_ORDER
    e["order"] = order
    e["knl"][: len(knl)] = knl
    e["ksl"][: len(ksl)] = ksl
    e["hxl"] = hxl
    e["length"] = length
    return e


def rf(voltage: float, frequency: float, lag_deg: float) -> np.ndarray:
    e = _blank()
    e["type"] = RF
    e["p"][:3] = (voltage, frequency, lag_deg)
    return e


def xyshift(dx: float, dy: float) -> np.ndarray:
    e = _blank()
    e["type"] = XYSHIFT
    e["p"][:2] = (dx, dy)
    return e


def srotation(angle_rad: float) -> np.ndarray:
    e = _blank()
    e["type"] = SROTATION
    e["p"][0] = angle_rad
    return e


def ap_circle(r: float) -> np.ndarray:
    e = _blank()
    e["type"] = AP_CIRCLE
    e["p"][0] = r
    return e


def ap_ellipse(a: float, b: float) -> np.ndarray:
    e = _blank()
    e["type"] = AP_ELLIPSE
    e["p"][:2] = (a, b)
    return e


def ap_rect(xmin: float, xmax: float, ymin: float, ymax: float) -> np.ndarray:
    e = _blank()
    e["type"] = AP_RECT
    e["p"][:4] = (xmin, xmax, ymin, ymax)
    return e


def marker() -> np.ndarray:
    e = _blank()
    e["type"] = MARKER
    return e


def quadrupole(length: float, k1: float, k1s: float = 0.0, slices: int = 4) -> np.ndarray:
    """Thick quadrupole of length [m] and gradient k1, k1s [m^-2], tracked as
    `slices` drift-kick-drift slices."""
    e = _blank()
    e["type"] = QUADRUPOLE
    e["length"] = length
    e["p"][0] = k1
    e["p"][1] = k1s
    e["p"][2] = slices
    return e


def sbend(length: float, angle: float, k1: float = 0.0, slices: int = 4) -> np.ndarray:
    """Thick sector bend of length [m], bending angle [rad] and gradient k1
    [m^-2], tracked as `slices` drift-kick-drift slices."""
    e = _blank()
    e["type"] = SBEND
    e["length"] = length
    e["p"][0] = angle
    e["p"][1] = k1
    e["p"][2] = slices
    return e


def thick_ring(n_cells: int = 16, k1: float = 0.06) -> np.ndarray:
    """Ring of thick elements: n_cells x [QF (1 m, 4 slices), sector bend (6 m,
    pi/n_cells, 6 slices), circular aperture 30 mm, drift 2 m, QD (1 m, with a
    small skew gradient), bend, elliptic aperture 30 x 20 mm, drift 2 m, thin
    sextupole]."""
    ang = 2.0 * math.pi / (2 * n_cells)
    cell = [quadrupole(1.0, k1, slices=4), sbend(6.0, ang, slices=6), ap_circle(0.03),
            drift(2.0), quadrupole(1.0, -k1, k1s=1e-4, slices=4), sbend(6.0, ang, slices=6),
            ap_ellipse(0.03, 0.02), drift(2.0), multipole(knl=[0.0, 0.0, 0.2])]
    return line(cell * n_cells)


def line(elements) -> np.ndarray:
    """Stack element records into a contiguous C-compatible array."""
    out = np.zeros(len(elements), dtype=ELEMENT_DTYPE)
    for i, e in enumerate(elements):
        out[i] = e
    return out


# ------------------------------------------------------------ lattice design
def _thin_cell_matrix(k_f: float, k_d: float, half: float) -> tuple[np.ndarray, np.ndarray]:
    """2x2 linear matrices (x, y) of [QF(k_f) . drift . QD(k_d) . drift] for thin
    kicks dpx = -k x (x plane) and dpy = +k y (y plane); used only to design inputs."""
    def kick(k):
        return np.array([[1.0, 0.0], [-k, 1.0]])

    def dr(L):
        return np.array([[1.0, L], [0.0, 1.0]])

    mx = dr(half) @ kick(k_d) @ dr(half) @ kick(k_f)
    my = dr(half) @ kick(-k_d) @ dr(half) @ kick(-k_f)
    return mx, my


def _twiss_from_matrix(m: np.ndarray) -> tuple[float, float, float]:
    cmu = 0.5 * (m[0, 0] + m[1, 1])
    smu = math.copysign(math.sqrt(1.0 - cmu * cmu), m[0, 1])
    beta = m[0, 1] / smu
    alpha = (m[0, 0] - m[1, 1]) / (2.0 * smu)
    return beta, alpha, math.atan2(smu, cmu) % (2 * math.pi)


def design_fodo(mu_x: float, mu_y: float, half: float) -> tuple[float, float]:
    """Quadrupole strengths (k_f > 0, k_d < 0) giving cell phase advances
    mu_x, mu_y [rad] for a thin FODO cell of two drifts of length ``half``."""
    k = np.array([1.0 / (half * math.sqrt(2.0)), -1.0 / (half * math.sqrt(2.0))])
    for _ in range(60):
        def resid(kk):
            mx, my = _thin_cell_matrix(kk[0], kk[1], half)
            return np.array([0.5 * np.trace(mx) - math.cos(mu_x),
                             0.5 * np.trace(my) - math.cos(mu_y)])
        r = resid(k)
        if np.max(np.abs(r)) < 1e-15:
            break
        jac = np.zeros((2, 2))
        for j in range(2):
            dk = np.zeros(2)
            dk[j] = 1e-9
            jac[:, j] = (resid(k + dk) - resid(k - dk)) / 2e-9
        k = k - np.linalg.solve(jac, r)
    return float(k[0]), float(k[1])


def cell_twiss_at_qf_entry(k_f: float, k_d: float, half: float):
    """(beta_x, alpha_x, beta_y, alpha_y) just upstream of the thin QF of a
    periodic thin FODO cell; lattice-design helper for placing grids in sigma."""
    mx, my = _thin_cell_matrix(k_f, k_d, half)
    bx, ax, _ = _twiss_from_matrix(mx)
    by, ay, _ = _twiss_from_matrix(my)
    return bx, ax, by, ay


# ----------------------------------------------------------------- configs
CFG1_F = 35.36
CFG1_HALF = 50.0
CFG1_K2L = 0.05
CFG1_APERTURE = 0.040


def cfg1_lattice(sextupoles: bool = True, rf_on: bool = True,
                 apertures: bool = True, expanded_drift: bool = False,
                 n_cells: int = 100) -> np.ndarray:
    """Plain thin FODO ring: element 0 is the RF cavity (6 MV, 400 MHz, lag 0),
    then ``n_cells`` x [QF, SF, AP, D50, QD, SD, AP, D50] (801 elements).
    Elements that are switched off stay in place as markers so element
    indices do not move."""
    k = 1.0 / CFG1_F
    els = [rf(6e6, 400e6, 0.0) if rf_on else marker()]
    for _ in range(n_cells):
        els += [
            multipole(knl=[0.0, k]),
            multipole(knl=[0.0, 0.0, CFG1_K2L]) if sextupoles else marker(),
            ap_circle(CFG1_APERTURE) if apertures else marker(),
            drift(CFG1_HALF, expanded_drift),
            multipole(knl=[0.0, -k]),
            multipole(knl=[0.0, 0.0, -CFG1_K2L]) if sextupoles else marker(),
            ap_circle(CFG1_APERTURE) if apertures else marker(),
            drift(CFG1_HALF, expanded_drift),
        ]
    return line(els)


CFG1_SIGMAS = np.array([1.3e-3, 1e-5, 1.3e-3, 1e-5, 0.1, 1e-4])


def gaussian_particles(n: int, seed: int, sigmas=CFG1_SIGMAS) -> np.ndarray:
    """(n, 6) independent Gaussian coordinates (x, px, y, py, zeta, delta).
    Row i depends only on (seed, i) for i < n, so a larger draw starts with
    the smaller one."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, 6)) * np.asarray(sigmas)[None, :]


def cfg1_particles(n: int = 1000, seed: int = 20231001) -> np.ndarray:
    return gaussian_particles(n, seed)


def cfg1m_lattice(seed: int = 7, sigma_d: float = 1e-4, sigma_t: float = 1e-4) -> np.ndarray:
    """cfg1 with every quadrupole wrapped in shift and rotation pairs:
    Shift(d) Rot(t) Q Rot(-t) Shift(-d), random d and t (seeded)."""
    base = cfg1_lattice()
    rng = np.random.default_rng(seed)
    els = []
    for e in base:
        if e["type"] == MULTIPOLE and e["order"] == 1:
            dx, dy = rng.normal(0.0, sigma_d, 2)
            th = rng.normal(0.0, sigma_t)
            els += [xyshift(dx, dy), srotation(th), e.copy(), srotation(-th), xyshift(-dx, -dy)]
        else:
            els.append(e.copy())
    return line(els)


# --- field-error model: b_n, a_n ~ N(0, (1e-4 * 10^-(n-2))^2) for n = 2..10,
# relative to the main field at r0, converted to integrated strengths.
ERR_R0 = 0.017


def add_field_errors(el: np.ndarray, main_order: int, rng: np.random.Generator,
                     rel: float = 1e-4, r0: float = ERR_R0) -> np.ndarray:
    """Return a copy of multipole ``el`` (main order m) raised to order 10 with
    random relative errors: dknl_n = K_m b_n n!/m! r0^(m-n), same for ksl with a_n."""
    e = el.copy()
    m = main_order
    km = float(e["knl"][m])
    for n in range(2, MAX_ORDER + 1):
        s = rel * 10.0 ** (-(n - 2))
        bn, an = rng.normal(0.0, s, 2)
        scale = km * math.factorial(n) / math.factorial(m) * r0 ** (m - n)
        e["knl"][n] += scale * bn
        e["ksl"][n] += scale * an
    e["order"] = MAX_ORDER
    return e


def errored_cfg1_lattice(seed: int) -> np.ndarray:
    """cfg1 with the error model on all 200 quadrupoles and 200 sextupoles."""
    rng = np.random.default_rng(seed)
    out = cfg1_lattice().copy()
    for i in range(len(out)):
        e = out[i]
        if e["type"] == MULTIPOLE:
            m = 1 if abs(e["knl"][1]) > 0 else 2
            out[i] = add_field_errors(e, m, rng)
    return out


# cfg2: 2000 cells x [AP, QF, D, MF, D, AP, QD, D, MD, D], D = 25 m, exactly
# 20,000 elements; in cells 0, 250, ..., 1750 the MF slot holds an RF cavity.
CFG2_CELLS = 2000
CFG2_D = 25.0
CFG2_QFRAC = (0.31, 0.32)
CFG2_K2L = 0.12            # main sextupole strength (+ at MF, - at MD), m^-2
CFG2_EMIT = 1e-8           # geometric emittance defining sigma [m]
CFG2_DELTA = 2.7e-4


def cfg2_quads(n_cells: int = CFG2_CELLS, qfrac=CFG2_QFRAC) -> tuple[float, float]:
    n_int = n_cells // 4          # ~90 deg per cell
    mux = 2 * math.pi * (n_int + qfrac[0]) / n_cells
    muy = 2 * math.pi * (n_int + qfrac[1]) / n_cells
    return design_fodo(mux, muy, 2 * CFG2_D)


def cfg2_lattice(seed: int = 2002, k2l: float = CFG2_K2L, n_cells: int = CFG2_CELLS,
                 errors: bool = True, rf_cells: int = 8) -> np.ndarray:
    kf, kd = cfg2_quads(n_cells)
    rng = np.random.default_rng(seed)
    rf_every = n_cells // rf_cells
    els = []
    for c in range(n_cells):
        qf = multipole(knl=[0.0, kf])
        qd = multipole(knl=[0.0, kd])
        mf = multipole(knl=[0.0, 0.0, k2l])
        md = multipole(knl=[0.0, 0.0, -k2l])
        if errors:
            qf = add_field_errors(qf, 1, rng)
            qd = add_field_errors(qd, 1, rng)
            mf = add_field_errors(mf, 2, rng)
            md = add_field_errors(md, 2, rng)
        slot = rf(0.75e6, 400e6, 0.0) if (c % rf_every == 0 and c // rf_every < rf_cells) else mf
        els += [ap_circle(CFG1_APERTURE), qf, drift(CFG2_D), slot, drift(CFG2_D),
                ap_circle(CFG1_APERTURE), qd, drift(CFG2_D), md, drift(CFG2_D)]
    return line(els)


def polar_grid(n_r: int = 2000, n_theta: int = 50, r_max_sigma: float = 10.0,
               twiss=(1.0, 0.0, 1.0, 0.0), emit: float = CFG2_EMIT,
               delta: float = CFG2_DELTA) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Dynamic-aperture grid: r_i = r_max i/(n_r-1) [sigma], theta_j = (j+1/2)(pi/2)/n_theta.
    Returns (coords (n_theta*n_r, 6), r_sigma, theta); particle index = j*n_r + i
    (ray-major), so neighbouring particles have neighbouring amplitudes.
    Normalised momenta are zero: px = -alpha x / beta."""
    bx, ax, by, ay = twiss
    r = r_max_sigma * np.arange(n_r) / (n_r - 1)
    th = (np.arange(n_theta) + 0.5) * (0.5 * math.pi) / n_theta
    rr = np.tile(r, n_theta)
    tt = np.repeat(th, n_r)
    sx = math.sqrt(bx * emit)
    sy = math.sqrt(by * emit)
    c = np.zeros((n_r * n_theta, 6))
    c[:, 0] = rr * np.cos(tt) * sx
    c[:, 2] = rr * np.sin(tt) * sy
    c[:, 1] = -ax * c[:, 0] / bx
    c[:, 3] = -ay * c[:, 2] / by
    c[:, 5] = delta
    return c, rr, tt


def random_amplitudes(n: int, r_max_sigma: float, twiss, seed: int, emit: float = CFG2_EMIT,
                      delta: float = CFG2_DELTA) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Training set of the loss predictor: r ~ U(0, r_max) [sigma],
    theta ~ U(0, pi/2), zero normalised momenta, zeta = 0, fixed delta.
    Returns (coords (n, 6), r_sigma, theta)."""
    rng = np.random.default_rng(seed)
    r = rng.random(n) * r_max_sigma
    th = rng.random(n) * 0.5 * math.pi
    bx, ax, by, ay = twiss
    c = np.zeros((n, 6))
    c[:, 0] = r * np.cos(th) * math.sqrt(bx * emit)
    c[:, 2] = r * np.sin(th) * math.sqrt(by * emit)
    c[:, 1] = -ax * c[:, 0] / bx
    c[:, 3] = -ay * c[:, 2] / by
    c[:, 5] = delta
    return c, r, th


def cfg1_twiss():
    """(beta_x, alpha_x, beta_y, alpha_y) at element 0 of cfg1 (the RF is thin
    and longitudinal, so this is the QF entry of the periodic cell)."""
    k = 1.0 / CFG1_F
    return cell_twiss_at_qf_entry(k, -k, CFG1_HALF)


def cfg2_grid(n_r: int = 2000, n_theta: int = 50, r_max_sigma: float = 10.0):
    kf, kd = cfg2_quads()
    tw = cell_twiss_at_qf_entry(kf, kd, 2 * CFG2_D)
    return polar_grid(n_r, n_theta, r_max_sigma, tw)


def cfg1_grid(n_r: int = 2000, n_theta: int = 50, r_max_sigma: float = 10.0):
    k = 1.0 / CFG1_F
    tw = cell_twiss_at_qf_entry(k, -k, CFG1_HALF)
    return polar_grid(n_r, n_theta, r_max_sigma, tw)


# cfg3: 64 errored cfg1 variants, N_v = 2000 + floor(U * 48001)
def cfg3_counts(n_variants: int = 64, seed: int = 3003) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (2000 + np.floor(rng.random(n_variants) * 48001)).astype(np.int64)


def cfg3_variant(v: int, n: int, lattice_seed_base: int = 30000,
                 particle_seed_base: int = 31000):
    return errored_cfg1_lattice(lattice_seed_base + v), gaussian_particles(n, particle_seed_base + v)


# cfg5: electron ring for synchrotron radiation.  n_cells x [QF, SF, AP, D/2,
# B, D/2, QD, SD, AP, D/2, B, D/2] with thin bends B (hxl = knl0 = theta over
# the radiation length Lr) and n_rf RF cavities placed before the QF of evenly
# spaced cells.  Lr is fixed so that the design energy loss per turn is
# about u0_over_e0 of the beam energy (values below were chosen for
# u0_over_e0 = 1e-3 with 1666 cells and 1e-2 with 100 cells); the RF voltage is
# 3 x U0, phased for electrons (charge -1) at lag = -asin(U0/V).
CFG5_CELLS = 1666
CFG5_LR = {1666: 15.817206401282936, 100: 26.351465864537374}
CFG5_U0_OVER_E0 = {1666: 1e-3, 100: 1e-2}


def cfg5_lattice(n_cells: int = CFG5_CELLS, n_rf: int = 8, rf_factor: float = 3.0,
                 sextupoles: bool = True, apertures: bool = True) -> np.ndarray:
    ref = ELECTRON_45GEV6
    e0 = math.sqrt(ref.p0c_eV ** 2 + ref.mass0_eV ** 2)
    u0 = CFG5_U0_OVER_E0[n_cells] * e0
    v_tot = rf_factor * u0
    lag = -math.degrees(math.asin(u0 / v_tot))
    theta = 2 * math.pi / (2 * n_cells)
    lr = CFG5_LR[n_cells]
    k = 1.0 / CFG1_F
    bend = multipole(knl=[theta], hxl=theta, length=lr)
    rf_cells = set(int(j * n_cells / n_rf) for j in range(n_rf))
    els = []
    for c in range(n_cells):
        if c in rf_cells:
            els.append(rf(v_tot / n_rf, 400e6, lag))
        els += [
            multipole(knl=[0.0, k]),
            multipole(knl=[0.0, 0.0, CFG1_K2L]) if sextupoles else marker(),
            ap_circle(CFG1_APERTURE) if apertures else marker(),
            drift(CFG1_HALF / 2), bend.copy(), drift(CFG1_HALF / 2),
            multipole(knl=[0.0, -k]),
            multipole(knl=[0.0, 0.0, -CFG1_K2L]) if sextupoles else marker(),
            ap_circle(CFG1_APERTURE) if apertures else marker(),
            drift(CFG1_HALF / 2), bend.copy(), drift(CFG1_HALF / 2),
        ]
    return line(els)


CFG5_SIGMAS = np.array([1e-4, 1e-6, 1e-5, 1e-7, 3e-3, 4e-4])


def cfg5_particles(n: int = 1_000_000, seed: int = 50505) -> np.ndarray:
    """6D Gaussian electrons with roughly equilibrium-sized sigmas."""
    return gaussian_particles(n, seed, CFG5_SIGMAS)


# Mode emittances [m] of the matched cfg5 ensemble (horizontal, vertical,
# longitudinal in canonical zeta-pzeta): the horizontal and vertical ones
# give sigma_x ~ 1e-4 m and sigma_y ~ 1e-5 m at the line start, the
# longitudinal one an energy spread near the ring's equilibrium 4.3e-4.
CFG5_EMITTANCES = (6.0e-11, 3.4e-12, 1.2e-6)


def standard_normals(n: int, seed: int = 50506) -> np.ndarray:
    """(n, 6) independent standard normal deviates (seeded), the random input
    of a matched ensemble."""
    return np.random.default_rng(seed).standard_normal((n, 6))
