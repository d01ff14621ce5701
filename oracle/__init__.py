"""CPU FP64 oracle for the thin-lattice tracking path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing in the product package
imports it, and it imports nothing from the product package.

``oracle.c`` holds the element maps and the turn loop (plain C, FP64,
``-ffp-contract=off``).  This module adds ctypes marshalling and the
host-side analysis built on the one-turn map: the central-difference
Jacobian and the uncoupled linear normal form (paper section "Twiss
module", steps 2 and 3).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["oracle.c"]
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-march=x86-64-v3",
          "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (it is the checker, never the product path)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    if not force and os.path.exists(LIB):
        lib_t = os.path.getmtime(LIB)
        if all(os.path.getmtime(s) <= lib_t for s in srcs):
            return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, *srcs, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(LIB)
        L.oracle_track.restype = ctypes.c_int64
        L.oracle_track_backward.restype = ctypes.c_int64
        L.oracle_init.restype = ctypes.c_int
        L.oracle_track_canonical.restype = ctypes.c_int
        L.oracle_track_rad.restype = ctypes.c_int64
        L.oracle_uniform.restype = ctypes.c_double
        L.oracle_uniform.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        for fn in ("oracle_sin", "oracle_cos", "oracle_log"):
            getattr(L, fn).restype = ctypes.c_double
            getattr(L, fn).argtypes = [ctypes.c_double]
        L.oracle_gauss_at.restype = ctypes.c_double
        L.oracle_gauss_at.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32]
        _lib = L
    return _lib


class _Parts(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("x", "px", "y", "py", "zeta", "delta", "ptau", "rpp", "rvv",
                 "state", "at_element", "at_turn", "pid")] + [("n", ctypes.c_int64)]


FLOAT_FIELDS = ("x", "px", "y", "py", "zeta", "delta", "ptau", "rpp", "rvv")
INT_FIELDS = ("state", "at_element", "at_turn")


class Particles:
    """Structure-of-arrays FP64 particle set held in numpy arrays."""

    def __init__(self, n: int):
        self.n = int(n)
        for f in FLOAT_FIELDS:
            setattr(self, f, np.zeros(self.n, dtype=np.float64))
        for f in INT_FIELDS:
            setattr(self, f, np.zeros(self.n, dtype=np.int32))
        self.particle_id = np.zeros(self.n, dtype=np.int64)
        self.turn = 0

    def _struct(self) -> _Parts:
        s = _Parts()
        for f in FLOAT_FIELDS + INT_FIELDS:
            setattr(s, f, getattr(self, f).ctypes.data)
        s.pid = self.particle_id.ctypes.data
        s.n = self.n
        return s

    def copy(self) -> "Particles":
        p = Particles(self.n)
        for f in FLOAT_FIELDS + INT_FIELDS + ("particle_id",):
            getattr(p, f)[:] = getattr(self, f)
        p.turn = self.turn
        return p

    def coords(self) -> np.ndarray:
        return np.stack([self.x, self.px, self.y, self.py, self.zeta, self.delta], axis=1)

    def subset(self, idx) -> "Particles":
        idx = np.asarray(idx)
        p = Particles(len(idx))
        for f in FLOAT_FIELDS + INT_FIELDS + ("particle_id",):
            getattr(p, f)[:] = getattr(self, f)[idx]
        p.turn = self.turn
        return p


def _ref3(ref) -> np.ndarray:
    if hasattr(ref, "as_array"):
        return np.ascontiguousarray(ref.as_array(), dtype=np.float64)
    return np.ascontiguousarray(np.asarray(ref, dtype=np.float64))


THICK_QUAD, THICK_SBEND = 11, 12


def expand_thick(elements) -> np.ndarray:
    """Thick quadrupoles (length L, p = k1, k1s, N) and sector bends (length
    L, p = angle, k1, N) as N drift-kick-drift slices with the kicks at the
    slice midpoints (a second-order symplectic splitting of the thick map,
    paper section on the tracking engine): with d = L/N, a drift d/2, then N
    times [kick, drift d], the last drift d/2.  Quadrupole kick: thin
    multipole of order 1 with knl1 = k1 d, ksl1 = k1s d.  Bend kick: thin
    multipole with knl0 = hxl = angle/N over the length d (its curvature
    terms give the weak focusing and the path-length change) and knl1 = k1 d.
    Thin elements pass unchanged."""
    el = np.ascontiguousarray(elements)
    if not np.isin(el["type"], (THICK_QUAD, THICK_SBEND)).any():
        return el
    out = []
    for e in el:
        t = int(e["type"])
        if t not in (THICK_QUAD, THICK_SBEND):
            out.append(e.copy())
            continue
        L, Nf = float(e["length"]), float(e["p"][2])
        if not (L > 0.0 and 1.0 <= Nf <= 10000.0 and Nf == math.floor(Nf)):
            raise ValueError("thick element needs length > 0 and an integer slice count")
        N = int(Nf)
        d = L / float(N)
        half = 0.5 * d
        kick = np.zeros((), dtype=el.dtype)
        kick["type"] = 3
        kick["order"] = 1
        if t == THICK_QUAD:
            kick["knl"][1] = float(e["p"][0]) * d
            kick["ksl"][1] = float(e["p"][1]) * d
        else:
            a = float(e["p"][0]) / float(N)
            kick["knl"][0] = a
            kick["hxl"] = a
            kick["length"] = d
            kick["knl"][1] = float(e["p"][1]) * d
        for j in range(N + 1):
            dr = np.zeros((), dtype=el.dtype)
            dr["type"] = 1
            dr["length"] = half if j in (0, N) else d
            out.append(dr)
            if j < N:
                out.append(kick.copy())
    res = np.zeros(len(out), dtype=el.dtype)
    for i, e in enumerate(out):
        res[i] = e
    return res


def _els(elements) -> np.ndarray:
    a = np.ascontiguousarray(elements)
    assert a.dtype.itemsize == 248, "element records must use the 248-byte layout"
    return expand_thick(a)


def init(coords6, ref, first_id: int = 0) -> Particles:
    """Particles from (n, 6) coordinates (x, px, y, py, zeta, delta)."""
    c = np.ascontiguousarray(coords6, dtype=np.float64).reshape(-1, 6)
    p = Particles(c.shape[0])
    s = p._struct()
    r = _ref3(ref)
    lib().oracle_init(c.ctypes.data_as(ctypes.c_void_p), ctypes.c_int64(p.n),
                      ctypes.c_int64(first_id), r.ctypes.data_as(ctypes.c_void_p),
                      ctypes.byref(s))
    return p


def track(elements, ref, parts: Particles, n_turns: int, nthreads: int = 0,
          radiation: int = 0, seed: int = 0) -> int:
    """Forward tracking in place from turn ``parts.turn``; returns passes.
    radiation: 0 off, 1 mean energy loss, 2 mean + Gaussian quantum excitation
    (Philox stream keyed by ``seed``, counter (particle id, turn, element)),
    3 photon by photon (the spectrum table of ``oracle.photons``)."""
    el = _els(elements)
    r = _ref3(ref)
    if radiation == 3:
        _set_photon_table()
    s = parts._struct()
    passes = lib().oracle_track_rad(el.ctypes.data_as(ctypes.c_void_p), ctypes.c_int32(len(el)),
                                    r.ctypes.data_as(ctypes.c_void_p), ctypes.byref(s),
                                    ctypes.c_int32(parts.turn), ctypes.c_int32(n_turns),
                                    ctypes.c_int32(nthreads), ctypes.c_int32(radiation),
                                    ctypes.c_uint64(seed))
    if passes < 0:
        raise ValueError("oracle_track rejected its input (code %d)" % passes)
    parts.turn += n_turns
    return int(passes)


_PHOTON_TABLE_SET = False


def _set_photon_table():
    global _PHOTON_TABLE_SET
    if not _PHOTON_TABLE_SET:
        from . import photons
        g = np.ascontiguousarray(photons.table())
        if lib().oracle_set_photon_table(g.ctypes.data_as(ctypes.c_void_p),
                                         ctypes.c_int32(len(g))) != 0:
            raise RuntimeError("oracle_set_photon_table failed")
        _PHOTON_TABLE_SET = True


def track_backward(elements, ref, parts: Particles, n_turns: int, nthreads: int = 0) -> int:
    el = _els(elements)
    r = _ref3(ref)
    s = parts._struct()
    passes = lib().oracle_track_backward(el.ctypes.data_as(ctypes.c_void_p),
                                         ctypes.c_int32(len(el)),
                                         r.ctypes.data_as(ctypes.c_void_p), ctypes.byref(s),
                                         ctypes.c_int32(parts.turn), ctypes.c_int32(n_turns),
                                         ctypes.c_int32(nthreads))
    if passes < 0:
        raise ValueError("oracle_track_backward rejected its input (code %d)" % passes)
    parts.turn -= n_turns
    return int(passes)


def refine_losses(elements, ref, parts: Particles, n_vertices: int = 64, ds: float = 0.01,
                  n_bisect: int = 30, with_tests: bool = False):
    """Loss-location refinement of the particles lost on an aperture: (s, x, y)
    of the first exit from the polygon-interpolated aperture between the
    previous aperture and the one that caught each particle, NaN elsewhere
    (the reading is stated at oracle_refine_losses in oracle.c)."""
    el = _els(elements)
    r = _ref3(ref)
    st = parts._struct()
    out = [np.zeros(parts.n, dtype=np.float64) for _ in range(3)]
    tests = np.zeros(parts.n, dtype=np.int32)
    f = lib().oracle_refine_losses
    f.restype = ctypes.c_int
    rc = f(el.ctypes.data_as(ctypes.c_void_p), ctypes.c_int32(len(el)),
           r.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st), ctypes.c_int32(n_vertices),
           ctypes.c_double(ds), ctypes.c_int32(n_bisect),
           *[a.ctypes.data_as(ctypes.c_void_p) for a in out + [tests]])
    if rc != 0:
        raise ValueError("oracle_refine_losses rejected its input (code %d)" % rc)
    return tuple(out) + ((tests,) if with_tests else ())


def track_record(elements, ref, coords6) -> np.ndarray:
    """One turn from the line start with the coordinates recorded at every
    element entry and after the last element: array (n_el + 1, n, 6) of
    (x, px, y, py, zeta, delta); apertures are not checked."""
    el = _els(elements)
    r = _ref3(ref)
    c = np.ascontiguousarray(coords6, dtype=np.float64).reshape(-1, 6)
    out = np.zeros((len(el) + 1, c.shape[0], 6))
    f = lib().oracle_track_record
    f.restype = ctypes.c_int
    rc = f(el.ctypes.data_as(ctypes.c_void_p), ctypes.c_int32(len(el)),
           r.ctypes.data_as(ctypes.c_void_p), c.ctypes.data_as(ctypes.c_void_p),
           ctypes.c_int64(c.shape[0]), out.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise ValueError("oracle_track_record rejected its input (code %d)" % rc)
    return out


def twiss(elements, ref, delta0: float = 0.0, h: float = 1e-8, hd: float = 1e-7,
          max_iter: int = 30, tol: float = 1e-15, guess=None) -> dict:
    """Optics by tracking (paper section "Twiss module"), transverse and
    uncoupled, at fixed momentum deviation delta0 (RF and longitudinal motion
    frozen: zeta starts at 0 and is not part of the orbit):
      1. closed orbit u* = T(u*) of the one-turn map on (x, px, y, py) by
         Newton's method, u <- u + (I - J)^-1 (T(u) - u), until the largest
         component of T(u) - u is below tol (or stops decreasing);
      2. Jacobian J of the one-turn map by central differences of particles
         displaced by +-h along each coordinate, and the momentum column m by
         +-hd in delta;
      3. the same differences at every element give the map M_e from the line
         start to element e and its momentum column m_e;
      4. per plane, from the one-turn 2x2 block [[a, b], [c, d]]:
         cos mu = (a + d)/2, sin mu = sign(b) sqrt(1 - cos^2 mu),
         beta0 = b / sin mu, alpha0 = (a - d)/(2 sin mu); at element e with
         block [[p, q], [r, t]] of M_e: beta = ((p beta0 - q alpha0)^2 + q^2)/beta0,
         alpha = -((p beta0 - q alpha0)(r beta0 - t alpha0) + q t)/beta0,
         phase = atan2(q, p beta0 - q alpha0), unwrapped to increase;
      5. dispersion eta_0 = (I - J)^-1 m, eta_e = M_e eta_0 + m_e.
    Returns the per-element table (n_el + 1 rows) and the tunes."""
    el = _els(elements)
    n_el = len(el)
    u = np.zeros(4) if guess is None else np.array(guess, dtype=np.float64)
    I4 = np.eye(4)

    def probe(u, with_delta):
        rows = [np.r_[u, 0.0, delta0]]
        for k in range(4):
            for sgn in (1.0, -1.0):
                v = np.r_[u, 0.0, delta0]
                v[k] += sgn * h
                rows.append(v)
        if with_delta:
            for sgn in (1.0, -1.0):
                rows.append(np.r_[u, 0.0, delta0 + sgn * hd])
        return np.array(rows)

    it, res, best = 0, np.inf, np.inf
    while True:
        out = track_record(el, ref, probe(u, False))
        end = out[n_el]
        J = np.empty((4, 4))
        for k in range(4):
            J[:, k] = (end[1 + 2 * k, :4] - end[2 + 2 * k, :4]) / (2.0 * h)
        F = end[0, :4] - u
        res = float(np.max(np.abs(F)))
        if res <= tol or it >= max_iter or res >= best:
            break
        best = res
        u = u + np.linalg.solve(I4 - J, F)
        it += 1
    out = track_record(el, ref, probe(u, True))
    M = np.empty((n_el + 1, 4, 4))
    for k in range(4):
        M[:, :, k] = (out[:, 1 + 2 * k, :4] - out[:, 2 + 2 * k, :4]) / (2.0 * h)
    md = (out[:, 9, :4] - out[:, 10, :4]) / (2.0 * hd)
    J = M[n_el]
    eta0 = np.linalg.solve(I4 - J, md[n_el])
    eta = np.einsum("eij,j->ei", M, eta0) + md
    tab = {"s": np.concatenate([[0.0], np.cumsum(np.where(np.isin(el["type"], (1, 2)),
                                                          el["length"], 0.0))]),
           "x": out[:, 0, 0], "px": out[:, 0, 1], "y": out[:, 0, 2], "py": out[:, 0, 3],
           "dx": eta[:, 0], "dpx": eta[:, 1], "dy": eta[:, 2], "dpy": eta[:, 3]}
    q = {}
    for name, o in (("x", 0), ("y", 2)):
        a, b, c, d = J[o, o], J[o, o + 1], J[o + 1, o], J[o + 1, o + 1]
        cmu = 0.5 * (a + d)
        smu = math.copysign(math.sqrt(max(0.0, 1.0 - cmu * cmu)), b)
        b0 = b / smu
        a0 = (a - d) / (2.0 * smu)
        p_, q_, r_, t_ = M[:, o, o], M[:, o, o + 1], M[:, o + 1, o], M[:, o + 1, o + 1]
        bb = p_ * b0 - q_ * a0
        tab["bet" + name] = (bb * bb + q_ * q_) / b0
        tab["alf" + name] = -(bb * (r_ * b0 - t_ * a0) + q_ * t_) / b0
        th = np.arctan2(q_, bb)
        mu = np.zeros(n_el + 1)
        for e in range(1, n_el + 1):
            mu[e] = mu[e - 1] + (th[e] - th[e - 1]) % (2.0 * math.pi)
        tab["mu" + name] = mu
        q["q" + name] = mu[n_el] / (2.0 * math.pi)
    tab.update(q)
    tab["iterations"] = it
    tab["residual"] = res
    return tab


def twiss_open(elements, ref, init, delta0: float = 0.0, h: float = 1e-9,
               hd: float = 1e-8) -> dict:
    """Optics of a line (or a portion of a ring given as its own element list)
    from given initial conditions, for an assigned momentum deviation (paper
    section "Twiss module"): init = (x, px, y, py, betx, alfx, bety, alfy, dx,
    dpx, dy, dpy) at the line start.  The orbit is the tracked initial orbit;
    the maps M_e and momentum columns m_e come from central differences of
    particles displaced around it as in twiss(); per plane
    beta = ((p beta0 - q alpha0)^2 + q^2)/beta0,
    alpha = -((p beta0 - q alpha0)(r beta0 - t alpha0) + q t)/beta0,
    phase = atan2(q, p beta0 - q alpha0) unwrapped from 0; dispersion
    eta_e = M_e eta_0 + m_e.  Same columns as twiss()."""
    el = _els(elements)
    n_el = len(el)
    init = np.asarray(init, dtype=np.float64)
    u = init[:4]
    rows = [np.r_[u, 0.0, delta0]]
    for k in range(4):
        for sgn in (1.0, -1.0):
            v = np.r_[u, 0.0, delta0]
            v[k] += sgn * h
            rows.append(v)
    for sgn in (1.0, -1.0):
        rows.append(np.r_[u, 0.0, delta0 + sgn * hd])
    out = track_record(el, ref, np.array(rows))
    M = np.empty((n_el + 1, 4, 4))
    for k in range(4):
        M[:, :, k] = (out[:, 1 + 2 * k, :4] - out[:, 2 + 2 * k, :4]) / (2.0 * h)
    md = (out[:, 9, :4] - out[:, 10, :4]) / (2.0 * hd)
    eta = np.einsum("eij,j->ei", M, init[8:12]) + md
    tab = {"s": np.concatenate([[0.0], np.cumsum(np.where(np.isin(el["type"], (1, 2)),
                                                          el["length"], 0.0))]),
           "x": out[:, 0, 0], "px": out[:, 0, 1], "y": out[:, 0, 2], "py": out[:, 0, 3],
           "dx": eta[:, 0], "dpx": eta[:, 1], "dy": eta[:, 2], "dpy": eta[:, 3]}
    for name, o, b0, a0 in (("x", 0, init[4], init[5]), ("y", 2, init[6], init[7])):
        p_, q_, r_, t_ = M[:, o, o], M[:, o, o + 1], M[:, o + 1, o], M[:, o + 1, o + 1]
        bb = p_ * b0 - q_ * a0
        tab["bet" + name] = (bb * bb + q_ * q_) / b0
        tab["alf" + name] = -(bb * (r_ * b0 - t_ * a0) + q_ * t_) / b0
        th = np.arctan2(q_, bb)
        mu = np.zeros(n_el + 1)
        for e in range(1, n_el + 1):
            mu[e] = mu[e - 1] + (th[e] - th[e - 1]) % (2.0 * math.pi)
        tab["mu" + name] = mu
    return tab


S4 = np.array([[0.0, 1.0, 0.0, 0.0], [-1.0, 0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 1.0],
               [0.0, 0.0, -1.0, 0.0]])


def twiss_coupled(elements, ref, delta0: float = 0.0, h: float = 1e-9, hd: float = 1e-8,
                  max_iter: int = 30, tol: float = 1e-15) -> dict:
    """Transverse optics with linear coupling (paper section "Twiss module":
    the normal form from the eigenvalues and eigenvectors of the one-turn
    Jacobian, the eigenvectors propagated by tracking).  From the 4x4 one-turn
    map J at the closed orbit (the same orbit and maps as twiss()):
      eigenvalues e^{+-i mu_I}, e^{+-i mu_II}; of each conjugate pair the
      eigenvector v with Im(v^H S v) > 0 is kept and scaled so that
      v^H S v = 2i (S the 4x4 symplectic form); mode I is the one whose
      summed horizontal beta along the line, sum_e |v_e,1|^2, exceeds its
      summed vertical beta sum_e |v_e,3|^2 (the x-like mode);
      at element e, v_e = M_e v: beta_xI = |v_e,1|^2, beta_yI = |v_e,3|^2 (and
      likewise for mode II); the phase of mode I follows arg(v_e,1) and that
      of mode II arg(v_e,3): through a drift the phase advances by the change
      of the argument taken in [0, 2 pi), through a thin element (no length:
      a kick or a frame change, which can turn the components) by the change
      taken in (-pi, pi]; the eigen-tunes are the phases at the line end /
      2 pi.
    For an uncoupled ring beta_xI, beta_yII and the phases equal the
    uncoupled ones (v = (sqrt(beta), (i - alpha)/sqrt(beta), 0, 0))."""
    el = _els(elements)
    base = twiss(el, ref, delta0=delta0, h=h, hd=hd, max_iter=max_iter, tol=tol)
    u = np.array([base["x"][0], base["px"][0], base["y"][0], base["py"][0]])
    rows = [np.r_[u, 0.0, delta0]]
    for k in range(4):
        for sgn in (1.0, -1.0):
            v = np.r_[u, 0.0, delta0]
            v[k] += sgn * h
            rows.append(v)
    out = track_record(el, ref, np.array(rows))
    n_el = len(el)
    M = np.empty((n_el + 1, 4, 4))
    for k in range(4):
        M[:, :, k] = (out[:, 1 + 2 * k, :4] - out[:, 2 + 2 * k, :4]) / (2.0 * h)
    lam, vec = np.linalg.eig(M[n_el])
    modes = []
    for j in range(4):
        v = vec[:, j]
        c = np.conj(v) @ S4 @ v
        if c.imag <= 0.0:
            continue
        v = v * math.sqrt(2.0 / c.imag)
        modes.append(v)
    if len(modes) != 2:
        raise ValueError("one-turn map is not stably oscillating in two modes")
    prop = [np.einsum("eij,j->ei", M, v) for v in modes]
    xlike = [float(np.sum(np.abs(ve[:, 0]) ** 2) - np.sum(np.abs(ve[:, 2]) ** 2)) for ve in prop]
    order = (0, 1) if xlike[0] >= xlike[1] else (1, 0)
    res = {"s": base["s"], "qx_uncoupled": base["qx"], "qy_uncoupled": base["qy"]}
    for name, j, comp in (("1", order[0], 0), ("2", order[1], 2)):
        ve = prop[j]
        res["betx" + name] = np.abs(ve[:, 0]) ** 2
        res["bety" + name] = np.abs(ve[:, 2]) ** 2
        th = np.angle(ve[:, comp])
        mu = np.zeros(n_el + 1)
        for e in range(1, n_el + 1):
            dth = (th[e] - th[e - 1]) % (2.0 * math.pi)
            if not (int(el["type"][e - 1]) in (1, 2) and el["length"][e - 1] > 0.0):
                if dth > math.pi:
                    dth -= 2.0 * math.pi
            mu[e] = mu[e - 1] + dth
        res["mu" + name] = mu
        res["q" + name] = mu[n_el] / (2.0 * math.pi)
    return res


def chromaticity(elements, ref, delta0: float = 0.0, eps: float = 1e-6, **kw):
    """dQ/d delta as (Q(delta0 + eps) - Q(delta0 - eps)) / (2 eps), each tune from
    the optics by tracking at that momentum (its own closed orbit)."""
    p = twiss(elements, ref, delta0=delta0 + eps, **kw)
    m = twiss(elements, ref, delta0=delta0 - eps, **kw)
    return (p["qx"] - m["qx"]) / (2.0 * eps), (p["qy"] - m["qy"]) / (2.0 * eps)


def reference(ref) -> tuple[float, float]:
    """(beta0, gamma0) as the oracle computes them."""
    out = np.zeros(2)
    r = _ref3(ref)
    lib().oracle_reference(r.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p))
    return float(out[0]), float(out[1])


def one_turn(elements, ref, u6, n_turns: int = 1, radiation: int = 0) -> np.ndarray:
    """Canonical map u = (x, px, y, py, zeta, pzeta) -> T^n(u); radiation 1
    adds the mean energy loss of radiating multipoles (no deviates)."""
    el = _els(elements)
    r = _ref3(ref)
    u = np.array(u6, dtype=np.float64)
    st = lib().oracle_track_canonical(el.ctypes.data_as(ctypes.c_void_p), ctypes.c_int32(len(el)),
                                      r.ctypes.data_as(ctypes.c_void_p),
                                      u.ctypes.data_as(ctypes.c_void_p), ctypes.c_int32(n_turns),
                                      ctypes.c_int32(radiation))
    if st != 1:
        raise RuntimeError("reference trajectory lost (state %d)" % st)
    return u


DEFAULT_FD_STEPS = np.array([1e-7, 1e-9, 1e-7, 1e-9, 1e-6, 1e-8])


def jacobian(elements, ref, u0=None, h=DEFAULT_FD_STEPS, n_turns: int = 1,
             richardson: bool = True, radiation: int = 0) -> np.ndarray:
    """Central-difference Jacobian of the canonical one-turn map (Twiss step 2):
    J[:, j] = (T(u0 + h_j e_j) - T(u0 - h_j e_j)) / (2 h_j), optionally
    Richardson-extrapolated from steps h and h/2."""
    u0 = np.zeros(6) if u0 is None else np.asarray(u0, dtype=np.float64)

    def cd(hh):
        J = np.zeros((6, 6))
        for j in range(6):
            e = np.zeros(6)
            e[j] = hh[j]
            J[:, j] = (one_turn(elements, ref, u0 + e, n_turns, radiation)
                       - one_turn(elements, ref, u0 - e, n_turns, radiation)) / (2.0 * hh[j])
        return J

    h = np.asarray(h, dtype=np.float64)
    J1 = cd(h)
    if not richardson:
        return J1
    J2 = cd(h / 2.0)
    return (4.0 * J2 - J1) / 3.0


S6 = np.kron(np.eye(3), np.array([[0.0, 1.0], [-1.0, 0.0]]))


def symplectic_error(J: np.ndarray) -> float:
    return float(np.max(np.abs(J.T @ S6 @ J - S6)))


def normal_form_2x2(M: np.ndarray) -> dict:
    """Uncoupled linear normal form of a 2x2 block (Twiss step 3 for one plane):
    cos mu = tr/2, sin mu = sign(M12) sqrt(1 - cos^2), beta = M12/sin mu,
    alpha = (M11 - M22)/(2 sin mu)."""
    cmu = 0.5 * (M[0, 0] + M[1, 1])
    smu = math.copysign(math.sqrt(max(0.0, 1.0 - cmu * cmu)), M[0, 1])
    beta = M[0, 1] / smu
    alpha = (M[0, 0] - M[1, 1]) / (2.0 * smu)
    mu = math.atan2(smu, cmu) % (2.0 * math.pi)
    return {"cos_mu": cmu, "sin_mu": smu, "beta": beta, "alpha": alpha,
            "q": mu / (2.0 * math.pi)}


def closed_orbit_6d(elements, ref, radiation: int = 0, guess=None, h=DEFAULT_FD_STEPS,
                    tol: float = 1e-15, max_iter: int = 20) -> np.ndarray:
    """Fixed point u* = T(u*) of the canonical 6D one-turn map (RF included;
    with radiation 1 the mean energy loss shifts it) by Newton's method,
    u <- u + (I - J)^-1 (T(u) - u), J by central differences at u, until the
    largest component of T(u) - u is below tol or stops decreasing."""
    u = np.zeros(6) if guess is None else np.array(guess, dtype=np.float64)
    best = np.inf
    for _ in range(max_iter):
        r = one_turn(elements, ref, u, 1, radiation) - u
        res = float(np.max(np.abs(r)))
        if res <= tol or res >= best:
            break
        best = res
        J = jacobian(elements, ref, u, h, richardson=False, radiation=radiation)
        u = u + np.linalg.solve(np.eye(6) - J, r)
    return u


def _mode_shares(v) -> np.ndarray:
    """Im(conj(v_2p) v_2p+1) per plane p: the plane's part of v^H S v / 2i."""
    return np.array([np.imag(np.conj(v[2 * p]) * v[2 * p + 1]) for p in range(3)])


def normal_form_6d(elements, ref, radiation: int = 0, h=DEFAULT_FD_STEPS) -> dict:
    """6D linear normal form by tracking (paper section "Twiss module": the
    closed orbit by a root finder, the one-turn Jacobian by central
    differences, the eigenvalues and eigenvectors of the Jacobian; with
    radiation their moduli give the damping per turn).  In canonical
    coordinates (x, px, y, py, zeta, pzeta): the eigen-decomposition is
    LAPACK's (numpy.linalg.eig); of each complex-conjugate pair the
    eigenvector with Im(v^H S v) > 0 is kept and scaled to v^H S v = 2i;
    mode k is the one whose share Im(conj(v_2p) v_2p+1) is largest in plane
    p = k (the assignment of modes to planes that maximises the summed
    shares), its phase set so that v_2k is real and positive.  Returns the
    closed orbit co, J, per mode the eigenvalue lam, tune q = arg(lam)/2 pi
    mod 1, damping -ln|lam| per turn and eigenvector v (6 complex)."""
    import itertools
    co = closed_orbit_6d(elements, ref, radiation, h=h)
    J = jacobian(elements, ref, co, h, radiation=radiation)
    w, V = np.linalg.eig(J)
    modes = []
    used = np.zeros(6, dtype=bool)
    for i in np.argsort(-np.abs(w.imag)):
        if used[i]:
            continue
        j = int(np.argmin(np.abs(w - np.conj(w[i])) + used * 1e300 + (np.arange(6) == i) * 1e300))
        used[i] = used[j] = True
        v = V[:, i]
        lam = w[i]
        n = float(np.sum(_mode_shares(v)))
        if n < 0:
            v, lam, n = np.conj(v), np.conj(lam), -n
        modes.append((lam, v / math.sqrt(n)))
    if len(modes) != 3:
        raise RuntimeError("the one-turn map has real eigenvalues (unstable or at a resonance)")
    shares = np.array([_mode_shares(v) for _, v in modes])
    perm = max(itertools.permutations(range(3)), key=lambda pm: sum(shares[pm[k], k] for k in range(3)))
    lam = np.zeros(3, dtype=complex)
    vec = np.zeros((3, 6), dtype=complex)
    for k in range(3):
        l, v = modes[perm[k]]
        ph = v[2 * k] / abs(v[2 * k])
        lam[k] = l
        vec[k] = v / ph
    q = (np.angle(lam) / (2.0 * math.pi)) % 1.0
    return {"co": co, "J": J, "lam": lam, "q": q, "damping": -np.log(np.abs(lam)), "v": vec}


def matched_gaussian(nf: dict, ref, eps, gauss) -> np.ndarray:
    """Gaussian ensemble matched to the 6D normal form: for mode k with
    emittance eps_k, z_k = sqrt(eps_k) (g_2k + i g_2k+1) from the given
    standard normals g (n, 6); u = co + sum_k Re(v_k z_k) in canonical
    coordinates; returned as (x, px, y, py, zeta, delta) rows with
    ptau = beta0 pzeta and delta = w / (1 + sqrt(1 + w)), w = ptau (ptau + 2/beta0)."""
    b0, _ = reference(ref)
    g = np.asarray(gauss, dtype=np.float64)
    u = np.tile(nf["co"], (len(g), 1))
    for k in range(3):
        z = math.sqrt(eps[k]) * (g[:, 2 * k] + 1j * g[:, 2 * k + 1])
        u = u + np.real(np.outer(z, nf["v"][k]))
    ptau = b0 * u[:, 5]
    w = ptau * (ptau + 2.0 / b0)
    out = u.copy()
    out[:, 5] = w / (1.0 + np.sqrt(1.0 + w))
    return out


def regular_mask(elements, ref, coords6, n_turns: int = 100, rtol: float = 1e-13,
                 floor_frac: float = 1e-3) -> np.ndarray:
    """Regular-orbit classification decided by the oracle alone: particle i is
    regular if its twin, started with x moved by one ulp, stays within
    ``rtol * max(|o|, s_c)`` of it in every coordinate after ``n_turns`` turns,
    where s_c = floor_frac x the ensemble RMS of that coordinate.  Lost
    particles (either twin) are not regular."""
    c = np.array(coords6, dtype=np.float64).reshape(-1, 6)
    a = init(c, ref)
    c2 = c.copy()
    c2[:, 0] = np.nextafter(c2[:, 0], np.inf)
    b = init(c2, ref)
    track(elements, ref, a, n_turns)
    track(elements, ref, b, n_turns)
    ok = (a.state == 1) & (b.state == 1)
    ca, cb = a.coords(), b.coords()
    if ok.any():
        sc = floor_frac * np.sqrt(np.mean(ca[ok] ** 2, axis=0))
    else:
        sc = np.zeros(6)
    err = np.abs(ca - cb) / np.maximum(np.abs(ca), sc[None, :])
    return ok & np.all(err <= rtol, axis=1)


# ------------------------------------------------------------------ RNG
def philox(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block: 4 words from a 4-word counter and 2-word key."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def philox_stream(seed: int, ctr0, n_blocks: int) -> np.ndarray:
    """n_blocks consecutive blocks from counter ctr0 (128-bit increment), key = seed."""
    out = np.zeros(4 * n_blocks, dtype=np.uint32)
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr0])
    lib().oracle_philox_stream(ctypes.c_uint64(seed), c, ctypes.c_int64(n_blocks),
                               out.ctypes.data_as(ctypes.c_void_p))
    return out


def philox_constants() -> np.ndarray:
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox_constants(o)
    return np.array(list(o), dtype=np.uint32)


def uniform(wa: int, wb: int) -> float:
    return float(lib().oracle_uniform(wa, wb))


def gauss_at(seed: int, pid: int, turn: int, element: int, draw: int = 0) -> float:
    return float(lib().oracle_gauss_at(seed, pid, turn, element, draw))


# ------------------------------------------------------------ retire policy
def audit_mask(seed: int, pids, fraction: float = 0.05) -> np.ndarray:
    """Audit set of the retire policy: particle id k is audited iff the first
    word of Philox4x32-10 with key = seed and counter (k_lo, k_hi, 2^32 - 1, 0)
    is below ceil(fraction 2^32), an exact integer comparison."""
    import math
    th = min(math.ceil(fraction * 2.0 ** 32), 0xFFFFFFFF)
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    out = np.zeros(len(pids), dtype=bool)
    for i, k in enumerate(np.asarray(pids, dtype=np.int64)):
        k = int(k) & 0xFFFFFFFFFFFFFFFF
        w = philox((k & 0xFFFFFFFF, k >> 32, 0xFFFFFFFF, 0), key)
        out[i] = int(w[0]) < th
    return out


def dynamic_aperture(state, radii, n_r: int, n_theta: int) -> np.ndarray:
    """Per-ray dynamic aperture of a polar scan (particle index j n_r + i is
    radius i of ray j): the smallest radius on the ray whose particle was lost
    (state <= 0); rays with no loss get +inf (censored at the scan's edge)."""
    st = np.asarray(state).reshape(n_theta, n_r)
    r = np.asarray(radii, dtype=np.float64).reshape(n_theta, n_r)
    out = np.full(n_theta, np.inf)
    for j in range(n_theta):
        lost = np.nonzero(st[j] <= 0)[0]
        if len(lost):
            out[j] = r[j, lost].min()
    return out


def wilson_upper(k: int, n: int, z: float = 1.6448536269514722) -> float:
    """Upper end of Wilson's score interval for k successes in n trials at
    normal quantile z (one-sided 95 % by default); 1 for n = 0.  The audit of
    the retire policy bounds its false-retire fraction with it."""
    if n == 0:
        return 1.0
    p = k / n
    centre = p + z * z / (2 * n)
    half = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n))
    return min(1.0, (centre + half) / (1 + z * z / n))


def audit_verdict(state, audit_flags, fallback_rate: float) -> dict:
    """The audit after tracking to the horizon: the flagged particles are the
    audit; lost ones have state 0 or -1; the retirements are rejected (full
    tracking resumes) iff some particle is retired (state 2) and the Wilson
    upper bound of the audit's loss fraction exceeds fallback_rate."""
    st = np.asarray(state)
    fl = np.asarray(audit_flags) != 0
    audited = int(fl.sum())
    lost = int((fl & ((st == 0) | (st == -1))).sum())
    upper = wilson_upper(lost, audited)
    return {"audited": audited, "lost": lost, "upper": upper,
            "fallback": bool((st == 2).any() and upper > fallback_rate)}


def rule_score(feat) -> np.ndarray:
    """Score of the retire rule without the network: minus the larger of the
    two tune-diffusion features (columns 8 and 9); NaN if either is NaN."""
    f = np.asarray(feat, dtype=np.float32)
    return -np.maximum(f[:, 8], f[:, 9])


def select_threshold(logit, label, max_false_rate: float):
    """Retire threshold by brute force over every candidate: the smallest
    logit value tau (finite) such that among rows with logit >= tau the
    fraction with label 0 is <= max_false_rate; +inf if none."""
    z = np.asarray(logit, dtype=np.float64)
    y = np.asarray(label)
    best = np.inf
    for t in np.unique(z[np.isfinite(z)]):
        sel = z >= t
        if np.mean(y[sel] == 0) <= max_false_rate:
            best = min(best, t)
    return best


# ---------------------------------------------------- elementary functions
def xsin(x: float) -> float:
    """The tracker's sine (the series evaluation both implementations follow)."""
    return float(lib().oracle_sin(x))


def xcos(x: float) -> float:
    return float(lib().oracle_cos(x))


def xlog(x: float) -> float:
    return float(lib().oracle_log(x))
