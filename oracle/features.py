"""FP64 reference of the early-turn features of the loss predictor
(test infrastructure only).

Input: the coordinates (x, px, y, py) recorded at element 0 at the start of
turns 0..T-1 (T = 1024), the linear optics (beta, alpha per plane) at element
0, the emittance that defines one sigma, and the aperture radius.  The paper
only cites chaos indicators and machine-learned dynamic aperture; the feature
list is this project's reading of the workload description ("initial
amplitudes, FFT tune estimates, action drift, max excursion; 16 features"):

  normalised coordinates  u = x / sqrt(beta),  pu = (alpha x + beta px) / sqrt(beta)
  action                  J = (u^2 + pu^2) / 2,  amplitude A = sqrt(2 J / emit) [sigma]
  f0, f1   A_x, A_y at turn 0             f2  sqrt(f0^2 + f1^2)     f3  atan2(f1, f0)
  f4, f5   tunes from turns 0..511        f6, f7  tunes from turns 512..1023
  f8, f9   log10(circular |f6 - f4| + 1e-12), same for y      (tune diffusion)
  f10, f11 (<J> over the last quarter + e) / (<J> over the first quarter + e) - 1
  f12, f13 std(J) / (mean(J) + e) over all turns          (e = 1e-6 emit)
  f14      max_t sqrt(x^2 + y^2) / r_aperture
  f15      max_t (A_x^2 + A_y^2) / (f2^2 + 1e-6)

Tune of a 512-turn window: complex signal z_n = u_n - i pu_n (a normalised
rotation by 2 pi Q gives z_n ~ exp(2 pi i Q n)), Hann window
w_n = sin^2(pi n / 512), discrete Fourier transform Z_k = sum_n w_n z_n
exp(-2 pi i k n / 512), peak bin k*, and the Hann three-point interpolation
d = 2 (|Z_k*+1| - |Z_k*-1|) / (|Z_k*-1| + 2 |Z_k*| + |Z_k*+1|) (indices mod
512); Q = ((k* + d) / 512) mod 1.
"""
from __future__ import annotations

import numpy as np

N_FEATURES = 16
WINDOW = 512


def normalise(x, px, beta, alpha):
    sb = np.sqrt(beta)
    return x / sb, (alpha * x + beta * px) / sb


def tune_fft(u: np.ndarray, pu: np.ndarray) -> np.ndarray:
    """Tunes of the signals along the last axis (length WINDOW)."""
    n = u.shape[-1]
    w = np.sin(np.pi * np.arange(n) / n) ** 2
    Z = np.abs(np.fft.fft((u - 1j * pu) * w, axis=-1))
    k = np.argmax(Z, axis=-1)
    a = np.take_along_axis(Z, ((k - 1) % n)[..., None], -1)[..., 0]
    b = np.take_along_axis(Z, k[..., None], -1)[..., 0]
    c = np.take_along_axis(Z, ((k + 1) % n)[..., None], -1)[..., 0]
    d = 2.0 * (c - a) / (a + 2.0 * b + c)
    return ((k + d) / n) % 1.0


def circ_diff(a, b):
    d = np.abs(a - b) % 1.0
    return np.minimum(d, 1.0 - d)


def features(rec: np.ndarray, twiss4, emit: float, r_aperture: float) -> np.ndarray:
    """rec: [T, 4, N] recorded (x, px, y, py); returns [N, 16]."""
    rec = np.asarray(rec, dtype=np.float64)
    T = rec.shape[0]
    assert T == 2 * WINDOW
    bx, ax, by, ay = twiss4
    x, px, y, py = rec[:, 0], rec[:, 1], rec[:, 2], rec[:, 3]        # [T, N]
    ux, pux = normalise(x, px, bx, ax)
    uy, puy = normalise(y, py, by, ay)
    jx = 0.5 * (ux * ux + pux * pux)
    jy = 0.5 * (uy * uy + puy * puy)
    e = 1e-6 * emit
    f = np.zeros((rec.shape[2], N_FEATURES))
    f[:, 0] = np.sqrt(2 * jx[0] / emit)
    f[:, 1] = np.sqrt(2 * jy[0] / emit)
    f[:, 2] = np.hypot(f[:, 0], f[:, 1])
    f[:, 3] = np.arctan2(f[:, 1], f[:, 0])
    f[:, 4] = tune_fft(ux[:WINDOW].T, pux[:WINDOW].T)
    f[:, 5] = tune_fft(uy[:WINDOW].T, puy[:WINDOW].T)
    f[:, 6] = tune_fft(ux[WINDOW:].T, pux[WINDOW:].T)
    f[:, 7] = tune_fft(uy[WINDOW:].T, puy[WINDOW:].T)
    f[:, 8] = np.log10(circ_diff(f[:, 6], f[:, 4]) + 1e-12)
    f[:, 9] = np.log10(circ_diff(f[:, 7], f[:, 5]) + 1e-12)
    q = T // 4
    f[:, 10] = (jx[-q:].mean(0) + e) / (jx[:q].mean(0) + e) - 1.0
    f[:, 11] = (jy[-q:].mean(0) + e) / (jy[:q].mean(0) + e) - 1.0
    f[:, 12] = jx.std(0) / (jx.mean(0) + e)
    f[:, 13] = jy.std(0) / (jy.mean(0) + e)
    f[:, 14] = np.max(np.hypot(x, y), axis=0) / r_aperture
    f[:, 15] = np.max(2 * (jx + jy) / emit, axis=0) / (f[:, 2] ** 2 + 1e-6)
    return f


def record(elements, ref, coords, turns: int = 2 * WINDOW, nthreads: int = 0,
           fp32: bool = False) -> tuple:
    """Track with the oracle and record (x, px, y, py) at element 0 at the
    start of each turn; returns (rec [turns, 4, N], oracle particles).  A
    particle lost during turn u keeps, from turn u + 1 on, the coordinates it
    had when it entered the element that lost it.  ``fp32`` rounds the record
    to single precision, the recorder's storage format (values returned as
    float64)."""
    import oracle
    p = oracle.init(coords, ref)
    rec = np.zeros((turns, 4, p.n))
    for t in range(turns):
        rec[t] = np.stack([p.x, p.px, p.y, p.py])
        oracle.track(elements, ref, p, 1, nthreads=nthreads)
    if fp32:
        rec = rec.astype(np.float32).astype(np.float64)
    return rec, p
