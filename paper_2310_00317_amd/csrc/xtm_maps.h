// xtm_maps.h -- element maps of the thin-lattice tracker as device functions.
//
// Shared by the statically built kernels and by the per-line kernels that
// the library generates and compiles at run time, so both apply exactly the
// same operations.  Every fused multiply-add is an explicit fma(); the code is
// compiled with -ffp-contract=off, so the operation order written here is the
// rounding contract (paper section "Lattice modelling and single particle
// tracking": thin elements, multipolar errors, RF cavities, tilts and
// misalignments as reference-frame changes; apertures from section
// "Particle-matter interaction and collimation studies").
#pragma once

namespace xtmm {

struct Pt {
  double x, px, y, py, zeta, delta, ptau, rpp, rvv;
  // invariants of delta refreshed whenever ptau changes; they are the values
  // the formulas would recompute, so caching them does not change rounding
  double opd2, u, bpt;
};

__device__ __forceinline__ void refresh(Pt& q, double beta0) {
  const double opd = 1.0 + q.delta;
  q.opd2 = opd * opd;
  q.u = q.delta * (2.0 + q.delta);
  q.bpt = beta0 * q.ptau;
}

// Square root and quotient for operands well inside the exponent range,
// both correctly rounded (the same values as sqrt() and a/b, whose generic
// sequences add exponent-scaling and special-case steps for operands near
// the limits; without them the drift's dependent chain is a quarter shorter).
//   sqrt_in: x in [2^-600, 2^600].  Goldschmidt's iteration from the
//   hardware's reciprocal-square-root estimate y: g = x y ~ sqrt x and
//   h = y/2 ~ 1/(2 sqrt x) refined together by r = 1/2 - h g, then two
//   Newton corrections g += (x - g^2) h.
//   div_in: a/b for |a| in [2^-600, 2^1000], b in [2^-300, 3], |a/b| within
//   [2^-960, 2^1000].  Newton's iteration r += r (1 - b r) twice from the
//   hardware's reciprocal estimate, the product q = a r, and one correction
//   by the exact remainder, q + r (a - b q) (Markstein's quotient step).  The
//   reciprocal converges from below and may stop one unit short of the
//   rounded 1/b; the corrected quotient is then still the rounded a/b except
//   in one family: a divisor whose significand is all ones (b = 2^k (2 -
//   2^-52)) and a power-of-two numerator, where the exact q + r (a - b q) is
//   a tie.  Callers keep that family out (the drift's window below).
//   div_by_root: a / sqrt_in(x) with the reciprocal taken from the square
//   root's own iteration: after Goldschmidt's step h approximates
//   1/(2 sqrt x) about as closely as one Newton step from the hardware
//   reciprocal would (both estimates are within 2^-24 of their values, so
//   either is within about 2^-47 after it), and one Newton step on 2h, the
//   product and Markstein's step follow as in div_in (the same exclusions).
//   This takes the reciprocal estimate and one dependent Newton step off the
//   chain from the square root to the quotient.
__device__ __forceinline__ double sqrt_in(double x, double& h_out) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y;
  double h = y * 0.5;
  const double r = fma(-h, g, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  h_out = h;
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
}

__device__ __forceinline__ double sqrt_in(double x) {
  double h;
  return sqrt_in(x, h);
}

__device__ __forceinline__ double div_by_root(double a, double root, double h) {
  double r = 2.0 * h;
  const double e = fma(-root, r, 1.0);
  r = fma(r, e, r);
  const double q = a * r;
  const double rho = fma(-root, q, a);
  return fma(rho, r, q);
}

__device__ __forceinline__ double div_in(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  double e = fma(-b, r, 1.0);
  r = fma(r, e, r);
  e = fma(-b, r, 1.0);
  r = fma(r, e, r);
  const double q = a * r;
  const double rho = fma(-b, q, a);
  return fma(rho, r, q);
}

// Exact drift over L: pz = sqrt((1+d)^2 - px^2 - py^2), lp = L / pz,
// x += px lp, y += py lp, zeta += lp ((d(2+d) - px^2 - py^2) / (1+pz) - beta0 ptau),
// every square root and quotient correctly rounded.  The particle is lost
// unless pz^2 > 0 (imaginary longitudinal momentum, or NaN).
// The short sequences above serve the window
//   pz^2 in (2^-600, 4), so pz in (2^-300, 2) and 1 + pz in (1, 3);
//   a = d(2+d) - px^2 - py^2 with |a| >= 2^-600 (|a| < 2^1000 whenever pz^2
//   is finite);
//   1 + pz != 2 - 2^-52, the one all-ones divisor in (1, 3);
//   the drift length as the lattice packer classed it (the drift record's
//   order): 0, |L| in [2^-600, 2^600] and not a power of two, served for
//   every pz; 1, a power of two in that range, served unless pz's
//   significand is all ones (the one case of L / pz in the excluded family);
//   2, any other length, zero included, never served.
// Other operands take the generic operations on a rare branch.
struct DriftIn {
  double px2, py2, pz2, a;
};

__device__ __forceinline__ DriftIn drift_in(const Pt& q) {
  DriftIn d;
  d.px2 = q.px * q.px;
  d.py2 = q.py * q.py;
  d.pz2 = q.opd2 - d.px2 - d.py2;
  d.a = q.u - d.px2 - d.py2;
  return d;
}

// window test of the operands known before the square root
__device__ __forceinline__ bool drift_window(const DriftIn& d) {
  return (d.pz2 > 0x1p-600) & (d.pz2 < 4.0) & (fabs(d.a) >= 0x1p-600);
}

__device__ __forceinline__ void drift_apply(Pt& q, double lp, double dq) {
  q.x = fma(q.px, lp, q.x);
  q.y = fma(q.py, lp, q.y);
  q.zeta = fma(lp, dq - q.bpt, q.zeta);
}

__device__ __forceinline__ bool all_ones_significand(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  return (b & 0xfffffffffffffull) == 0xfffffffffffffull;
}

// Quotients of the drift: the short sequences where the window holds
// (`fast` returns whether it did), else the generic operations (for a lost
// particle the results are NaN and unused).  len_class: the drift record's
// order (see the window above).
__device__ __forceinline__ void drift_quotients(double L, const DriftIn& d, int len_class,
                                                double& lp, double& dq, bool& fast) {
  double h;
  const double pz = sqrt_in(d.pz2, h);
  const double b1 = 1.0 + pz;
  lp = div_by_root(L, pz, h);
  dq = div_in(d.a, b1);
  const bool len_ok = (len_class == 0) | ((len_class == 1) & !all_ones_significand(pz));
  fast = len_ok & drift_window(d) & (b1 != 0x1.fffffffffffffp+0);
}

__device__ __forceinline__ void drift_generic(double L, const DriftIn& d, double& lp, double& dq) {
  const double pz = sqrt(d.pz2);
  lp = L / pz;
  dq = d.a / (1.0 + pz);
}

// The whole drift; returns false if the particle is lost (its coordinates
// are then NaN and must not be used).  len_class: the drift record's order
// (0 for a length known to be served for every pz).
__device__ __forceinline__ bool drift_exact(Pt& q, double L, int len_class = 0) {
  const DriftIn d = drift_in(q);
  double lp, dq;
  bool fast;
  drift_quotients(L, d, len_class, lp, dq, fast);
  if (!fast) drift_generic(L, d, lp, dq);
  drift_apply(q, lp, dq);
  return d.pz2 > 0.0;
}

// The exact drift's loss test alone.
__device__ __forceinline__ bool drift_ok(const Pt& q) { return drift_in(q).pz2 > 0.0; }

// Drift of H = pzeta - (1+d) + (px^2+py^2)/(2(1+d)) over L.
__device__ __forceinline__ void drift_expanded(Pt& q, double L) {
  const double lr = L * q.rpp;
  q.x = fma(q.px, lr, q.x);
  q.y = fma(q.py, lr, q.y);
  const double pp = q.px * q.px + q.py * q.py;
  const double r3 = q.rpp * q.rpp * q.rpp;
  const double dz = (q.delta - q.bpt) * q.rpp - 0.5 * pp * r3 * (1.0 + q.bpt);
  q.zeta = fma(L, dz, q.zeta);
}

// Thin multipole of order N: dpx - i dpy = -sum_n c_n (x + i y)^n with
// c = (cr_N, ci_N, cr_{N-1}, ci_{N-1}, ..., cr_0, ci_0), by Horner:
// b <- b z + c_n, re = fma(br, x, fma(-bi, y, cr)), im = fma(br, y, fma(bi, x, ci)).
// Writes the field kick (dpx, dpy) to kx, ky.
template <int N>
__device__ __forceinline__ void multipole(Pt& q, const double* __restrict__ c, double& kx,
                                          double& ky) {
  double br = c[0], bi = c[1];
#pragma unroll
  for (int k = 1; k <= N; ++k) {
    const double cr = c[2 * k], ci = c[2 * k + 1];
    const double tr = fma(br, q.x, fma(-bi, q.y, cr));
    const double ti = fma(br, q.y, fma(bi, q.x, ci));
    br = tr;
    bi = ti;
  }
  q.px = q.px - br;
  q.py = q.py + bi;
  kx = -br;
  ky = bi;
}

// Frame curvature of a thin bend: dpx += hxl (1+d) - (knl0 hxl) x / Lr (Lr > 0),
// zeta -= hxl x (1 + beta0 ptau) rpp.
__device__ __forceinline__ void curvature(Pt& q, double hxl, double k0h, double lr) {
  double dpx = hxl * (1.0 + q.delta);
  if (lr > 0.0) dpx = dpx - k0h * q.x / lr;
  const double dz = hxl * q.x * (1.0 + q.bpt) * q.rpp;
  q.px = q.px + dpx;
  q.zeta = q.zeta - dz;
}

// Elementary functions used by the maps: the RF sine and the Box-Muller
// logarithm and cosine are evaluated from their series, step by step as the
// reference implementation does, so results agree bit for bit instead of
// within the ulp by which two math libraries may differ.
//   sin/cos: n = rint(x 2/pi); r = x - n pi/2 by three fused multiply-adds
//   with pi/2 = P1 + P2 + P3 (P1 = pi/2 rounded, P2 the remainder rounded,
//   P3 what is left); Taylor series of
//   sin r (to r^17) and cos r (to r^16) by Horner in r^2, the first omitted
//   terms under 0.02 ulp on |r| <= pi/4; quadrant n mod 4.
//   log: x = m 2^e, m in [sqrt(1/2), sqrt(2)); log m = 2 atanh((m-1)/(m+1))
//   by its odd series up to the 21st power (|s| <= 0.1716: the next term is
//   below 2.2e-19); log x = e ln2 + log m, ln 2 split like pi/2.  Domain:
//   finite x (sin, cos); finite x > 0 (log).
__device__ __forceinline__ void sincos_core(double x, double& sr, double& cr, int& quad) {
  const double n = rint(x * 0.6366197723675814);
  double r = fma(-n, 1.5707963267948966, x);
  r = fma(-n, 6.123233995736766e-17, r);
  r = fma(-n, -1.4973849048591698e-33, r);
  const double z = r * r;
  double a = 1.0 / 355687428096000.0;          // 1/17!
  a = fma(a, z, -1.0 / 1307674368000.0);       // -1/15!
  a = fma(a, z, 1.0 / 6227020800.0);           // 1/13!
  a = fma(a, z, -1.0 / 39916800.0);            // -1/11!
  a = fma(a, z, 1.0 / 362880.0);               // 1/9!
  a = fma(a, z, -1.0 / 5040.0);                // -1/7!
  a = fma(a, z, 1.0 / 120.0);                  // 1/5!
  a = fma(a, z, -1.0 / 6.0);                   // -1/3!
  sr = fma(r * z, a, r);
  double b = 1.0 / 20922789888000.0;           // 1/16!
  b = fma(b, z, -1.0 / 87178291200.0);         // -1/14!
  b = fma(b, z, 1.0 / 479001600.0);            // 1/12!
  b = fma(b, z, -1.0 / 3628800.0);             // -1/10!
  b = fma(b, z, 1.0 / 40320.0);                // 1/8!
  b = fma(b, z, -1.0 / 720.0);                 // -1/6!
  b = fma(b, z, 1.0 / 24.0);                   // 1/4!
  b = fma(b, z, -1.0 / 2.0);                   // -1/2!
  cr = fma(z, b, 1.0);
  quad = (int)((long long)n & 3);
}

__device__ __forceinline__ double xsin(double x) {
  double sr, cr;
  int k;
  sincos_core(x, sr, cr, k);
  const double v = (k & 1) ? cr : sr;
  return (k & 2) ? -v : v;
}

__device__ __forceinline__ double xcos(double x) {
  double sr, cr;
  int k;
  sincos_core(x, sr, cr, k);
  const double v = (k & 1) ? sr : cr;
  return ((k + 1) & 2) ? -v : v;
}

__device__ __forceinline__ double xlog(double x) {
  int e;
  double m = frexp(x, &e);
  if (m < 0.70710678118654752440) {
    m = m * 2.0;
    e = e - 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double p = 1.0 / 21.0;
  p = fma(p, z, 1.0 / 19.0);
  p = fma(p, z, 1.0 / 17.0);
  p = fma(p, z, 1.0 / 15.0);
  p = fma(p, z, 1.0 / 13.0);
  p = fma(p, z, 1.0 / 11.0);
  p = fma(p, z, 1.0 / 9.0);
  p = fma(p, z, 1.0 / 7.0);
  p = fma(p, z, 1.0 / 5.0);
  p = fma(p, z, 1.0 / 3.0);
  const double t = 2.0 * s;
  const double lm = fma(t * z, p, t);
  const double de = (double)e;
  return fma(de, 0.6931471805599453, fma(de, 2.3190468138462996e-17, lm));
}

// delta, rpp, rvv from ptau: v = ptau (ptau + 2/beta0), delta = v/(1 + sqrt(1+v)),
// rpp = 1/(1+delta), rvv = (1+delta)/(1 + beta0 ptau).
__device__ __forceinline__ void from_ptau(Pt& q, double beta0, double two_over_beta0) {
  const double v = q.ptau * (q.ptau + two_over_beta0);
  q.delta = v / (1.0 + sqrt(1.0 + v));
  q.rpp = 1.0 / (1.0 + q.delta);
  q.rvv = (1.0 + q.delta) / (1.0 + beta0 * q.ptau);
  refresh(q, beta0);
}

// Thin RF cavity: ptau += amp sin(phase - k zeta), amp = charge0 V / p0c,
// k = 2 pi f / (beta0 c).
__device__ __forceinline__ void rf(Pt& q, double amp, double k, double phase, double beta0,
                                   double two_over_beta0) {
  const double s = xsin(phase - k * q.zeta);
  q.ptau = q.ptau + amp * s;
  from_ptau(q, beta0, two_over_beta0);
}

// Out-of-line forms for per-line kernels of radiating lattices: there the
// inlined sine, Philox and logarithm constants would hold registers across
// the whole element loop (RF cavities are rare, and the radiation deviates
// are a small part of a bend's work).
__device__ __attribute__((noinline)) void rf_far(Pt& q, double amp, double k, double phase,
                                                 double beta0, double two_over_beta0) {
  rf(q, amp, k, phase, beta0, two_over_beta0);
}

__device__ __forceinline__ void xyshift(Pt& q, double dx, double dy) {
  q.x = q.x - dx;
  q.y = q.y - dy;
}

// Frame rotation: (x, y) <- (c x + s y, c y - s x), same for (px, py).
__device__ __forceinline__ void srotation(Pt& q, double c, double s) {
  const double x = c * q.x + s * q.y;
  const double y = c * q.y - s * q.x;
  const double px = c * q.px + s * q.py;
  const double py = c * q.py - s * q.px;
  q.x = x;
  q.y = y;
  q.px = px;
  q.py = py;
}

// Aperture predicates ("inside"); a NaN coordinate is outside and a particle
// exactly on the boundary is inside.
__device__ __forceinline__ bool in_circle(const Pt& q, double r2) {
  return q.x * q.x + q.y * q.y <= r2;
}
__device__ __forceinline__ bool in_ellipse(const Pt& q, double ia2, double ib2) {
  return q.x * q.x * ia2 + q.y * q.y * ib2 <= 1.0;
}
__device__ __forceinline__ bool in_rect(const Pt& q, double x0, double x1, double y0, double y1) {
  return (x0 <= q.x) & (q.x <= x1) & (y0 <= q.y) & (q.y <= y1);
}

// ------------------------------------------------------------------ RNG
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 128-bit counter, 64-bit
// key, ten rounds of two 32x32->64 multiplications whose halves are mixed
// with the other words and the key; the key advances by the Weyl increments
// floor(2^32 (golden ratio - 1)) and floor(2^32 (sqrt(3) - 1)) between rounds.
struct U4 {
  unsigned int a, b, c, d;
};

__device__ __forceinline__ U4 philox4x32_10(U4 ctr, unsigned int k0, unsigned int k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const unsigned int h0 = __umulhi(0xD2511F53u, ctr.a), l0 = 0xD2511F53u * ctr.a;
    const unsigned int h1 = __umulhi(0xCD9E8D57u, ctr.c), l1 = 0xCD9E8D57u * ctr.c;
    U4 n;
    n.a = h1 ^ ctr.b ^ k0;
    n.b = l1;
    n.c = h0 ^ ctr.d ^ k1;
    n.d = l0;
    ctr = n;
  }
  return ctr;
}

// Uniform in (0,1), exact in binary64: k = (wa << 20) | (wb >> 12), u = (k + 1/2) 2^-52.
__device__ __forceinline__ double uniform52(unsigned int wa, unsigned int wb) {
  const unsigned long long k = ((unsigned long long)wa << 20) | (unsigned long long)(wb >> 12);
  return ((double)k + 0.5) * 0x1p-52;
}

// Standard normal of (seed, particle id, turn, element, draw) by Box-Muller
// on one Philox block with counter (pid_lo, pid_hi, turn, element * 8 + draw).
__device__ __forceinline__ double gauss_at(unsigned long long seed, long long pid, int turn,
                                           int element, int draw) {
  U4 c;
  c.a = (unsigned int)(unsigned long long)pid;
  c.b = (unsigned int)((unsigned long long)pid >> 32);
  c.c = (unsigned int)turn;
  c.d = (unsigned int)element * 8u + (unsigned int)draw;
  const U4 w = philox4x32_10(c, (unsigned int)seed, (unsigned int)(seed >> 32));
  const double u1 = uniform52(w.a, w.b), u2 = uniform52(w.c, w.d);
  return sqrt(-2.0 * xlog(u1)) * xcos(6.283185307179586 * u2);
}

__device__ __attribute__((noinline)) double gauss_at_far(unsigned long long seed, long long pid,
                                                         int turn, int element, int draw) {
  return gauss_at(seed, pid, turn, element, draw);
}

// ------------------------------------------------------------ radiation
// Radiation in a thin multipole of radiation length Lr > 0, after its kick
// (kx, ky = field kick): h = |k| rpp / Lr, gamma = gamma0 (1 + beta0 ptau),
// mean loss dE = c_mean gamma^4 h^2 Lr with c_mean = (2/3) r m;
// quantum (mode 2): dE += sqrt(c_quant gamma^7 |h|^3 Lr) g, c_quant =
// 55/(24 sqrt 3) r m hbar_c; ptau -= dE/p0c, delta from ptau, and the
// momenta keep their angles: px, py *= (1+delta_new)/(1+delta_old).
struct Rad {
  double gamma0, c_mean, c_quant, p0c;
};

__device__ __forceinline__ void radiate(Pt& q, double kx, double ky, double lr, const Rad& rr,
                                        int mode, double g, double beta0, double two_over_beta0) {
  const double h = sqrt(kx * kx + ky * ky) * q.rpp / lr;
  const double gam = rr.gamma0 * (1.0 + q.bpt);
  const double g2 = gam * gam;
  const double g4 = g2 * g2;
  double de = rr.c_mean * g4 * h * h * lr;
  if (mode == 2) {
    const double g7 = g4 * g2 * gam;
    const double var = rr.c_quant * g7 * h * h * h * lr;
    de = de + sqrt(var) * g;
  }
  const double opd_old = 1.0 + q.delta;
  q.ptau = q.ptau - de / rr.p0c;
  from_ptau(q, beta0, two_over_beta0);
  const double f = (1.0 + q.delta) / opd_old;
  q.px = q.px * f;
  q.py = q.py * f;
}

// ------------------------------------------------- photon-by-photon emission
// The quantum model emitted photon by photon: along a radiating multipole
// the photons arrive as a Poisson process of mean count
// nbar = (5 / (2 sqrt 3)) (r m / hbar_c) gamma h Lr (that is alpha q^2 times
// the number of photons per radian of bending, 5/(2 sqrt 3) gamma), each
// with energy x u_c, u_c = (3/2) hbar_c gamma^3 h the critical energy, and x
// distributed as the universal synchrotron photon-number spectrum: the
// probability of x or more is
//   Q(x) = 3/(5 pi) int_0^inf exp(-x cosh t) cosh(5t/3) / cosh^2 t dt.
// Photon j of a kick uses Philox block (pid_lo, pid_hi, turn,
// element * 256 + j): its first uniform is the arrival's exponential
// spacing -ln u (in units of the mean count), its second the energy through
// the inverse of Q.  The inverse is tabulated (host-computed) as
// g(s) = x^(1/3) with Q(x) = exp(-s) at s = i / 64, i = 0 .. 2432, in single
// precision, and interpolated linearly in s; x = g^3.  At most 255 photons
// per kick.
constexpr int kPhotonNodes = 2433;

__device__ __forceinline__ double photon_x(const double* __restrict__ tab, double s) {
  const double v = s * 64.0;
  int i = (int)v;
  i = i < kPhotonNodes - 2 ? i : kPhotonNodes - 2;
  i = i > 0 ? i : 0;
  const double f = v - (double)i;
  const double a = tab[i], b = tab[i + 1];
  const double g = fma(f, b - a, a);
  return g * g * g;
}

__device__ __forceinline__ void radiate_photons(Pt& q, double kx, double ky, double lr,
                                                const double* __restrict__ tab, double c_nphot,
                                                double c_ucrit, double gamma0, double p0c,
                                                unsigned long long seed, long long pid, int turn,
                                                int element, double beta0,
                                                double two_over_beta0) {
  const double h = sqrt(kx * kx + ky * ky) * q.rpp / lr;
  const double gam = gamma0 * (1.0 + q.bpt);
  const double nbar = c_nphot * gam * h * lr;
  U4 c;
  c.a = (unsigned int)(unsigned long long)pid;
  c.b = (unsigned int)((unsigned long long)pid >> 32);
  c.c = (unsigned int)turn;
  double t = 0.0, sum = 0.0;
  for (int j = 0; j < 256; ++j) {
    c.d = (unsigned int)element * 256u + (unsigned int)j;
    const U4 w = philox4x32_10(c, (unsigned int)seed, (unsigned int)(seed >> 32));
    t = t - xlog(uniform52(w.a, w.b));
    if (!(t <= nbar)) break;
    sum = sum + photon_x(tab, -xlog(uniform52(w.c, w.d)));
  }
  if (sum == 0.0) return;
  const double g3 = gam * gam * gam;
  const double de = c_ucrit * g3 * h * sum;
  const double opd_old = 1.0 + q.delta;
  q.ptau = q.ptau - de / p0c;
  from_ptau(q, beta0, two_over_beta0);
  const double f = (1.0 + q.delta) / opd_old;
  q.px = q.px * f;
  q.py = q.py * f;
}

__device__ __attribute__((noinline)) void radiate_photons_far(
    Pt& q, double kx, double ky, double lr, const double* __restrict__ tab, double c_nphot,
    double c_ucrit, double gamma0, double p0c, unsigned long long seed, long long pid, int turn,
    int element, double beta0, double two_over_beta0) {
  radiate_photons(q, kx, ky, lr, tab, c_nphot, c_ucrit, gamma0, p0c, seed, pid, turn, element,
                  beta0, two_over_beta0);
}

// Radiation step of a multipole with radiation length lr (none if lr <= 0 or
// mode 0): mean (1), mean + Gaussian quantum excitation (2), photon by photon
// (3); the deviates are keyed by (seed, particle id, absolute turn, element
// index of the line as tracked, thick elements sliced).  kFar: the deviates'
// and photons' code out of line; kPhotons = false leaves mode 3 out (the
// caller never passes it).
template <bool kFar = false, bool kPhotons = true>
__device__ __forceinline__ void radiate_at(Pt& q, double kx, double ky, double lr, int mode,
                                           unsigned long long seed, long long pid, int turn,
                                           int element, double gamma0, double c_mean,
                                           double c_quant, double p0c, double beta0,
                                           double two_over_beta0, const double* ptab,
                                           double c_nphot, double c_ucrit) {
  if (mode == 0 || !(lr > 0.0)) return;
  if (kPhotons && mode == 3) {
    if (kFar)
      radiate_photons_far(q, kx, ky, lr, ptab, c_nphot, c_ucrit, gamma0, p0c, seed, pid, turn,
                          element, beta0, two_over_beta0);
    else
      radiate_photons(q, kx, ky, lr, ptab, c_nphot, c_ucrit, gamma0, p0c, seed, pid, turn,
                      element, beta0, two_over_beta0);
    return;
  }
  const double g = (mode == 2) ? (kFar ? gauss_at_far(seed, pid, turn, element, 0)
                                        : gauss_at(seed, pid, turn, element, 0))
                               : 0.0;
  Rad rr{gamma0, c_mean, c_quant, p0c};
  radiate(q, kx, ky, lr, rr, mode, g, beta0, two_over_beta0);
}

// Branch-free loss bookkeeping: the first failed check of a live lane
// records code = (turn in chunk) * n_el + element + 1 and the state.
__device__ __forceinline__ void mark(bool ok, int& code, int& st, int enc,
                                     int lost_state) {
  const bool now = (!ok) & (code == 0);
  code = now ? enc : code;
  st = now ? lost_state : st;
}

}  // namespace xtmm
