/*
 * oracle.c -- plain, slow, obviously-correct CPU FP64 reference of the thin
 * lattice tracking path (element-by-element tracking of a particle ensemble
 * through a ring, paper section "Lattice modelling and single particle
 * tracking").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP library; the two agree
 * only on the element-record layout and on the written formulas below.
 *
 * The paper names the elements (drifts, thin multipoles with multipolar
 * errors, RF cavities, tilts and misalignments as reference-frame changes,
 * aperture checks that stop lost particles) but prints no formula.  Each map
 * below is the standard accelerator-physics reading, stated next to it.
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off (every fused multiply-add
 * is an explicit fma() call; everything else is a correctly rounded IEEE op).
 *
 * Coordinates: x, y [m]; px = Px/P0, py = Py/P0; zeta = s - beta0 c t [m];
 * delta = (P - P0)/P0; derived and stored: ptau = (E - E0)/(P0 c),
 * rpp = 1/(1+delta), rvv = beta/beta0.  One species per run (chi = 1).
 *
 * Loss codes: state 1 alive, 0 outside an aperture, -1 imaginary or
 * non-finite longitudinal momentum in a drift (not pz^2 > 0).  On loss at
 * element e of turn t: at_element = e, at_turn = t, coordinates stay as
 * they entered e.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { O_DRIFT = 1, O_DRIFT_EXP = 2, O_MULT = 3, O_RF = 4, O_SHIFT = 5,
       O_SROT = 6, O_AP_CIRC = 7, O_AP_ELL = 8, O_AP_RECT = 9, O_MARKER = 10 };

#define O_MAXORD 10

double oracle_gauss_at(uint64_t seed, int64_t pid, int32_t turn, int32_t element, int32_t draw);

/* element record: same byte layout as the element-description interface */
typedef struct {
  int32_t type, order;
  double length;
  double knl[O_MAXORD + 1], ksl[O_MAXORD + 1];
  double hxl;
  double p[6];
} orc_elem;

typedef struct {
  double *x, *px, *y, *py, *zeta, *delta, *ptau, *rpp, *rvv;
  int32_t *state, *at_element, *at_turn;
  int64_t *pid;
  int64_t n;
} orc_parts;

typedef struct {
  double beta0, gamma0, p0c, mass0, charge0;
} orc_ref;

/* reference quantities: E0 = sqrt(p0c^2 + m^2), gamma0 = E0/m, beta0 = p0c/E0 */
static orc_ref make_ref(const double ref3[3]) {
  orc_ref r;
  r.mass0 = ref3[0];
  r.charge0 = ref3[1];
  r.p0c = ref3[2];
  double e0 = sqrt(r.p0c * r.p0c + r.mass0 * r.mass0);
  r.gamma0 = e0 / r.mass0;
  r.beta0 = r.p0c / e0;
  return r;
}

/* per-particle working copy */
typedef struct {
  double x, px, y, py, zeta, delta, ptau, rpp, rvv;
} orc_pt;

/* ptau from delta without cancellation: u = delta(2+delta),
   ptau = beta0 u / (1 + sqrt(1 + beta0^2 u))  (= sqrt((1+d)^2 + 1/(b0 g0)^2) - 1/b0) */
static void set_from_delta(orc_pt* q, double b0) {
  double u = q->delta * (2.0 + q->delta);
  q->ptau = b0 * u / (1.0 + sqrt(1.0 + b0 * b0 * u));
  q->rpp = 1.0 / (1.0 + q->delta);
  q->rvv = (1.0 + q->delta) / (1.0 + b0 * q->ptau);
}

/* delta from ptau: v = ptau (ptau + 2/beta0) = delta(2+delta),
   delta = v / (1 + sqrt(1 + v)) */
static void set_from_ptau(orc_pt* q, double b0) {
  double v = q->ptau * (q->ptau + 2.0 / b0);
  q->delta = v / (1.0 + sqrt(1.0 + v));
  q->rpp = 1.0 / (1.0 + q->delta);
  q->rvv = (1.0 + q->delta) / (1.0 + b0 * q->ptau);
}

/* Exact drift over L: straight flight, path L(1+delta)/pz, and
   dzeta = L - L(1+beta0 ptau)/pz written without cancellation as
   (L/pz) * ( (delta(2+delta) - px^2 - py^2)/(1+pz) - beta0 ptau ),
   with pz = sqrt((1+delta)^2 - px^2 - py^2).  Every quotient and the square
   root are the correctly rounded IEEE operations.  The particle is lost
   (return 0) unless pz^2 > 0: the longitudinal momentum is imaginary
   (or a coordinate is not a number). */
static int drift_exact(orc_pt* q, double L, double b0) {
  double opd = 1.0 + q->delta;
  double px2 = q->px * q->px;
  double py2 = q->py * q->py;
  double pz2 = opd * opd - px2 - py2;
  if (!(pz2 > 0.0)) return 0;
  double pz = sqrt(pz2);
  double lp = L / pz;
  q->x = fma(q->px, lp, q->x);
  q->y = fma(q->py, lp, q->y);
  double u = q->delta * (2.0 + q->delta);
  double dz = (u - px2 - py2) / (1.0 + pz) - b0 * q->ptau;
  q->zeta = fma(lp, dz, q->zeta);
  return 1;
}

/* Expanded drift, exact flow of H = pzeta - (1+delta) + (px^2+py^2)/(2(1+delta)):
   x += L px rpp, y += L py rpp,
   zeta += L [ (delta - beta0 ptau) rpp - (px^2+py^2) rpp^3 (1+beta0 ptau)/2 ]. */
static void drift_expanded(orc_pt* q, double L, double b0) {
  double lr = L * q->rpp;
  q->x = fma(q->px, lr, q->x);
  q->y = fma(q->py, lr, q->y);
  double pp = q->px * q->px + q->py * q->py;
  double r3 = q->rpp * q->rpp * q->rpp;
  double dz = (q->delta - b0 * q->ptau) * q->rpp - 0.5 * pp * r3 * (1.0 + b0 * q->ptau);
  q->zeta = fma(L, dz, q->zeta);
}

/* Thin multipole: dpx - i dpy = - sum_n (knl_n + i ksl_n) (x + i y)^n / n!,
   by Horner from the highest order down, each complex step
   b <- b z + c_n as re = fma(br, x, fma(-bi, y, cr)), im = fma(br, y, fma(bi, x, ci)).
   Curvature hxl (frame bend over the radiation length Lr):
   dpx += hxl (1+delta) - knl0 hxl x / Lr (Lr > 0), dzeta = -hxl x (1+beta0 ptau) rpp.
   sgn = +1 forward, -1 applies the exact inverse (x, y, delta unchanged). */
typedef struct { double cr[O_MAXORD + 1], ci[O_MAXORD + 1]; } orc_coef;

static void multipole_kick(orc_pt* q, const orc_elem* e, const orc_coef* c, double b0, double sgn,
                           double* fkx, double* fky) {
  int N = e->order;
  double br = c->cr[N], bi = c->ci[N];
  for (int n = N - 1; n >= 0; --n) {
    double tr = fma(br, q->x, fma(-bi, q->y, c->cr[n]));
    double ti = fma(br, q->y, fma(bi, q->x, c->ci[n]));
    br = tr;
    bi = ti;
  }
  *fkx = -br; /* field part of the kick, (dpx, dpy) */
  *fky = bi;
  if (sgn > 0) {
    q->px = q->px - br;
    q->py = q->py + bi;
  } else {
    q->px = q->px + br;
    q->py = q->py - bi;
  }
  if (e->hxl != 0.0) {
    double dpx = e->hxl * (1.0 + q->delta);
    if (e->length > 0.0) dpx = dpx - e->knl[0] * e->hxl * q->x / e->length;
    double dz = e->hxl * q->x * (1.0 + b0 * q->ptau) * q->rpp;
    if (sgn > 0) {
      q->px = q->px + dpx;
      q->zeta = q->zeta - dz;
    } else {
      q->px = q->px - dpx;
      q->zeta = q->zeta + dz;
    }
  }
}

/* Elementary functions of the tracking maps (RF sine, Box-Muller logarithm
   and cosine), written from their series so that any two implementations of
   the same steps agree bit for bit (libm's results may differ by an ulp
   between platforms, which chaotic or strongly damped motion amplifies).
   sin/cos: n = nearest integer to x (2/pi); r = x - n pi/2 with pi/2 split
   into P1 = pi/2 rounded to double, P2 = the rest rounded, P3 = what remains,
   each product applied by one fused multiply-add; then the Taylor series of sin and cos in r
   (|r| <= pi/4, truncated after r^17 and r^16: the first omitted terms,
   r^19/19! and r^18/18!, stay below 1e-19 and 2.1e-18, under 0.02 ulp of
   the results near pi/4), Horner in r^2, and the quadrant n mod 4 picks
   +-sin r or +-cos r.
   log: x = m 2^e with m in [sqrt(1/2), sqrt(2)); log m = 2 atanh(s),
   s = (m - 1)/(m + 1), by its series in s^2 up to s^21 (|s| <= 0.1716, so
   the first omitted term 2 s^23/23 stays below 2.2e-19); log x = e ln 2 +
   log m with ln 2 split like pi/2.  Accuracy (checked against libm in the
   tests): within two ulps over the ranges used. */
#define O_2_PI 0.6366197723675814          /* 2/pi rounded to double */
#define O_P1 1.5707963267948966            /* pi/2 rounded to double */
#define O_P2 6.123233995736766e-17          /* pi/2 - O_P1 rounded to double */
#define O_P3 -1.4973849048591698e-33        /* pi/2 - O_P1 - O_P2 */
#define O_LN2_1 0.6931471805599453          /* ln 2 rounded to double */
#define O_LN2_2 2.3190468138462996e-17      /* ln 2 - O_LN2_1 */
#define O_2PI 6.283185307179586             /* 2 pi rounded to double */

static void sincos_reduced(double x, double* sr, double* cr, int64_t* quadrant) {
  double n = rint(x * O_2_PI);
  double r = fma(-n, O_P1, x);
  r = fma(-n, O_P2, r);
  r = fma(-n, O_P3, r);
  double z = r * r;
  /* sin r = r + r z (S1 + z (S2 + ... + z S8)), S_k = (-1)^k / (2k+1)! */
  double ps = 1.0 / 355687428096000.0;
  ps = fma(ps, z, -1.0 / 1307674368000.0);
  ps = fma(ps, z, 1.0 / 6227020800.0);
  ps = fma(ps, z, -1.0 / 39916800.0);
  ps = fma(ps, z, 1.0 / 362880.0);
  ps = fma(ps, z, -1.0 / 5040.0);
  ps = fma(ps, z, 1.0 / 120.0);
  ps = fma(ps, z, -1.0 / 6.0);
  *sr = fma(r * z, ps, r);
  /* cos r = 1 + z (C1 + z (C2 + ...)), C_k = (-1)^k / (2k)! */
  double pc = 1.0 / 20922789888000.0;
  pc = fma(pc, z, -1.0 / 87178291200.0);
  pc = fma(pc, z, 1.0 / 479001600.0);
  pc = fma(pc, z, -1.0 / 3628800.0);
  pc = fma(pc, z, 1.0 / 40320.0);
  pc = fma(pc, z, -1.0 / 720.0);
  pc = fma(pc, z, 1.0 / 24.0);
  pc = fma(pc, z, -1.0 / 2.0);
  *cr = fma(z, pc, 1.0);
  *quadrant = (int64_t)n & 3;
}

double oracle_sin(double x) {
  double sr, cr;
  int64_t q;
  sincos_reduced(x, &sr, &cr, &q);
  return q == 0 ? sr : q == 1 ? cr : q == 2 ? -sr : -cr;
}

double oracle_cos(double x) {
  double sr, cr;
  int64_t q;
  sincos_reduced(x, &sr, &cr, &q);
  return q == 0 ? cr : q == 1 ? -sr : q == 2 ? -cr : sr;
}

double oracle_log(double x) {
  int e;
  double m = frexp(x, &e);
  if (m < 0.70710678118654752440) {
    m = m * 2.0;
    e = e - 1;
  }
  double s = (m - 1.0) / (m + 1.0);
  double z = s * s;
  /* log m = 2 s (1 + z/3 + z^2/5 + ... + z^10/21) */
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
  double t = 2.0 * s;
  double lm = fma(t * z, p, t);
  double de = (double)e;
  return fma(de, O_LN2_1, fma(de, O_LN2_2, lm));
}

/* RF cavity (thin): ptau += (q V / p0c) sin(lag pi/180 - k zeta), k = 2 pi f/(beta0 c);
   then delta, rpp, rvv from ptau.  No transverse kick. */
static void rf_kick(orc_pt* q, const orc_elem* e, const orc_ref* r, double sgn) {
  const double clight = 299792458.0;
  double amp = r->charge0 * e->p[0] / r->p0c;
  double k = 2.0 * M_PI * e->p[1] / (r->beta0 * clight);
  double phi = e->p[2] * M_PI / 180.0;
  double s = oracle_sin(phi - k * q->zeta);
  if (sgn > 0)
    q->ptau = q->ptau + amp * s;
  else
    q->ptau = q->ptau - amp * s;
  set_from_ptau(q, r->beta0);
}

/* Reference-frame rotation by angle t about s:
   (x, y) <- (c x + s y, c y - s x), same for (px, py). */
static void srot(orc_pt* q, double cth, double sth) {
  double x = cth * q->x + sth * q->y;
  double y = cth * q->y - sth * q->x;
  double px = cth * q->px + sth * q->py;
  double py = cth * q->py - sth * q->px;
  q->x = x; q->y = y; q->px = px; q->py = py;
}

/* aperture predicates written as "not inside", so a NaN coordinate is lost;
   a particle exactly on the boundary survives */
static int inside(const orc_pt* q, const orc_elem* e) {
  switch (e->type) {
    case O_AP_CIRC: {
      double r2 = e->p[0] * e->p[0];
      return q->x * q->x + q->y * q->y <= r2;
    }
    case O_AP_ELL: {
      double ia2 = 1.0 / (e->p[0] * e->p[0]);
      double ib2 = 1.0 / (e->p[1] * e->p[1]);
      return q->x * q->x * ia2 + q->y * q->y * ib2 <= 1.0;
    }
    case O_AP_RECT:
      return e->p[0] <= q->x && q->x <= e->p[1] && e->p[2] <= q->y && q->y <= e->p[3];
    default:
      return 1;
  }
}

/* Synchrotron radiation in a thin multipole of radiation length Lr > 0
   (paper section "Synchrotron radiation models and compensation": a "mean"
   model of deterministic energy loss and a "quantum" model with
   fluctuations; here the quantum part is the Gaussian diffusion limit).
   Curvature from the field kick h = |(dpx, dpy)| rpp / Lr; gamma = gamma0 (1 + beta0 ptau);
   mean loss dE = (2/3) r m gamma^4 h^2 Lr [eV];
   quantum:  dE += sqrt((55/(24 sqrt 3)) r m hbar_c gamma^7 |h|^3 Lr) g,  g ~ N(0,1)
   (r = classical radius of the species, m its rest energy [eV]);
   ptau -= dE/p0c; delta, rpp, rvv from ptau; px, py scaled by (1+delta_new)/(1+delta_old). */
#define O_R_ELECTRON 2.8179403262e-15
#define O_M_ELECTRON_EV 0.51099895000e6
#define O_HBAR_C_EVM 197.3269804e-9

static void radiate_photons(orc_pt* q, double fkx, double fky, double Lr, const orc_ref* r,
                            uint64_t seed, int64_t pid, int32_t turn, int32_t element);

static void radiate(orc_pt* q, double fkx, double fky, double Lr, const orc_ref* r, int mode,
                    double g) {
  double rclass = O_R_ELECTRON * (O_M_ELECTRON_EV / r->mass0) * r->charge0 * r->charge0;
  double h = sqrt(fkx * fkx + fky * fky) * q->rpp / Lr;
  double gam = r->gamma0 * (1.0 + r->beta0 * q->ptau);
  double g2 = gam * gam;
  double g4 = g2 * g2;
  double dE = (2.0 / 3.0) * rclass * r->mass0 * g4 * h * h * Lr;
  if (mode == 2) {
    double g7 = g4 * g2 * gam;
    double var = 55.0 / (24.0 * sqrt(3.0)) * rclass * r->mass0 * O_HBAR_C_EVM * g7 * h * h * h * Lr;
    dE = dE + sqrt(var) * g;
  }
  double opd_old = 1.0 + q->delta;
  q->ptau = q->ptau - dE / r->p0c;
  set_from_ptau(q, r->beta0);
  double f = (1.0 + q->delta) / opd_old;
  q->px = q->px * f;
  q->py = q->py * f;
}

/* c_n = (knl_n + i ksl_n) / n!  (n! as an exact double) */
static orc_coef* build_coefs(const orc_elem* el, int n_el) {
  orc_coef* c = (orc_coef*)calloc((size_t)(n_el > 0 ? n_el : 1), sizeof(orc_coef));
  for (int i = 0; i < n_el; ++i) {
    double fact = 1.0;
    for (int n = 0; n <= O_MAXORD; ++n) {
      if (n > 0) fact *= (double)n;
      c[i].cr[n] = el[i].knl[n] / fact;
      c[i].ci[n] = el[i].ksl[n] / fact;
    }
  }
  return c;
}

static int validate(const orc_elem* el, int n_el) {
  for (int i = 0; i < n_el; ++i) {
    int t = el[i].type;
    if (t < O_DRIFT || t > O_MARKER) return -2;
    if (t == O_MULT && (el[i].order < 0 || el[i].order > O_MAXORD)) return -2;
  }
  return 0;
}

static void load_pt(const orc_parts* P, int64_t i, orc_pt* q) {
  q->x = P->x[i]; q->px = P->px[i]; q->y = P->y[i]; q->py = P->py[i];
  q->zeta = P->zeta[i]; q->delta = P->delta[i]; q->ptau = P->ptau[i];
  q->rpp = P->rpp[i]; q->rvv = P->rvv[i];
}

static void store_pt(const orc_parts* P, int64_t i, const orc_pt* q) {
  P->x[i] = q->x; P->px[i] = q->px; P->y[i] = q->y; P->py[i] = q->py;
  P->zeta[i] = q->zeta; P->delta[i] = q->delta; P->ptau[i] = q->ptau;
  P->rpp[i] = q->rpp; P->rvv[i] = q->rvv;
}

/* apply element e to q; returns new state (1 alive, 0 aperture loss, -1 pz loss) */
static int apply(orc_pt* q, const orc_elem* e, const orc_coef* c, const orc_ref* r, double sgn,
                 double* fkx, double* fky) {
  *fkx = 0.0;
  *fky = 0.0;
  switch (e->type) {
    case O_DRIFT:
      return drift_exact(q, sgn * e->length, r->beta0) ? 1 : -1;
    case O_DRIFT_EXP:
      drift_expanded(q, sgn * e->length, r->beta0);
      return 1;
    case O_MULT:
      multipole_kick(q, e, c, r->beta0, sgn, fkx, fky);
      return 1;
    case O_RF:
      rf_kick(q, e, r, sgn);
      return 1;
    case O_SHIFT:
      q->x = q->x - sgn * e->p[0];
      q->y = q->y - sgn * e->p[1];
      return 1;
    case O_SROT:
      srot(q, cos(e->p[0]), sgn * sin(e->p[0]));
      return 1;
    case O_AP_CIRC:
    case O_AP_ELL:
    case O_AP_RECT:
      return inside(q, e) ? 1 : 0;
    default:
      return 1;
  }
}

/* ---------------------------------------------------------------- API */

/* Particle set-up from (n,6) host coordinates: derived variables from delta,
   state = 1, at_element = at_turn = 0, particle_id = first_id + i. */
int oracle_init(const double* coords6, int64_t n, int64_t first_id, const double ref3[3],
                orc_parts* P) {
  orc_ref r = make_ref(ref3);
  for (int64_t i = 0; i < n; ++i) {
    orc_pt q;
    memset(&q, 0, sizeof q);
    q.x = coords6[6 * i + 0]; q.px = coords6[6 * i + 1];
    q.y = coords6[6 * i + 2]; q.py = coords6[6 * i + 3];
    q.zeta = coords6[6 * i + 4]; q.delta = coords6[6 * i + 5];
    set_from_delta(&q, r.beta0);
    store_pt(P, i, &q);
    P->state[i] = 1;
    P->at_element[i] = 0;
    P->at_turn[i] = 0;
    P->pid[i] = first_id + i;
  }
  return 0;
}

/* Forward tracking for n_turns turns starting at turn t0:
   for t in [t0, t0+n): for e in 0..E-1: if alive apply(e); survivors get at_turn = t+1.
   Returns the number of (particle, element) applications made while alive
   (including the application at which a particle is lost), or < 0 on error. */
int64_t oracle_track_rad(const orc_elem* el, int32_t n_el, const double ref3[3], orc_parts* P,
                         int32_t t0, int32_t n_turns, int32_t nthreads, int32_t radiation,
                         uint64_t seed);

int64_t oracle_track(const orc_elem* el, int32_t n_el, const double ref3[3], orc_parts* P,
                     int32_t t0, int32_t n_turns, int32_t nthreads) {
  return oracle_track_rad(el, n_el, ref3, P, t0, n_turns, nthreads, 0, 0);
}

/* radiation: 0 off, 1 mean, 2 mean + quantum (Gaussian, Philox stream of
   (seed, particle id, turn, element)) */
int64_t oracle_track_rad(const orc_elem* el, int32_t n_el, const double ref3[3], orc_parts* P,
                         int32_t t0, int32_t n_turns, int32_t nthreads, int32_t radiation,
                         uint64_t seed) {
  if (n_turns < 0 || n_el < 0 || radiation < 0 || radiation > 3) return -1;
  if (validate(el, n_el)) return -2;
  orc_ref r = make_ref(ref3);
  orc_coef* c = build_coefs(el, n_el);
  int64_t passes = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : passes)
#endif
  for (int64_t i = 0; i < P->n; ++i) {
    if (P->state[i] != 1) continue;
    orc_pt q;
    load_pt(P, i, &q);
    int st = 1, lost_e = 0, lost_t = 0;
    for (int32_t t = t0; t < t0 + n_turns && st == 1; ++t) {
      for (int32_t e = 0; e < n_el; ++e) {
        ++passes;
        double fkx, fky;
        st = apply(&q, &el[e], &c[e], &r, 1.0, &fkx, &fky);
        if (st == 1 && radiation == 3 && el[e].type == O_MULT && el[e].length > 0.0) {
          radiate_photons(&q, fkx, fky, el[e].length, &r, seed, P->pid[i], t, e);
        } else if (st == 1 && radiation && el[e].type == O_MULT && el[e].length > 0.0) {
          double g = radiation == 2 ? oracle_gauss_at(seed, P->pid[i], t, e, 0) : 0.0;
          radiate(&q, fkx, fky, el[e].length, &r, radiation, g);
        }
        if (st != 1) { /* loss is decided before any coordinate is modified */
          lost_e = e;
          lost_t = t;
          break;
        }
      }
      if (st == 1) P->at_turn[i] = t + 1;
    }
    store_pt(P, i, &q);
    if (st != 1) {
      P->state[i] = st;
      P->at_element[i] = lost_e;
      P->at_turn[i] = lost_t;
    } else {
      P->at_element[i] = 0;
    }
  }
  free(c);
  return passes;
}

/* Backward tracking: turns in reverse, elements E-1..0, each applying its
   inverse (drift -L, kicks subtracted, shift +d, rotation -angle); apertures
   are still checked.  Survivors end with at_turn = t0 - n_turns.  Particles
   lost while going backward record the turn index being undone. */
int64_t oracle_track_backward(const orc_elem* el, int32_t n_el, const double ref3[3],
                              orc_parts* P, int32_t t0, int32_t n_turns, int32_t nthreads) {
  if (n_turns < 0 || n_el < 0) return -1;
  if (validate(el, n_el)) return -2;
  orc_ref r = make_ref(ref3);
  orc_coef* c = build_coefs(el, n_el);
  int64_t passes = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : passes)
#endif
  for (int64_t i = 0; i < P->n; ++i) {
    if (P->state[i] != 1) continue;
    orc_pt q;
    load_pt(P, i, &q);
    int st = 1, lost_e = 0, lost_t = 0;
    for (int32_t t = t0 - 1; t >= t0 - n_turns && st == 1; --t) {
      for (int32_t e = n_el - 1; e >= 0; --e) {
        ++passes;
        double fkx, fky;
        st = apply(&q, &el[e], &c[e], &r, -1.0, &fkx, &fky);
        if (st != 1) {
          lost_e = e;
          lost_t = t;
          break;
        }
      }
      if (st == 1) P->at_turn[i] = t;
    }
    store_pt(P, i, &q);
    if (st != 1) {
      P->state[i] = st;
      P->at_element[i] = lost_e;
      P->at_turn[i] = lost_t;
    }
  }
  free(c);
  return passes;
}

/* Track a single canonical 6-vector u = (x, px, y, py, zeta, pzeta) through
   n_turns turns (no apertures are skipped: a loss returns its state).  Used
   for the central-difference one-turn Jacobian, where the canonical partner of
   zeta is pzeta = ptau/beta0 (delta, rpp, rvv recomputed from ptau). */
int oracle_track_canonical(const orc_elem* el, int32_t n_el, const double ref3[3],
                           double* u6, int32_t n_turns, int32_t radiation) {
  if (validate(el, n_el) || radiation < 0 || radiation > 1) return -2;
  orc_ref r = make_ref(ref3);
  orc_coef* c = build_coefs(el, n_el);
  orc_pt q;
  q.x = u6[0]; q.px = u6[1]; q.y = u6[2]; q.py = u6[3]; q.zeta = u6[4];
  q.ptau = u6[5] * r.beta0;
  set_from_ptau(&q, r.beta0);
  int st = 1;
  for (int32_t t = 0; t < n_turns && st == 1; ++t)
    for (int32_t e = 0; e < n_el && st == 1; ++e) {
      double fkx, fky;
      st = apply(&q, &el[e], &c[e], &r, 1.0, &fkx, &fky);
      if (st == 1 && radiation && el[e].type == O_MULT && el[e].length > 0.0)
        radiate(&q, fkx, fky, el[e].length, &r, 1, 0.0);
    }
  u6[0] = q.x; u6[1] = q.px; u6[2] = q.y; u6[3] = q.py; u6[4] = q.zeta;
  u6[5] = q.ptau / r.beta0;
  free(c);
  return st;
}

/* reference quantities as the oracle computes them: beta0, gamma0 */
void oracle_reference(const double ref3[3], double out2[2]) {
  orc_ref r = make_ref(ref3);
  out2[0] = r.beta0;
  out2[1] = r.gamma0;
}

/* ------------------------------------------------------------------ RNG
 * Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11):
 * a 128-bit counter (c0..c3) and a 64-bit key (k0, k1); each of 10 rounds
 * multiplies c0 and c2 by two fixed odd 32-bit constants, keeps the high and
 * low halves, and mixes them with c1, c3 and the key:
 *   (h0,l0) = M0 * c0, (h1,l1) = M1 * c2,
 *   c <- (h1 ^ c1 ^ k0, l1, h0 ^ c3 ^ k1, l0);
 * between rounds the key advances by the Weyl increments
 * floor(2^32 (golden ratio - 1)) and floor(2^32 (sqrt(3) - 1)).
 */
#define O_PHILOX_M0 0xD2511F53u
#define O_PHILOX_M1 0xCD9E8D57u
#define O_PHILOX_W0 0x9E3779B9u
#define O_PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += O_PHILOX_W0;
      k1 += O_PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)O_PHILOX_M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)O_PHILOX_M1 * (uint64_t)c2;
    uint32_t h0 = (uint32_t)(p0 >> 32), l0 = (uint32_t)p0;
    uint32_t h1 = (uint32_t)(p1 >> 32), l1 = (uint32_t)p1;
    uint32_t n0 = h1 ^ c1 ^ k0;
    uint32_t n2 = h0 ^ c3 ^ k1;
    c0 = n0; c1 = l1; c2 = n2; c3 = l0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* n blocks from consecutive counters: block j uses (ctr0 + j) with carry
   through the 128-bit counter, key = (seed_lo, seed_hi). */
void oracle_philox_stream(uint64_t seed, const uint32_t ctr0[4], int64_t n_blocks, uint32_t* out) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int64_t j = 0; j < n_blocks; ++j) {
    uint32_t c[4];
    uint64_t lo = ((uint64_t)ctr0[1] << 32 | ctr0[0]) + (uint64_t)j;
    uint64_t carry = lo < (uint64_t)j ? 1u : 0u;
    uint64_t hi = ((uint64_t)ctr0[3] << 32 | ctr0[2]) + carry;
    c[0] = (uint32_t)lo; c[1] = (uint32_t)(lo >> 32);
    c[2] = (uint32_t)hi; c[3] = (uint32_t)(hi >> 32);
    oracle_philox4x32_10(c, key, out + 4 * j);
  }
}

/* Uniform in (0,1) from two words: k = (w_a << 20) | (w_b >> 12) (52 bits),
   u = (k + 1/2) 2^-52, exact in binary64. */
double oracle_uniform(uint32_t wa, uint32_t wb) {
  uint64_t k = ((uint64_t)wa << 20) | (uint64_t)(wb >> 12);
  return ((double)k + 0.5) * 0x1p-52;
}

/* Standard normal by Box-Muller from one Philox block:
   u1 from (w0, w1), u2 from (w2, w3); g = sqrt(-2 ln u1) cos(2 pi u2). */
double oracle_gauss(const uint32_t w[4]) {
  double u1 = oracle_uniform(w[0], w[1]);
  double u2 = oracle_uniform(w[2], w[3]);
  return sqrt(-2.0 * oracle_log(u1)) * oracle_cos(O_2PI * u2);
}

/* Gaussian deviate of (seed, particle id, turn, element): counter
   (pid_lo, pid_hi, turn, element * 8 + draw). */
double oracle_gauss_at(uint64_t seed, int64_t pid, int32_t turn, int32_t element, int32_t draw) {
  uint32_t ctr[4] = {(uint32_t)(uint64_t)pid, (uint32_t)((uint64_t)pid >> 32), (uint32_t)turn,
                     (uint32_t)element * 8u + (uint32_t)draw};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  oracle_philox4x32_10(ctr, key, w);
  return oracle_gauss(w);
}

/* ------------------------------------------------ photon-by-photon emission */

/* The quantum model as individual photons (paper section "Synchrotron
   radiation models and compensation").  Along a radiating multipole of
   length Lr a particle with gamma = gamma0 (1 + beta0 ptau) and curvature
   h = |field kick| rpp / Lr emits photons as a Poisson process: the mean
   count is alpha q^2 times 5/(2 sqrt 3) gamma per radian of bending, i.e.
   nbar = 5/(2 sqrt 3) (r m / hbar_c) gamma h Lr (r m / hbar_c = alpha q^2).
   Photon j uses the Philox block of counter (pid_lo, pid_hi, turn,
   element * 256 + j): the uniform of words 0,1 extends the arrival time by an
   exponential spacing, t_j = t_{j-1} - ln u, and the photon exists while
   t_j <= nbar (at most 255 photons); the uniform of words 2,3 gives its
   energy x u_c, u_c = (3/2) hbar_c gamma^3 h, through the sampling table of
   the spectrum's inverse (oracle/photons.py): x = g^3, g interpolated
   linearly at s = -ln u between the tabulated g(i/64).  The photons' total
   energy leaves ptau at once; delta, rpp, rvv follow and px, py keep their
   angles, as in the mean model. */
static double* o_photon_g = NULL;
static int32_t o_photon_n = 0;

int oracle_set_photon_table(const double* g, int32_t n) {
  if (n < 2) return -1;
  double* t = (double*)malloc((size_t)n * sizeof(double));
  if (!t) return -1;
  memcpy(t, g, (size_t)n * sizeof(double));
  free(o_photon_g);
  o_photon_g = t;
  o_photon_n = n;
  return 0;
}

static double photon_energy(double s) {
  double v = s * 64.0;
  int32_t i = (int32_t)v;
  if (i > o_photon_n - 2) i = o_photon_n - 2;
  if (i < 0) i = 0;
  double f = v - (double)i;
  double a = o_photon_g[i], b = o_photon_g[i + 1];
  double g = fma(f, b - a, a);
  return g * g * g;
}

static void radiate_photons(orc_pt* q, double fkx, double fky, double Lr, const orc_ref* r,
                            uint64_t seed, int64_t pid, int32_t turn, int32_t element) {
  double rclass = O_R_ELECTRON * (O_M_ELECTRON_EV / r->mass0) * r->charge0 * r->charge0;
  double h = sqrt(fkx * fkx + fky * fky) * q->rpp / Lr;
  double gam = r->gamma0 * (1.0 + r->beta0 * q->ptau);
  double nbar = 5.0 / (2.0 * sqrt(3.0)) * rclass * r->mass0 / O_HBAR_C_EVM * gam * h * Lr;
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  double t = 0.0, sum = 0.0;
  for (uint32_t j = 0; j < 256u; ++j) {
    uint32_t ctr[4] = {(uint32_t)(uint64_t)pid, (uint32_t)((uint64_t)pid >> 32), (uint32_t)turn,
                       (uint32_t)element * 256u + j};
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    t = t - oracle_log(oracle_uniform(w[0], w[1]));
    if (!(t <= nbar)) break;
    sum = sum + photon_energy(-oracle_log(oracle_uniform(w[2], w[3])));
  }
  if (sum == 0.0) return;
  double g3 = gam * gam * gam;
  double dE = 1.5 * O_HBAR_C_EVM * g3 * h * sum;
  double opd_old = 1.0 + q->delta;
  q->ptau = q->ptau - dE / r->p0c;
  set_from_ptau(q, r->beta0);
  double f = (1.0 + q->delta) / opd_old;
  q->px = q->px * f;
  q->py = q->py * f;
}

/* the four Philox constants as used above: multipliers M0, M1 and the Weyl
   key increments W0, W1 (exposed so tests can check the increments against
   their closed forms) */
void oracle_philox_constants(uint32_t out[4]) {
  out[0] = O_PHILOX_M0;
  out[1] = O_PHILOX_M1;
  out[2] = O_PHILOX_W0;
  out[3] = O_PHILOX_W1;
}

/* ------------------------------------------------ loss-location refinement */

/* Loss-location refinement (paper section "Simulation of beam losses",
   aperture figure: losses localised beyond the per-element aperture checks
   by backtracking each lost particle and testing it against an aperture
   model refined by polygonal interpolation).  The paper gives no steps; the
   reading here:

   Geometry.  s of element e is the summed length of the drifts before it
   (thin elements have none); C = s of the line end.  Each XYShift (x -= dx,
   y -= dy) and SRotation ((x, y) <- (c x + s y, c y - s x)) changes the
   frame of the coordinates after it; G_e maps the coordinates a particle
   has entering element e to the frame of the line start:
   line = A_e u + b_e, G_0 = identity, a shift gives b += A d, a rotation
   gives A <- A R^T.  Each aperture becomes a polygon of M vertices: the
   points where rays from its own origin at angles 2 pi k / M meet its
   boundary (circle r; ellipse 1/sqrt(c^2/a^2 + s^2/b^2); rectangle: the
   nearest side along the ray, which needs the origin inside it), mapped to
   the line frame by G of the aperture.

   Path.  A particle lost on aperture e_L (its stored coordinates are those
   it entered e_L with) is backtracked through the inverse maps of the
   elements after the previous aperture e_P (cyclic: the previous turn's
   last aperture when e_L is the first), then tracked forward again over the
   same elements.  Inside a drift its line-frame position moves on the
   straight segment between the drift's entry and exit points.

   Aperture between e_P and e_L: vertex k is P_k + w (L_k - P_k),
   w = (s - s_P)/(s_L - s_P), with P and L the two polygons.

   Search.  Each drift is cut into K = ceil(length/ds) equal sub-steps; the
   end of each sub-step is tested (even-odd crossing rule against the
   interpolated polygon); the first sub-step whose end lies outside is
   bisected n_bisect times.  s_loss is the outer end of the final interval
   and (x, y) its line-frame position.  A particle whose path never leaves
   the interpolated polygon, or whose backtracking fails, keeps s_L and its
   position at e_L.  Radiation is not undone (the inverse of a radiating
   multipole is its kick alone).

   Rounding.  lerp(a, b, f) = fma(f, b - a, a); G is applied as
   (a11 x + a12 y) + b1; the crossing test compares
   (xj - xi)(py - yi) - (px - xi)(yj - yi) with zero; everything else is one
   correctly rounded operation per written operator.
   tests (optional) receives the number of polygon tests made per particle.
   Returns 0, -1 on bad arguments, -2 on bad elements, -6 when a
   rectangle does not contain its origin. */
typedef struct { double a11, a12, a21, a22, b1, b2; } orc_frame;

static double o_lerp(double a, double b, double f) { return fma(f, b - a, a); }

static void o_to_line(const orc_frame* g, double ux, double uy, double* lx, double* ly) {
  double t1 = g->a11 * ux;
  double t2 = g->a12 * uy;
  double t3 = g->a21 * ux;
  double t4 = g->a22 * uy;
  *lx = (t1 + t2) + g->b1;
  *ly = (t3 + t4) + g->b2;
}

static int o_is_ap(int t) { return t == O_AP_CIRC || t == O_AP_ELL || t == O_AP_RECT; }
static int o_is_drift(int t) { return t == O_DRIFT || t == O_DRIFT_EXP; }

/* even-odd crossing test of (px, py) against polygon P + w (L - P) */
static int o_in_poly(double px, double py, const double* P, const double* Lp, int M, double w) {
  int in = 0;
  for (int k = 0; k < M; ++k) {
    int kn = (k + 1 == M) ? 0 : k + 1;
    double xi = o_lerp(P[2 * k], Lp[2 * k], w);
    double yi = o_lerp(P[2 * k + 1], Lp[2 * k + 1], w);
    double xj = o_lerp(P[2 * kn], Lp[2 * kn], w);
    double yj = o_lerp(P[2 * kn + 1], Lp[2 * kn + 1], w);
    if ((yi > py) != (yj > py)) {
      double t1 = (xj - xi) * (py - yi);
      double t2 = (px - xi) * (yj - yi);
      double cr = t1 - t2;
      if (yj > yi ? cr > 0.0 : cr < 0.0) in = !in;
    }
  }
  return in;
}

int oracle_refine_losses(const orc_elem* el, int32_t n_el, const double ref3[3],
                         const orc_parts* P, int32_t M, double ds, int32_t n_bisect,
                         double* s_out, double* x_out, double* y_out, int32_t* tests) {
  if (n_el <= 0 || M < 4 || !(ds > 0.0) || n_bisect < 0 || n_bisect > 60) return -1;
  if (validate(el, n_el)) return -2;
  orc_ref r = make_ref(ref3);
  orc_coef* c = build_coefs(el, n_el);
  double* s = (double*)malloc(sizeof(double) * (size_t)(n_el + 1));
  orc_frame* G = (orc_frame*)malloc(sizeof(orc_frame) * (size_t)(n_el + 1));
  int32_t* prev = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_el);
  double* poly = (double*)calloc((size_t)n_el * 2 * (size_t)M, sizeof(double));
  int rc = 0;
  /* s positions and frames */
  s[0] = 0.0;
  G[0].a11 = 1.0; G[0].a12 = 0.0; G[0].a21 = 0.0; G[0].a22 = 1.0; G[0].b1 = 0.0; G[0].b2 = 0.0;
  for (int32_t e = 0; e < n_el; ++e) {
    s[e + 1] = o_is_drift(el[e].type) ? s[e] + el[e].length : s[e];
    orc_frame g = G[e];
    if (el[e].type == O_SHIFT) {
      double dx = el[e].p[0], dy = el[e].p[1];
      double t1 = g.a11 * dx, t2 = g.a12 * dy, t3 = g.a21 * dx, t4 = g.a22 * dy;
      g.b1 = (t1 + t2) + g.b1;
      g.b2 = (t3 + t4) + g.b2;
    } else if (el[e].type == O_SROT) {
      double cs = cos(el[e].p[0]), sn = sin(el[e].p[0]);
      double a11 = g.a11 * cs + g.a12 * sn;
      double a12 = g.a12 * cs - g.a11 * sn;
      double a21 = g.a21 * cs + g.a22 * sn;
      double a22 = g.a22 * cs - g.a21 * sn;
      g.a11 = a11; g.a12 = a12; g.a21 = a21; g.a22 = a22;
    }
    G[e + 1] = g;
  }
  const double C = s[n_el];
  /* aperture polygons in the line frame and the previous aperture of each */
  int32_t last_ap = -1;
  for (int32_t e = 0; e < n_el; ++e)
    if (o_is_ap(el[e].type)) last_ap = e;
  for (int32_t e = 0, pa = last_ap; e < n_el; ++e) {
    if (!o_is_ap(el[e].type)) continue;
    prev[e] = pa;
    pa = e;
    const double* p = el[e].p;
    if (el[e].type == O_AP_RECT && !(p[0] < 0.0 && 0.0 < p[1] && p[2] < 0.0 && 0.0 < p[3])) {
      rc = -6;
      goto done;
    }
    for (int32_t k = 0; k < M; ++k) {
      double ang = 2.0 * M_PI * (double)k / (double)M;
      double cs = cos(ang), sn = sin(ang);
      double rad;
      if (el[e].type == O_AP_CIRC) {
        rad = p[0];
      } else if (el[e].type == O_AP_ELL) {
        double q = (cs * cs) / (p[0] * p[0]) + (sn * sn) / (p[1] * p[1]);
        rad = 1.0 / sqrt(q);
      } else {
        rad = INFINITY;
        if (cs > 0.0) rad = fmin(rad, p[1] / cs);
        if (cs < 0.0) rad = fmin(rad, p[0] / cs);
        if (sn > 0.0) rad = fmin(rad, p[3] / sn);
        if (sn < 0.0) rad = fmin(rad, p[2] / sn);
      }
      o_to_line(&G[e], rad * cs, rad * sn, &poly[((size_t)e * M + k) * 2],
                &poly[((size_t)e * M + k) * 2 + 1]);
    }
  }
  for (int64_t i = 0; i < P->n; ++i) {
    s_out[i] = NAN; x_out[i] = NAN; y_out[i] = NAN;
    int32_t nt = 0;
    if (tests) tests[i] = 0;
    int32_t eL = P->at_element[i];
    if (P->state[i] != 0 || eL < 0 || eL >= n_el || !o_is_ap(el[eL].type)) continue;
    int32_t eP = prev[eL];
    double sL = s[eL];
    double sP = eP < eL ? s[eP] : s[eP] - C;
    orc_pt q;
    load_pt(P, i, &q);
    o_to_line(&G[eL], q.x, q.y, &x_out[i], &y_out[i]);
    s_out[i] = sL;
    if (!(sL - sP > 0.0)) continue;
    /* backtrack to the exit of the previous aperture */
    int ok = 1;
    for (int32_t j = (eL + n_el - 1) % n_el; j != eP; j = (j + n_el - 1) % n_el) {
      double fkx, fky;
      if (apply(&q, &el[j], &c[j], &r, -1.0, &fkx, &fky) != 1) { ok = 0; break; }
    }
    if (!ok) continue;
    /* forward again, searching each drift */
    const double* PP = &poly[(size_t)eP * M * 2];
    const double* PL = &poly[(size_t)eL * M * 2];
    double sc = sP;
    for (int32_t j = (eP + 1) % n_el; j != eL; j = (j + 1) % n_el) {
      double fkx, fky;
      if (!o_is_drift(el[j].type)) {
        apply(&q, &el[j], &c[j], &r, 1.0, &fkx, &fky);
        continue;
      }
      double L = el[j].length;
      double v0x, v0y, v1x, v1y;
      o_to_line(&G[j], q.x, q.y, &v0x, &v0y);
      if (apply(&q, &el[j], &c[j], &r, 1.0, &fkx, &fky) != 1) { ok = 0; break; }
      o_to_line(&G[j], q.x, q.y, &v1x, &v1y);
      if (L > 0.0) {
        int64_t K = (int64_t)ceil(L / ds);
        if (K < 1) K = 1;
        int found = 0;
        for (int64_t k = 1; k <= K && !found; ++k) {
          double f = (double)k / (double)K;
          double sf = sc + L * f;
          double w = (sf - sP) / (sL - sP);
          ++nt;
          if (tests) tests[i] = nt;
          if (o_in_poly(o_lerp(v0x, v1x, f), o_lerp(v0y, v1y, f), PP, PL, M, w)) continue;
          double lo = (double)(k - 1) / (double)K, hi = f;
          for (int32_t b = 0; b < n_bisect; ++b) {
            double m = 0.5 * (lo + hi);
            double sm = sc + L * m;
            double wm = (sm - sP) / (sL - sP);
            ++nt;
            if (tests) tests[i] = nt;
            if (o_in_poly(o_lerp(v0x, v1x, m), o_lerp(v0y, v1y, m), PP, PL, M, wm))
              lo = m;
            else
              hi = m;
          }
          s_out[i] = sc + L * hi;
          x_out[i] = o_lerp(v0x, v1x, hi);
          y_out[i] = o_lerp(v0y, v1y, hi);
          found = 1;
        }
        if (found) break;
      }
      sc = sc + L;
    }
  }
done:
  free(c); free(s); free(G); free(prev); free(poly);
  return rc;
}

/* ------------------------------------------------------ optics by tracking */

/* One turn of n particles from the line start with the coordinates
   (x, px, y, py, zeta, delta) recorded at the entry of every element and
   after the last: out[(e n + i) 6 + c], e = 0..n_el.  Apertures are not
   checked (the optics of the bare lattice, paper section "Twiss module");
   a particle whose drift leaves the longitudinal-momentum window keeps the
   coordinates it entered that drift with.  Set-up as oracle_init. */
int oracle_track_record(const orc_elem* el, int32_t n_el, const double ref3[3],
                        const double* coords6, int64_t n, double* out) {
  if (n_el < 0 || n < 0) return -1;
  if (validate(el, n_el)) return -2;
  orc_ref r = make_ref(ref3);
  orc_coef* c = build_coefs(el, n_el);
  for (int64_t i = 0; i < n; ++i) {
    orc_pt q;
    memset(&q, 0, sizeof q);
    q.x = coords6[6 * i + 0]; q.px = coords6[6 * i + 1];
    q.y = coords6[6 * i + 2]; q.py = coords6[6 * i + 3];
    q.zeta = coords6[6 * i + 4]; q.delta = coords6[6 * i + 5];
    set_from_delta(&q, r.beta0);
    int alive = 1;
    for (int32_t e = 0; e <= n_el; ++e) {
      double* o = out + ((size_t)e * (size_t)n + (size_t)i) * 6;
      o[0] = q.x; o[1] = q.px; o[2] = q.y; o[3] = q.py; o[4] = q.zeta; o[5] = q.delta;
      if (e == n_el || !alive || el[e].type == O_AP_CIRC || el[e].type == O_AP_ELL ||
          el[e].type == O_AP_RECT)
        continue;
      orc_pt q0 = q;
      double fkx, fky;
      if (apply(&q, &el[e], &c[e], &r, 1.0, &fkx, &fky) != 1) {
        q = q0;
        alive = 0;
      }
    }
  }
  free(c);
  return 0;
}
