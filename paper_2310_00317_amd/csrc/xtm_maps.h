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

// Exact drift over L: pz = sqrt((1+d)^2 - px^2 - py^2), lp = L/pz,
// x += px lp, y += py lp, zeta += lp ((d(2+d) - px^2 - py^2)/(1+pz) - beta0 ptau).
// Returns false when pz^2 is not positive (or NaN): the particle is lost; the
// arithmetic still runs (producing NaN) so the caller needs no branch.
__device__ __forceinline__ bool drift_exact(Pt& q, double L) {
  const double px2 = q.px * q.px;
  const double py2 = q.py * q.py;
  const double pz2 = q.opd2 - px2 - py2;
  const bool ok = pz2 > 0.0;
  const double pz = sqrt(pz2);
  const double lp = L / pz;
  q.x = fma(q.px, lp, q.x);
  q.y = fma(q.py, lp, q.y);
  const double dz = (q.u - px2 - py2) / (1.0 + pz) - q.bpt;
  q.zeta = fma(lp, dz, q.zeta);
  return ok;
}

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
  const double s = sin(phase - k * q.zeta);
  q.ptau = q.ptau + amp * s;
  from_ptau(q, beta0, two_over_beta0);
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

// Branch-free loss bookkeeping: the first failed check of a live lane
// records code = (turn in chunk) * n_el + element + 1 and the state.
__device__ __forceinline__ void mark(bool ok, int& code, int& st, int enc,
                                     int lost_state) {
  const bool now = (!ok) & (code == 0);
  code = now ? enc : code;
  st = now ? lost_state : st;
}

}  // namespace xtmm
