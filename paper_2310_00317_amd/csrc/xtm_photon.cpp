// xtm_photon.cpp -- inverse of the synchrotron photon-number spectrum for the
// photon-by-photon radiation model (paper section "Synchrotron radiation
// models and compensation": the quantum model emits individual photons).
//
// A photon of a particle bending with curvature h has energy x u_c, u_c =
// (3/2) hbar_c gamma^3 h, with x distributed as the universal spectrum whose
// photon-number density is n(x) = 3/(5 pi) int_x^inf K_{5/3}(t) dt.  With
// K_nu(t) = int_0^inf exp(-t cosh a) cosh(nu a) da, integrating over t gives
// closed one-dimensional integrals for the density, the tail and the head:
//   n(x) = 3/(5 pi) int_0^inf exp(-x cosh a) cosh(5a/3) / cosh a da
//   Q(x) = P(X > x)  = 3/(5 pi) int_0^inf exp(-x cosh a) cosh(5a/3) / cosh^2 a da
//   F(x) = P(X <= x) = 3/(5 pi) int_0^inf (1 - exp(-x cosh a)) cosh(5a/3) / cosh^2 a da
// (Q(0) = 1 since int_0^inf cosh(5a/3)/cosh^2 a da = 5 pi / 3).  The
// integrands are even and analytic in the strip |Im a| < pi/2, so the
// trapezoidal rule converges geometrically; a step of 1/12 on [0, 130]
// leaves an error far below double rounding.
//
// The table holds g(s) = x^(1/3) with Q(x) = exp(-s) at s = i / 64, found by
// Newton's method in y = x^(1/3) (on F(y^3) = 1 - exp(-s) while s <= ln 2,
// on ln Q(y^3) = -s beyond), each value rounded to single precision.
#include <cmath>
#include <mutex>
#include <vector>

#include "xtm_internal.h"

namespace xtm {
namespace {

struct SpectrumSums {
  std::vector<double> ch, wb;  // cosh a_k, trapezoid weight x cosh(5 a_k/3) / cosh^2 a_k
  SpectrumSums() {
    const double h = 1.0 / 12.0;
    for (int k = 0; k * h <= 130.0; ++k) {
      const double a = k * h, c = std::cosh(a);
      ch.push_back(c);
      wb.push_back((k == 0 ? 0.5 * h : h) * std::cosh(5.0 * a / 3.0) / (c * c));
    }
  }
  // 5 pi / 3 times Q(x), F(x) and n(x)
  void eval(double x, long double* q, long double* f, long double* d) const {
    long double sq = 0, sf = 0, sd = 0;
    for (size_t k = 0; k < ch.size(); ++k) {
      const double xc = x * ch[k];
      const double e = xc < 745.0 ? std::exp(-xc) : 0.0;
      sq += (long double)wb[k] * e;
      sd += (long double)wb[k] * e * ch[k];
      sf += (long double)wb[k] * -std::expm1(-xc);
    }
    *q = sq;
    *f = sf;
    *d = sd;
  }
};

std::vector<double> build_photon_table() {
  const SpectrumSums sp;
  const long double norm = 3.0L / (5.0L * 3.141592653589793238462643383279502884L);
  std::vector<double> g(kPhotonTableNodes, 0.0);
  double y = 0.0;
  for (int i = 1; i < kPhotonTableNodes; ++i) {
    const double s = i / 64.0;
    // first node from the small-x law F(x) ~ 1.2315 x^(1/3); then the
    // previous node's root
    if (i == 1) y = s / 1.2315;
    double last = INFINITY;
    for (int it = 0; it < 60; ++it) {
      long double q, f, d;
      sp.eval(y * y * y, &q, &f, &d);
      q *= norm;
      f *= norm;
      d *= norm;
      long double phi, dphi;
      if (s <= 0.6931471805599453) {
        phi = f + std::expm1((long double)-s);
        dphi = d * 3.0L * y * y;
      } else {
        phi = std::log(q) + s;
        dphi = -d / q * 3.0L * y * y;
      }
      const double step = (double)(-phi / dphi);
      const double yn = y + step > 0.0 ? y + step : 0.5 * y;
      const double size = std::fabs(yn - y);
      y = yn;
      if (size <= 1e-17 * y || size >= last) break;
      last = size;
    }
    g[i] = (double)(float)y;
  }
  return g;
}

std::once_flag g_table_once;
std::vector<double>* g_table = nullptr;

}  // namespace

const std::vector<double>& photon_table_host() {
  std::call_once(g_table_once, [] { g_table = new std::vector<double>(build_photon_table()); });
  return *g_table;
}

}  // namespace xtm
