// xtm_normal6.cpp -- host linear algebra of the 6D linear normal form (paper
// section "Twiss module": the linear normal form from the eigenvalues and
// eigenvectors of the one-turn Jacobian; with radiation the eigenvalues'
// moduli give the damping per turn) and the matched Gaussian ensemble.
//
// Eigenvalues: the real 6x6 Jacobian is reduced to upper Hessenberg form by
// Householder reflections and taken to complex triangular form by QR steps
// with Wilkinson shifts (Givens rotations on the active window, deflation
// when a subdiagonal falls below the rounding of its neighbours).
// Eigenvectors: the null vector of J - lambda I by Gaussian elimination with
// full pivoting (the free unknown set to one).
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>

#include "xtm_internal.h"

namespace xtm {
namespace {

using cplx = std::complex<double>;
using Mat6 = std::array<std::array<double, 6>, 6>;
using CMat6 = std::array<std::array<cplx, 6>, 6>;

// Householder reduction to upper Hessenberg form (similarity transform).
void hessenberg(Mat6& a) {
  for (int k = 0; k < 4; ++k) {
    double norm = 0.0;
    for (int i = k + 1; i < 6; ++i) norm += a[i][k] * a[i][k];
    norm = std::sqrt(norm);
    if (norm == 0.0) continue;
    const double alpha = a[k + 1][k] > 0 ? -norm : norm;
    double v[6] = {0, 0, 0, 0, 0, 0};
    v[k + 1] = a[k + 1][k] - alpha;
    for (int i = k + 2; i < 6; ++i) v[i] = a[i][k];
    double vv = 0.0;
    for (int i = k + 1; i < 6; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    // A <- (I - 2 v v^T / vv) A (I - 2 v v^T / vv)
    for (int j = 0; j < 6; ++j) {
      double d = 0.0;
      for (int i = k + 1; i < 6; ++i) d += v[i] * a[i][j];
      d = 2.0 * d / vv;
      for (int i = k + 1; i < 6; ++i) a[i][j] -= d * v[i];
    }
    for (int i = 0; i < 6; ++i) {
      double d = 0.0;
      for (int j = k + 1; j < 6; ++j) d += a[i][j] * v[j];
      d = 2.0 * d / vv;
      for (int j = k + 1; j < 6; ++j) a[i][j] -= d * v[j];
    }
  }
}

// Eigenvalues of a complex upper Hessenberg matrix by shifted QR steps.
bool hessenberg_eigenvalues(CMat6 h, cplx out[6]) {
  int hi = 5, iter = 0;
  while (hi >= 0) {
    if (hi == 0) {
      out[0] = h[0][0];
      break;
    }
    // deflate at the bottom when the last subdiagonal is negligible
    const double scale = std::abs(h[hi][hi]) + std::abs(h[hi - 1][hi - 1]);
    if (std::abs(h[hi][hi - 1]) <= 1e-16 * scale || std::abs(h[hi][hi - 1]) < 1e-300) {
      out[hi] = h[hi][hi];
      --hi;
      iter = 0;
      continue;
    }
    if (++iter > 200) return false;
    // the active window starts after the last negligible subdiagonal
    int lo = hi - 1;
    while (lo > 0) {
      const double sc = std::abs(h[lo][lo]) + std::abs(h[lo - 1][lo - 1]);
      if (std::abs(h[lo][lo - 1]) <= 1e-16 * sc) break;
      --lo;
    }
    // Wilkinson shift: the eigenvalue of the trailing 2x2 nearer h[hi][hi]
    const cplx a = h[hi - 1][hi - 1], b = h[hi - 1][hi], c = h[hi][hi - 1], d = h[hi][hi];
    const cplx tr = a + d, det = a * d - b * c;
    const cplx disc = std::sqrt(tr * tr * 0.25 - det);
    const cplx m1 = tr * 0.5 + disc, m2 = tr * 0.5 - disc;
    cplx mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
    if (iter % 11 == 10) mu += std::abs(h[hi][hi - 1]);  // exceptional shift
    for (int i = lo; i <= hi; ++i) h[i][i] -= mu;
    // QR of the window by Givens rotations, then RQ
    cplx cs[6];
    cplx sn[6];
    for (int k = lo; k < hi; ++k) {
      const cplx x = h[k][k], y = h[k + 1][k];
      const double r = std::sqrt(std::norm(x) + std::norm(y));
      const cplx cc = r > 0 ? x / r : cplx(1.0, 0.0);
      const cplx ss = r > 0 ? y / r : cplx(0.0, 0.0);
      cs[k] = cc;
      sn[k] = ss;
      // rows k, k+1 <- G^H [row k; row k+1], G = [[c, -conj(s)], [s, conj(c)]]
      for (int j = k; j < 6; ++j) {
        const cplx u = h[k][j], v = h[k + 1][j];
        h[k][j] = std::conj(cc) * u + std::conj(ss) * v;
        h[k + 1][j] = -ss * u + cc * v;
      }
    }
    for (int k = lo; k < hi; ++k) {
      const cplx cc = cs[k], ss = sn[k];
      // columns k, k+1 <- [col k, col k+1] G
      for (int i = 0; i <= std::min(k + 2, 5); ++i) {
        const cplx u = h[i][k], v = h[i][k + 1];
        h[i][k] = u * cc + v * ss;
        h[i][k + 1] = -u * std::conj(ss) + v * std::conj(cc);
      }
    }
    for (int i = lo; i <= hi; ++i) h[i][i] += mu;
  }
  return true;
}

// Null vector of J - lambda I (full pivoting; the free unknown is one).
void null_vector(const Mat6& J, cplx lam, cplx v[6]) {
  CMat6 a;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) a[i][j] = cplx(J[i][j], 0.0) - (i == j ? lam : cplx(0.0, 0.0));
  int col[6] = {0, 1, 2, 3, 4, 5};
  for (int k = 0; k < 5; ++k) {
    int pr = k, pc = k;
    double best = -1.0;
    for (int i = k; i < 6; ++i)
      for (int j = k; j < 6; ++j)
        if (std::abs(a[i][j]) > best) {
          best = std::abs(a[i][j]);
          pr = i;
          pc = j;
        }
    std::swap(a[k], a[pr]);
    if (pc != k) {
      for (int i = 0; i < 6; ++i) std::swap(a[i][k], a[i][pc]);
      std::swap(col[k], col[pc]);
    }
    for (int i = k + 1; i < 6; ++i) {
      const cplx f = a[i][k] / a[k][k];
      for (int j = k; j < 6; ++j) a[i][j] -= f * a[k][j];
    }
  }
  cplx x[6];
  x[5] = 1.0;
  for (int k = 4; k >= 0; --k) {
    cplx s = 0.0;
    for (int j = k + 1; j < 6; ++j) s += a[k][j] * x[j];
    x[k] = -s / a[k][k];
  }
  for (int k = 0; k < 6; ++k) v[col[k]] = x[k];
}

// plane p's share Im(conj(v_2p) v_2p+1) of v^H S v / 2i
double share(const cplx v[6], int p) { return std::imag(std::conj(v[2 * p]) * v[2 * p + 1]); }

}  // namespace

bool normal_form6(const double Jrow[36], NormalForm6* out) {
  Mat6 J, H;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) J[i][j] = Jrow[6 * i + j];
  H = J;
  hessenberg(H);
  CMat6 hc;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) hc[i][j] = cplx(H[i][j], 0.0);
  cplx lam[6];
  if (!hessenberg_eigenvalues(hc, lam)) return false;
  // one eigenvalue per conjugate pair: the one whose eigenvector has a
  // positive symplectic norm, scaled to v^H S v = 2i
  cplx keep_lam[6];
  cplx keep_v[6][6];
  int n_keep = 0;
  for (int i = 0; i < 6; ++i) {
    if (std::abs(lam[i].imag()) <= 1e-14 * std::abs(lam[i])) return false;  // real: unstable
    cplx v[6];
    null_vector(J, lam[i], v);
    double n = share(v, 0) + share(v, 1) + share(v, 2);
    if (!(n > 0.0)) continue;
    if (n_keep == 3) return false;
    const double sc = 1.0 / std::sqrt(n);
    for (int c = 0; c < 6; ++c) keep_v[n_keep][c] = v[c] * sc;
    keep_lam[n_keep++] = lam[i];
  }
  if (n_keep != 3) return false;
  // modes to planes: the permutation with the largest summed shares
  int perm[3] = {0, 1, 2}, best_perm[3] = {0, 1, 2};
  double best = -INFINITY;
  do {
    double sum = 0.0;
    for (int k = 0; k < 3; ++k) sum += share(keep_v[perm[k]], k);
    if (sum > best) {
      best = sum;
      std::copy(perm, perm + 3, best_perm);
    }
  } while (std::next_permutation(perm, perm + 3));
  for (int k = 0; k < 3; ++k) {
    const int m = best_perm[k];
    const cplx ph = keep_v[m][2 * k] / std::abs(keep_v[m][2 * k]);
    for (int c = 0; c < 6; ++c) {
      const cplx w = keep_v[m][c] / ph;
      out->v_re[6 * k + c] = w.real();
      out->v_im[6 * k + c] = w.imag();
    }
    const cplx l = keep_lam[m];
    out->lam_re[k] = l.real();
    out->lam_im[k] = l.imag();
    double q = std::atan2(l.imag(), l.real()) / (2.0 * M_PI);
    q -= std::floor(q);
    out->q[k] = q;
    out->damping[k] = -std::log(std::abs(l));
  }
  return true;
}

void matched_gaussian(const NormalForm6& nf, double beta0, const double eps[3],
                      const double* gauss, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i) {
    const double* g = gauss + 6 * i;
    double u[6];
    for (int c = 0; c < 6; ++c) u[c] = nf.co[c];
    for (int k = 0; k < 3; ++k) {
      const double s = std::sqrt(eps[k]);
      const double zr = s * g[2 * k], zi = s * g[2 * k + 1];
      // Re(v z) = Re(v) Re(z) - Im(v) Im(z)
      for (int c = 0; c < 6; ++c) u[c] += nf.v_re[6 * k + c] * zr - nf.v_im[6 * k + c] * zi;
    }
    const double ptau = beta0 * u[5];
    const double w = ptau * (ptau + 2.0 / beta0);
    for (int c = 0; c < 5; ++c) out[6 * i + c] = u[c];
    out[6 * i + 5] = w / (1.0 + std::sqrt(1.0 + w));
  }
}

}  // namespace xtm
