// Host set-up of the prolate spheroidal taper psi_0(c, x).
//
// The paper (Section 2) divides the image by c, the inverse transform of the
// anti-aliasing kernel C, and (Section 3) takes c separable.  The library uses
// the zeroth prolate spheroidal wave function for c1.  Its expansion in
// normalised Legendre functions Pbar_k = sqrt(k + 1/2) P_k has coefficients
// given by the lowest eigenvector of the prolate operator
//   L psi = -d/dx[(1 - x^2) dpsi/dx] + c^2 x^2 psi,
// which is symmetric tridiagonal on the even degrees k = 0, 2, 4, ...:
//   diagonal     k(k+1) + c^2 (2k(k+1) - 1) / ((2k+3)(2k-1))
//   off-diagonal c^2 (k+1)(k+2) / ((2k+3) sqrt((2k+1)(2k+5)))   (k, k+2)
// The eigenvalue comes from Sturm-sequence bisection, the vector from inverse
// iteration with a shift just below it (the shifted matrix is then positive
// definite, so the tridiagonal LDL^T solve needs no pivoting).  The device
// evaluates the series at the pixel positions (tables.hip).
#include <cmath>
#include <vector>

#include "internal.h"

namespace sepw {

namespace {

// number of eigenvalues of the tridiagonal (d, e) below x
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
  int count = 0;
  double q = d[0] - x;
  if (q < 0) ++count;
  for (size_t j = 1; j < d.size(); ++j) {
    double prev = (q == 0.0) ? 1e-300 : q;
    q = (d[j] - x) - e[j - 1] * e[j - 1] / prev;
    if (q < 0) ++count;
  }
  return count;
}

}  // namespace

int pswf_coefficients(double c, double* out, int max_terms, double* psi_at_0) {
  int m = (int)(2.0 * c + 40.0);
  if (m > max_terms) m = max_terms;
  if (m < 2) m = 2;
  std::vector<double> d(m), e(m - 1);
  for (int j = 0; j < m; ++j) {
    double k = 2.0 * j;
    d[j] = k * (k + 1) + c * c * (2 * k * (k + 1) - 1) / ((2 * k + 3) * (2 * k - 1));
    if (j + 1 < m)
      e[j] = c * c * (k + 1) * (k + 2) / ((2 * k + 3) * std::sqrt((2 * k + 1) * (2 * k + 5)));
  }
  // Gershgorin interval, then bisection for the smallest eigenvalue
  double lo = d[0], hi = d[0];
  for (int j = 0; j < m; ++j) {
    double r = (j > 0 ? std::fabs(e[j - 1]) : 0.0) + (j + 1 < m ? std::fabs(e[j]) : 0.0);
    lo = std::fmin(lo, d[j] - r);
    hi = std::fmax(hi, d[j] + r);
  }
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(d, e, mid) >= 1) hi = mid; else lo = mid;
  }
  double lam = lo;
  double sigma = lam - (1e-12 * std::fabs(lam) + 1e-12);
  // inverse iteration: (A - sigma I) z = b, LDL^T (Thomas) solve
  std::vector<double> z(m, 1.0), piv(m), y(m);
  for (int it = 0; it < 4; ++it) {
    piv[0] = d[0] - sigma;
    y[0] = z[0];
    for (int j = 1; j < m; ++j) {
      double l = e[j - 1] / piv[j - 1];
      piv[j] = (d[j] - sigma) - l * e[j - 1];
      y[j] = z[j] - l * y[j - 1];
    }
    z[m - 1] = y[m - 1] / piv[m - 1];
    for (int j = m - 2; j >= 0; --j) z[j] = (y[j] - e[j] * z[j + 1]) / piv[j];
    double nrm = 0;
    for (int j = 0; j < m; ++j) nrm += z[j] * z[j];
    nrm = std::sqrt(nrm);
    for (int j = 0; j < m; ++j) z[j] /= nrm;
  }
  // psi_0(0) = sum_j z_j Pbar_{2j}(0);  P_{n+1}(0) = -n/(n+1) P_{n-1}(0)
  double p_even = 1.0, psi0 = 0.0;
  for (int j = 0; j < m; ++j) {
    int k = 2 * j;
    if (j > 0) p_even *= -(double)(k - 1) / (double)k;
    psi0 += z[j] * std::sqrt(k + 0.5) * p_even;
  }
  if (psi0 < 0) {
    for (int j = 0; j < m; ++j) z[j] = -z[j];
    psi0 = -psi0;
  }
  for (int j = 0; j < m; ++j) out[j] = z[j];
  *psi_at_0 = psi0;
  return m;
}

}  // namespace sepw
