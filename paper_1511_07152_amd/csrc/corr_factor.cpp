// The correction table F_w - F~_w (Section 6) as a short sum of separable
// terms, so that the correction runs on the separable matrix-core kernels.
//
// For plane k, arrange the table as the matrix
//     M_k[(fu, su)][(fv, sv)] = C[k][fu][fv][sv][su]
// (rows: coarse u sub-cell and u tap, columns: the same for v).  Every block
// (fu, fv) of it is a 2D transform of the same image-domain function
// c1(l) c1(m) [exp(2 pi i w (n - 1)) - g(l) g(m)], whose exponent gap is a
// short polynomial in l^2 and m^2 (the cross term l^2 m^2 and the fourth-power
// terms the separable screen misses), so M_k has a small numerical rank that
// holds across all sub-cells at once:
//     M_k = sum_r a_r b_r^T,   a_r indexed by (fu, su), b_r by (fv, sv),
// i.e. C[k][fu][fv] = sum_r a_r[fu] (x) b_r[fv]: term r is a separable kernel
// whose u taps depend on the u sub-cell only and whose v taps on the v
// sub-cell only.  The terms come from cross approximation with complete
// pivoting (take the largest residual entry, subtract the outer product of its
// row and column), which stops once every residual entry is within tol of the
// table's largest entry; the check is on the residual itself, so the result
// holds whatever the pivots.
//
// When the two axes share their screen coefficients M_k is complex symmetric
// (M_k = M_k^T), and symmetric elimination (pivot on the largest diagonal
// residual entry d, term a = column / sqrt(d), subtract a a^T) gives terms
// with b_r = a_r: the u and v tables of a term are then one table, which the
// kernels stage in LDS like the separable pair.  It is used only when every
// pivot is at least a tenth of the largest residual entry (else the general
// form), and its residual is checked against the table as above.
//
// Each term is then written as a pair of ordinary tables on the separable
// lattice ([P][O][S], the visibility's own sub-cell f in 1/O): the row of f
// holds the S_c taps of the coarse sample the correction uses for f (the
// 1/O_c lattice point nearest to f, ties up, possibly in the next cell) at
// the S-tap positions that sample covers, and zeros elsewhere.  Gridding and
// degridding with those tables then add exactly term r of the correction.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "internal.h"

namespace sepw {

namespace {

typedef std::complex<double> cd;

// Coarse sample of sub-cell f (0 <= f < O) on the 1/Oc lattice: its sub-cell
// fc and whether it lies in the next cell (t = f - O/2, r = O/Oc,
// g = floor((t + floor(r/2)) / r) in [-Oc/2, Oc/2]).
void coarse(int f, int O, int Oc, int* fc, int* next) {
  const int r = O / Oc, t = f - O / 2;
  const int num = t + r / 2;
  const int g = num >= 0 ? num / r : -((-num + r - 1) / r);
  *next = g + Oc / 2 >= Oc ? 1 : 0;
  *fc = g + Oc / 2 - *next * Oc;
}

// Terms of one plane's matrix R (m x m, row-major) until every residual
// entry is within tol: appends a_r, b_r to fa, fb and returns the count, or
// -1 (more than max_rank terms, a non-finite entry, or in the symmetric form
// a pivot below a tenth of the largest residual entry).
int factor_plane(std::vector<cd> R, int m, bool sym, int max_rank, double tol, std::vector<cd>* fa,
                 std::vector<cd>* fb) {
  int r = 0;
  while (true) {
    size_t best = 0;
    double bmax = -1.0;
    for (size_t i = 0; i < R.size(); ++i) {
      const double v = std::abs(R[i]);
      if (v > bmax) {
        bmax = v;
        best = i;
      }
    }
    if (!std::isfinite(bmax)) return -1;
    if (!(bmax > tol)) return r;              // converged (also for an all-zero plane)
    if (r == max_rank) return -1;
    std::vector<cd> a(m), b(m);
    if (sym) {
      int pd = 0;
      for (int i = 1; i < m; ++i)
        if (std::abs(R[(size_t)i * m + i]) > std::abs(R[(size_t)pd * m + pd])) pd = i;
      const cd d = R[(size_t)pd * m + pd];
      if (std::abs(d) < 0.1 * bmax) return -1;
      const cd q = std::sqrt(d);
      for (int i = 0; i < m; ++i) a[i] = b[i] = R[(size_t)i * m + pd] / q;
    } else {
      const int pi = (int)(best / m), pj = (int)(best % m);
      const cd piv = R[best];
      for (int i = 0; i < m; ++i) a[i] = R[(size_t)i * m + pj];
      for (int j = 0; j < m; ++j) b[j] = R[(size_t)pi * m + j] / piv;
    }
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) R[(size_t)i * m + j] -= a[i] * b[j];
    fa->insert(fa->end(), a.begin(), a.end());
    fb->insert(fb->end(), b.begin(), b.end());
    ++r;
  }
}

}  // namespace

int factor_corr_table(const float2* C, int P, int O, int S, int Oc, int Sc, int max_rank,
                      double tol_rel, std::vector<float2>* tu, std::vector<float2>* tv,
                      bool* shared) {
  const int m = Oc * Sc;
  const int64_t nC = (int64_t)P * Oc * Oc * Sc * Sc;
  double cmax = 0.0;
  for (int64_t i = 0; i < nC; ++i) cmax = std::max(cmax, (double)std::hypot(C[i].x, C[i].y));
  const double tol = tol_rel * cmax;
  std::vector<std::vector<cd>> M(P, std::vector<cd>((size_t)m * m));
  bool sym = true;
  for (int k = 0; k < P; ++k) {
    std::vector<cd>& A = M[k];
    for (int fu = 0; fu < Oc; ++fu)
      for (int fv = 0; fv < Oc; ++fv)
        for (int sv = 0; sv < Sc; ++sv)
          for (int su = 0; su < Sc; ++su) {
            const float2 c = C[(((int64_t)k * Oc + fu) * Oc + fv) * Sc * Sc + sv * Sc + su];
            A[(size_t)(fu * Sc + su) * m + fv * Sc + sv] = cd(c.x, c.y);
          }
    for (int i = 0; i < m && sym; ++i)
      for (int j = 0; j < i && sym; ++j)
        sym = std::abs(A[(size_t)i * m + j] - A[(size_t)j * m + i]) <= 0.5 * tol;
  }
  // per plane: factors a_r (length m, index fu Sc + su) and b_r (fv Sc + sv);
  // symmetric terms leave half the tolerance to the asymmetry
  std::vector<std::vector<cd>> fa(P), fb(P);
  std::vector<int> rank(P, 0);
  *shared = sym;
  for (int k = 0; k < P && *shared; ++k) {
    rank[k] = factor_plane(M[k], m, true, max_rank, 0.5 * tol, &fa[k], &fb[k]);
    if (rank[k] < 0) *shared = false;
  }
  if (!*shared)
    for (int k = 0; k < P; ++k) {
      fa[k].clear();
      fb[k].clear();
      rank[k] = factor_plane(M[k], m, false, max_rank, tol, &fa[k], &fb[k]);
      if (rank[k] < 0) return -1;
    }
  int rmax = 0;
  for (int k = 0; k < P; ++k) rmax = std::max(rmax, rank[k]);
  // term tables on the separable lattice, zero for planes of lower rank
  const int H = S / 2, hc = Sc / 2;
  const size_t one = (size_t)P * O * S;
  tu->assign((size_t)rmax * one, make_float2(0.f, 0.f));
  tv->assign((size_t)rmax * one, make_float2(0.f, 0.f));
  for (int k = 0; k < P; ++k)
    for (int r = 0; r < rank[k]; ++r)
      for (int f = 0; f < O; ++f) {
        int fc = 0, next = 0;
        coarse(f, O, Oc, &fc, &next);
        const int base = H + next - hc;   // S-tap position of coarse tap 0
        float2* ru = tu->data() + (size_t)r * one + ((size_t)k * O + f) * S;
        float2* rv = tv->data() + (size_t)r * one + ((size_t)k * O + f) * S;
        for (int s = 0; s < Sc; ++s) {
          const cd a = fa[k][(size_t)r * m + fc * Sc + s];
          const cd b = fb[k][(size_t)r * m + fc * Sc + s];
          ru[base + s] = make_float2((float)a.real(), (float)a.imag());
          rv[base + s] = make_float2((float)b.real(), (float)b.imag());
        }
      }
  return rmax;
}

}  // namespace sepw
