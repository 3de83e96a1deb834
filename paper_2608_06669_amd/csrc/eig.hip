// Explicitly shifted QR iteration in complex arithmetic (Golub & Van Loan,
// Matrix Computations, the shifted QR algorithm on Hessenberg matrices):
// on the active unreduced block, A - mu I = QR by Givens rotations and
// A <- RQ + mu I, with the Wilkinson shift (the eigenvalue of the trailing
// 2 x 2 block nearer its last diagonal entry) and an occasional ad hoc
// shift against cycling; a subdiagonal entry below eps times its diagonal
// neighbours is set to zero and the block splits. Complex arithmetic lets
// the conjugate pairs of a real matrix come out one at a time.
#include "eig.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <limits>
#include <vector>

namespace pnk {

bool hessenberg_eigenvalues(const double* H, int m, double* re, double* im) {
  using C = std::complex<double>;
  if (m <= 0) return true;
  std::vector<C> a((size_t)m * m);
  double anorm = 0.0;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      const double x = j >= i - 1 ? H[(size_t)i * m + j] : 0.0;
      a[(size_t)i * m + j] = x;
      anorm += std::fabs(x);
    }
  auto A = [&](int i, int j) -> C& { return a[(size_t)i * m + j]; };
  std::vector<C> eig(m), cs(m), sn(m);
  const double eps = std::numeric_limits<double>::epsilon();
  int hi = m - 1, iter = 0;
  while (hi >= 0) {
    // the unreduced block [lo, hi]
    int lo = hi;
    while (lo > 0) {
      double s = std::abs(A(lo, lo)) + std::abs(A(lo - 1, lo - 1));
      if (s == 0.0) s = anorm;
      if (std::abs(A(lo, lo - 1)) <= eps * s) {
        A(lo, lo - 1) = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {
      eig[hi] = A(hi, hi);
      --hi;
      iter = 0;
      continue;
    }
    if (++iter > 60 * m + 100) return false;
    const C p = A(hi - 1, hi - 1), q = A(hi - 1, hi), r = A(hi, hi - 1), d = A(hi, hi);
    const C half = 0.5 * (p + d);
    const C disc = std::sqrt(half * half - (p * d - q * r));
    const C l1 = half + disc, l2 = half - disc;
    C mu = std::abs(l1 - d) < std::abs(l2 - d) ? l1 : l2;
    if (iter % 11 == 10) mu = d + 0.75 * std::abs(r);  // ad hoc shift
    for (int k = lo; k <= hi; ++k) A(k, k) -= mu;
    // A - mu I = Q R: G_k = [conj(c) conj(s); -s c] zeroes the subdiagonal
    for (int k = lo; k < hi; ++k) {
      const C x = A(k, k), y = A(k + 1, k);
      const double rr = std::hypot(std::abs(x), std::abs(y));
      const C c = rr == 0.0 ? C(1.0) : x / rr, s = rr == 0.0 ? C(0.0) : y / rr;
      for (int j = k; j <= hi; ++j) {
        const C u = A(k, j), v = A(k + 1, j);
        A(k, j) = std::conj(c) * u + std::conj(s) * v;
        A(k + 1, j) = -s * u + c * v;
      }
      cs[k] = c;
      sn[k] = s;
    }
    // R Q: the adjoints from the right, in order
    for (int k = lo; k < hi; ++k) {
      const C c = cs[k], s = sn[k];
      for (int i = lo; i <= std::min(k + 1, hi); ++i) {
        const C u = A(i, k), v = A(i, k + 1);
        A(i, k) = u * c + v * s;
        A(i, k + 1) = -u * std::conj(s) + v * std::conj(c);
      }
    }
    for (int k = lo; k <= hi; ++k) A(k, k) += mu;
  }
  for (int i = 0; i < m; ++i) {
    re[i] = eig[i].real();
    im[i] = eig[i].imag();
  }
  return true;
}

}  // namespace pnk
