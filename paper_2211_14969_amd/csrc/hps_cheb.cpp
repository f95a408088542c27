// Chebyshev extreme points and the spectral differentiation matrix on
// [-1, 1] (host side, FP64).  Sec. 2 of the paper puts a p x p tensor grid of
// Chebyshev points on every leaf and differentiates spectrally; the points
// must include the interval ends so that the leaf edges carry nodes.
//
// t_k = -cos(pi k/(p-1)), k = 0..p-1 (increasing).  The first-derivative
// matrix of the degree-(p-1) interpolant is, with weights w_0 = w_{p-1} = 2
// and w_k = 1 otherwise, D[k][l] = (w_k/w_l)(-1)^(k+l)/(t_k - t_l) for
// k != l, and each diagonal entry is minus the sum of the rest of its row
// (so D maps constants to zero).  The second derivative is D*D, formed in
// extended precision and rounded once.
//
// Corner weights (for operators with a mixed term, whose interior rows reach
// the leaf corners): E[0][q] and E[1][q], q = 0..p-3, evaluate at t = -1 and
// t = +1 the degree-(p-3) polynomial through the values at the p-2 interior
// points t_1..t_{p-2} (Lagrange basis of those points).
#include <cmath>
#include <vector>

#include "hps_internal.h"

namespace hps {

void cheb_tables(int p, double *t, double *D, double *D2, double *E) {
  const int n = p - 1;
  const long double pi = 3.141592653589793238462643383279502884L;
  // sin form: exactly antisymmetric about the midpoint
  for (int k = 0; k < p; ++k)
    t[k] = (double)std::sin(pi * (long double)(2 * k - n) / (2.0L * (long double)n));
  std::vector<long double> Dl((size_t)p * p, 0.0L);
  for (int k = 0; k < p; ++k) {
    long double rowsum = 0.0L;
    const long double wk = (k == 0 || k == n) ? 2.0L : 1.0L;
    for (int l = 0; l < p; ++l) {
      if (l == k) continue;
      const long double wl = (l == 0 || l == n) ? 2.0L : 1.0L;
      const long double sgn = ((k + l) & 1) ? -1.0L : 1.0L;
      const long double v = (wk / wl) * sgn / ((long double)t[k] - (long double)t[l]);
      Dl[(size_t)k * p + l] = v;
      rowsum += v;
    }
    Dl[(size_t)k * p + k] = -rowsum;
  }
  for (int k = 0; k < p; ++k)
    for (int l = 0; l < p; ++l) D[(size_t)k * p + l] = (double)Dl[(size_t)k * p + l];
  for (int k = 0; k < p; ++k)
    for (int l = 0; l < p; ++l) {
      long double acc = 0.0L;
      for (int q = 0; q < p; ++q) acc += Dl[(size_t)k * p + q] * Dl[(size_t)q * p + l];
      D2[(size_t)k * p + l] = (double)acc;
    }
  const int m = p - 2;
  for (int q = 0; q < m; ++q) {
    long double lo = 1.0L, hi = 1.0L;
    const long double tq = (long double)t[q + 1];
    for (int r = 0; r < m; ++r) {
      if (r == q) continue;
      const long double tr = (long double)t[r + 1];
      lo *= (-1.0L - tr) / (tq - tr);
      hi *= (1.0L - tr) / (tq - tr);
    }
    E[q] = (double)lo;
    E[m + q] = (double)hi;
  }
}

}  // namespace hps
