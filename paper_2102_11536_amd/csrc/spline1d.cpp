// Host-side univariate toolkit: open uniform knots, Gauss-Legendre rule,
// B-spline values/derivatives per element (Sec. 5.1), the univariate
// parametric mass matrix of the preconditioner (Sec. 5.4) and its dense
// inverse on the free coefficients.
#include "ga_internal.h"

#include <cmath>
#include <vector>

namespace ga {

// Gauss-Legendre nodes/weights on [0,1]: Newton iteration on the Legendre
// polynomial evaluated by its three-term recurrence.
void gauss_legendre01(int nq, std::vector<double>& t, std::vector<double>& w) {
  t.assign(nq, 0.0);
  w.assign(nq, 0.0);
  for (int i = 0; i < nq; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (nq + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= nq; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (nq == 1) { p1 = x; p0 = 1.0; }
      dp = nq * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= nq; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (nq == 1) { p1 = x; p0 = 1.0; }
      dp = nq * (x * p1 - p0) / (x * x - 1.0);
    }
    // nodes returned in increasing order on [0,1]
    t[nq - 1 - i] = 0.5 * (x + 1.0);
    w[nq - 1 - i] = 1.0 / ((1.0 - x * x) * dp * dp);  // = 0.5 * 2/((1-x^2)P'^2)
  }
}

// Knot value i of the open uniform vector with n elements and degree p.
static inline double knot(int i, int n, int p) {
  if (i <= p) return 0.0;
  if (i >= n + p) return 1.0;
  return double(i - p) / n;
}

// Values and first derivatives of the p+1 B-splines that are nonzero on
// element e (basis indices e..e+p), at x inside that element, by the
// triangular form of the Cox-de Boor recursion.
void basis_on_element(int n, int p, int e, double x, double* val, double* der) {
  const int s = e + p;  // knot span index: knot(s) <= x < knot(s+1)
  double N[8], left[8], right[8], Nm1[8];
  N[0] = 1.0;
  for (int j = 1; j <= p; ++j) {
    left[j] = x - knot(s + 1 - j, n, p);
    right[j] = knot(s + j, n, p) - x;
    if (j == p)
      for (int r = 0; r < p; ++r) Nm1[r] = N[r];
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      double den = right[r + 1] + left[j - r];
      double tmp = den != 0.0 ? N[r] / den : 0.0;
      N[r] = saved + right[r + 1] * tmp;
      saved = left[j - r] * tmp;
    }
    N[j] = saved;
  }
  for (int r = 0; r <= p; ++r) val[r] = N[r];
  if (p == 0) {
    der[0] = 0.0;
    return;
  }
  // degree p-1 functions nonzero on the span: indices e+1 .. e+p (Nm1[0..p-1]);
  // derivative of basis e+r: p*(N_{e+r,p-1}/(k_{e+r+p}-k_{e+r}) - N_{e+r+1,p-1}/(k_{e+r+p+1}-k_{e+r+1}))
  for (int r = 0; r <= p; ++r) {
    int i = e + r;
    double a = (r >= 1) ? Nm1[r - 1] : 0.0;
    double b = (r <= p - 1) ? Nm1[r] : 0.0;
    double d1 = knot(i + p, n, p) - knot(i, n, p);
    double d2 = knot(i + p + 1, n, p) - knot(i + 1, n, p);
    der[r] = (d1 != 0.0 ? p * a / d1 : 0.0) - (d2 != 0.0 ? p * b / d2 : 0.0);
  }
}

Axis1D build_axis(int n, int p, int lo, int mf_free) {
  Axis1D ax;
  ax.n = n;
  ax.p = p;
  ax.q = p + 1;
  ax.m = n + p;
  ax.lo = lo;
  ax.mf = mf_free;
  std::vector<double> t, w;
  gauss_legendre01(ax.q, t, w);
  const int P1 = p + 1;
  ax.B.assign((size_t)n * ax.q * P1, 0.0);
  ax.D.assign((size_t)n * ax.q * P1, 0.0);
  ax.w.assign((size_t)n * ax.q, 0.0);
  double val[8], der[8];
  for (int e = 0; e < n; ++e)
    for (int j = 0; j < ax.q; ++j) {
      double x = (e + t[j]) / n;
      basis_on_element(n, p, e, x, val, der);
      for (int r = 0; r < P1; ++r) {
        ax.B[((size_t)e * ax.q + j) * P1 + r] = val[r];
        ax.D[((size_t)e * ax.q + j) * P1 + r] = der[r];
      }
      ax.w[(size_t)e * ax.q + j] = w[j] / n;
    }
  // univariate parametric mass matrix on the free coefficients (indices lo..lo+mf-1)
  const int mf = ax.mf;
  std::vector<double> Mh((size_t)mf * mf, 0.0);
  for (int e = 0; e < n; ++e)
    for (int j = 0; j < ax.q; ++j) {
      const double* b = &ax.B[((size_t)e * ax.q + j) * P1];
      double wj = ax.w[(size_t)e * ax.q + j];
      for (int r = 0; r < P1; ++r)
        for (int c = 0; c < P1; ++c) {
          int i1 = e + r - lo, i2 = e + c - lo;
          if (i1 < 0 || i2 < 0 || i1 >= mf || i2 >= mf) continue;
          Mh[(size_t)i1 * mf + i2] += wj * b[r] * b[c];
        }
    }
  ax.dhat.resize(mf);
  for (int i = 0; i < mf; ++i) ax.dhat[i] = Mh[(size_t)i * mf + i];
  // dense inverse through a Cholesky factor L L^T
  std::vector<double> L((size_t)mf * mf, 0.0);
  for (int j = 0; j < mf; ++j) {
    double s = Mh[(size_t)j * mf + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * mf + k] * L[(size_t)j * mf + k];
    double ljj = std::sqrt(s);
    L[(size_t)j * mf + j] = ljj;
    for (int i = j + 1; i < mf; ++i) {
      double v = Mh[(size_t)i * mf + j];
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * mf + k] * L[(size_t)j * mf + k];
      L[(size_t)i * mf + j] = v / ljj;
    }
  }
  ax.chol.assign((size_t)(mf + p) * P1, 0.0);
  for (int i = 0; i < mf; ++i) {
    ax.chol[(size_t)i * P1] = 1.0 / L[(size_t)i * mf + i];
    for (int d = 1; d <= p && i - d >= 0; ++d) ax.chol[(size_t)i * P1 + d] = L[(size_t)i * mf + i - d];
  }
  ax.Minv.assign((size_t)mf * mf, 0.0);
  std::vector<double> y(mf);
  for (int c = 0; c < mf; ++c) {
    for (int i = 0; i < mf; ++i) {  // L y = e_c
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) v -= L[(size_t)i * mf + k] * y[k];
      y[i] = v / L[(size_t)i * mf + i];
    }
    for (int i = mf - 1; i >= 0; --i) {  // L^T x = y
      double v = y[i];
      for (int k = i + 1; k < mf; ++k) v -= L[(size_t)k * mf + i] * ax.Minv[(size_t)k * mf + c];
      ax.Minv[(size_t)i * mf + c] = v / L[(size_t)i * mf + i];
    }
  }
  // symmetrise (the inverse of a symmetric matrix; removes rounding asymmetry)
  for (int i = 0; i < mf; ++i)
    for (int j = i + 1; j < mf; ++j) {
      double a = 0.5 * (ax.Minv[(size_t)i * mf + j] + ax.Minv[(size_t)j * mf + i]);
      ax.Minv[(size_t)i * mf + j] = a;
      ax.Minv[(size_t)j * mf + i] = a;
    }
  return ax;
}

}  // namespace ga
