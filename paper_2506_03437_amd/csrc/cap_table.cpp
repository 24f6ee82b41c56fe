// Volume share of a d-ball beyond a hyperplane, for the recall model.
//
// The share of a ball of radius rho beyond a hyperplane at distance h from
// its centre is a hyperspherical cap; with t = h / rho in [0, 1) its share of
// the ball is 1/2 * I_{1 - t^2}((d + 1) / 2, 1/2), I being the regularised
// incomplete beta function (Sec. 5, "Geometric Model", cites this closed form).  The search
// looks the share up in a table of 1,024 evenly spaced t in [0, 1] with
// linear interpolation (Sec. 5.1, "Performance Optimizations"); this file fills that table.
//
// I_x(a, b) is evaluated from its continued fraction
//   I_x(a, b) = x^a (1 - x)^b / (a B(a, b)) * 1 / (1 + e_1 / (1 + e_2 / (1 + ...)))
//   e_{2m+1} = -(a + m)(a + b + m) x / ((a + 2m)(a + 2m + 1))
//   e_{2m}   =  m (b - m) x / ((a + 2m - 1)(a + 2m))
// (NIST DLMF 8.17.22), summed with the modified Lentz method (Thompson and
// Barnett, J. Comput. Phys. 64, 1986).  The fraction converges fast for
// x < (a + 1) / (a + b + 2); above that the symmetry
// I_x(a, b) = 1 - I_{1-x}(b, a) is used, with 1 - x passed in exactly (t^2)
// rather than recomputed from x.
#include <cmath>

#include "index.hpp"

namespace qk {
namespace {

// 1 / (1 + e_1 / (1 + e_2 / (1 + ...))) for I_x(a, b).
double beta_fraction(double a, double b, double x) {
  const double tiny = 1e-300;
  double f = 1.0, C = 1.0, D = 0.0;
  for (int j = 1; j <= 20000; ++j) {
    const int m = j / 2;
    double e;
    if (j & 1) e = -(a + m) * (a + b + m) * x / ((a + 2.0 * m) * (a + 2.0 * m + 1.0));
    else e = m * (b - m) * x / ((a + 2.0 * m - 1.0) * (a + 2.0 * m));
    D = 1.0 + e * D;
    if (std::fabs(D) < tiny) D = tiny;
    C = 1.0 + e / C;
    if (std::fabs(C) < tiny) C = tiny;
    D = 1.0 / D;
    const double delta = C * D;
    f *= delta;
    if (std::fabs(delta - 1.0) < 1e-16) break;
  }
  return 1.0 / f;
}

double log_beta(double a, double b) { return std::lgamma(a) + std::lgamma(b) - std::lgamma(a + b); }

// I_x(a, b) given x and y = 1 - x separately.
double reg_inc_beta(double a, double b, double x, double y) {
  if (x <= 0.0) return 0.0;
  if (y <= 0.0) return 1.0;
  if (x < (a + 1.0) / (a + b + 2.0)) {
    const double pre = std::exp(a * std::log(x) + b * std::log(y) - std::log(a) - log_beta(a, b));
    return pre * beta_fraction(a, b, x);
  }
  const double pre = std::exp(b * std::log(y) + a * std::log(x) - std::log(b) - log_beta(b, a));
  return 1.0 - pre * beta_fraction(b, a, y);
}

}  // namespace

double cap_fraction(double t, int d) {
  if (!(t < 1.0)) return 0.0;
  const double a = 0.5 * (d + 1), b = 0.5;
  const double tt = std::fabs(t);
  const double half = 0.5 * reg_inc_beta(a, b, 1.0 - tt * tt, tt * tt);
  return t >= 0.0 ? half : 1.0 - half;
}

void cap_fraction_table(int d, double* out) {
  for (int j = 0; j < CAP_TABLE_POINTS; ++j) out[j] = cap_fraction((double)j / (CAP_TABLE_POINTS - 1), d);
}

void cap_model_table(int d, double* out) {
  cap_fraction_table(d, out);
  const double a = 0.5 * (d + 1);
  out[CAP_TABLE_POINTS] = a;
  out[CAP_TABLE_POINTS + 1] = log_beta(a, 0.5);
}

}  // namespace qk
