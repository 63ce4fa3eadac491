// FP64 sinc quadrature of the Laplace-Gauss transform and the range split
// (sections 2.2-2.3).
//
//   p(z) = int_0^inf a(t) exp(-t^2 z^2) dt                        (eq laplace)
//   t_k = k h_M,  h_M = C0 log(M)/M,  M = R - 1                   (eq hM)
// The printed rule sums k = -M..M with a_k = a(t_k) h_M for an integral over
// R+; it is taken as the whole-line trapezoid rule of the even integrand
// folded onto k >= 0: a_0 = h_M a(0)/2, a_k = h_M a(t_k) for k >= 1, which
// gives R = M + 1 terms as the paper states for the Newton kernel.
//   Newton: a(t) = 2/sqrt(pi);  Yukawa: a(t) = 2/sqrt(pi) exp(-lambda^2/(4 t^2)).
// Long range: k = 0..R_l-1; short range: k = R_l..R-1 (eq Split_Qpoints).
// Criterion (A) (eq Split_crit_max) with delta = delta_rel * S(0).
#include <cmath>

#include "rs_internal.h"

namespace rs {

static double weight_fn(int kernel, double t, double lambda) {
  const double c = 2.0 / std::sqrt(M_PI);
  double yuk = 0.0;
  if (t > 0.0) yuk = c * std::exp(-lambda * lambda / (4.0 * t * t));
  switch (kernel) {
    case RS_NEWTON: return c;
    case RS_YUKAWA: return yuk;
    case RS_NEWTON_PLUS_YUKAWA: return c + yuk;
  }
  throw Error{RS_E_INVALID, "unknown kernel"};
}

Table build_table(const rs_grid& g, const rs_fdesc& f) {
  RS_REQUIRE(g.b > 0 && std::isfinite(g.b), "grid half width b must be positive");
  RS_REQUIRE(g.n >= 8 && g.n % 2 == 0, "grid size n must be even and >= 8");
  RS_REQUIRE(f.R >= 3 && f.R <= 256, "R must be in [3, 256]");
  RS_REQUIRE(f.kernel == RS_NEWTON || f.kernel == RS_YUKAWA || f.kernel == RS_NEWTON_PLUS_YUKAWA,
             "unknown kernel");
  if (f.kernel != RS_NEWTON)
    RS_REQUIRE(f.lambda > 0 && std::isfinite(f.lambda), "Yukawa lambda must be positive");
  const double C0 = f.C0 > 0 ? f.C0 : 3.0;
  const int M = f.R - 1;
  const double hM = C0 * std::log((double)M) / (double)M;
  Table T;
  T.R = f.R;
  T.t.resize(f.R);
  T.a.resize(f.R);
  for (int k = 0; k < f.R; ++k) {
    T.t[k] = k * hM;
    T.a[k] = hM * weight_fn(f.kernel, T.t[k], f.lambda) * (k == 0 ? 0.5 : 1.0);
  }
  T.S0 = 0.0;
  for (int k = 0; k < f.R; ++k) T.S0 += T.a[k];
  const double delta = (f.delta_rel > 0 ? f.delta_rel : 1e-4) * T.S0;

  if (f.R_l == -1) {
    RS_REQUIRE(f.sigma_split > 0, "sigma_split must be positive when R_l is chosen by criterion (A)");
    // short set = the tail on which a_k exp(-t_k^2 sigma^2) <= delta
    int R_l = f.R;
    for (int k = f.R - 1; k >= 0; --k) {
      if (T.a[k] * std::exp(-(T.t[k] * f.sigma_split) * (T.t[k] * f.sigma_split)) <= delta) R_l = k;
      else break;
    }
    RS_REQUIRE(R_l >= 1 && R_l <= f.R - 1, "criterion (A) leaves no long or no short terms");
    T.R_l = R_l;
  } else {
    RS_REQUIRE(f.R_l >= 1 && f.R_l <= f.R - 1, "R_l must be in [1, R-1]");
    T.R_l = f.R_l;
  }
  T.S_l0 = 0.0;
  for (int k = 0; k < T.R_l; ++k) T.S_l0 += T.a[k];

  const double h = 2.0 * g.b / (double)g.n;
  if (f.n_s == -1) {
    double sigma = 0.0;
    for (int k = T.R_l; k < f.R; ++k)
      if (T.a[k] > delta) sigma = std::fmax(sigma, std::sqrt(std::log(T.a[k] / delta)) / T.t[k]);
    int ns = (int)std::ceil(2.0 * sigma / h - 1e-12);
    if (ns < 1) ns = 1;
    if (ns % 2 == 0) ++ns;
    T.n_s = ns;
  } else {
    RS_REQUIRE(f.n_s >= 1 && f.n_s % 2 == 1, "n_s must be odd and positive");
    T.n_s = f.n_s;
  }
  RS_REQUIRE(T.n_s <= g.n + 1, "window wider than the grid");
  return T;
}

}  // namespace rs
