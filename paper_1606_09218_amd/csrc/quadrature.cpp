// FP64 sinc quadrature of the Laplace-Gauss transform and the range split
// (sections 2.2-2.3): the paper-literal rule and the exponentially convergent
// rule with the substitution t = e^s (expsinc_nodes below).
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

// Nodes and weights of the rule with the substitution t = e^s (reading of
// eq sinc_conv's exponential rate): the Newton integrand becomes
// (2/sqrt(pi)) e^{s - r^2 e^{2s}}, r-free in u = s + ln r.  The trapezoid
// step h leaves a relative discretisation error ~ e^{-pi^2/(2h)}, so the
// design accuracy is eps(h) = e^{-(pi^2/(2h) - ln 2)}; with Lh = -ln eps(h),
// the first node must sit at u = (ln(1/0.38) - Lh)/3 + h/2 for r = r_hi (left
// tail ~ e^{3u}/3) and the last at u = ln(Lh + 1)/2 for r = r_lo (right tail
// e^{-e^{2u}}).  The step is the one for which M = R - 1 nodes span exactly
// that range (the span shrinks and the demand grows as h falls: one root,
// found by bisection).  Nodes left of the first, where e^{-r^2 t^2} ~ 1, are
// summed as a geometric series into the t_0 = 0 term.
static void expsinc_nodes(int R, double r_lo, double r_hi, std::vector<double>& t,
                          std::vector<double>& an) {
  const int M = R - 1;
  const double span = std::log(r_hi) - std::log(r_lo);
  auto Lh = [](double h) { return M_PI * M_PI / (2.0 * h) - std::log(2.0); };
  auto first_u = [&](double h) { return (-std::log(0.38) - Lh(h)) / 3.0 + 0.5 * h; };
  auto last_u = [&](double h) { return 0.5 * std::log(Lh(h) + 1.0); };
  // covered minus required span, increasing in h
  auto gap = [&](double h) { return (M - 1) * h - (last_u(h) - first_u(h) + span); };
  // bracket: h at L = 200 (tiny step) and at L = 0.5
  double hlo = M_PI * M_PI / (2.0 * (200.0 + std::log(2.0)));
  double hhi = M_PI * M_PI / (2.0 * (0.5 + std::log(2.0)));
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (hlo + hhi);
    if (gap(mid) < 0) hlo = mid;
    else hhi = mid;
  }
  const double h = 0.5 * (hlo + hhi);
  const double s1 = first_u(h) - std::log(r_hi);
  const double c = 2.0 / std::sqrt(M_PI);
  t.assign(R, 0.0);
  an.assign(R, 0.0);
  an[0] = c * h * std::exp(s1) / std::expm1(h);
  for (int k = 1; k <= M; ++k) {
    t[k] = std::exp(s1 + (k - 1) * h);
    an[k] = c * h * t[k];
  }
}

Table build_table(const rs_grid& g, const rs_fdesc& f) {
  RS_REQUIRE(g.b > 0 && std::isfinite(g.b), "grid half width b must be positive");
  RS_REQUIRE(g.n >= 8 && g.n % 2 == 0, "grid size n must be even and >= 8");
  RS_REQUIRE(f.R >= 3 && f.R <= 256, "R must be in [3, 256]");
  RS_REQUIRE(f.kernel == RS_NEWTON || f.kernel == RS_YUKAWA || f.kernel == RS_NEWTON_PLUS_YUKAWA,
             "unknown kernel");
  if (f.kernel != RS_NEWTON)
    RS_REQUIRE(f.lambda > 0 && std::isfinite(f.lambda), "Yukawa lambda must be positive");
  RS_REQUIRE(f.rule == RS_RULE_PAPER_LITERAL || f.rule == RS_RULE_EXP_SINC, "unknown quadrature rule");
  Table T;
  T.R = f.R;
  T.t.resize(f.R);
  T.a.resize(f.R);
  if (f.rule == RS_RULE_PAPER_LITERAL) {
    const double C0 = f.C0 > 0 ? f.C0 : 3.0;
    const int M = f.R - 1;
    const double hM = C0 * std::log((double)M) / (double)M;
    for (int k = 0; k < f.R; ++k) {
      T.t[k] = k * hM;
      T.a[k] = hM * weight_fn(f.kernel, T.t[k], f.lambda) * (k == 0 ? 0.5 : 1.0);
    }
  } else {
    const double r_lo = f.r_lo > 0 ? f.r_lo : 2.0 * g.b / (double)g.n;
    const double r_hi = f.r_hi > 0 ? f.r_hi : 2.0 * std::sqrt(3.0) * g.b;
    RS_REQUIRE(std::isfinite(r_lo) && std::isfinite(r_hi) && r_lo < r_hi, "need 0 < r_lo < r_hi");
    std::vector<double> an;
    expsinc_nodes(f.R, r_lo, r_hi, T.t, an);
    // the Newton weight (2/sqrt(pi)) h t_k times a(t_k) / a_Newton
    const double c = 2.0 / std::sqrt(M_PI);
    for (int k = 0; k < f.R; ++k) T.a[k] = an[k] * (weight_fn(f.kernel, T.t[k], f.lambda) / c);
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
