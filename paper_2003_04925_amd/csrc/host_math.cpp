// Host FP64 scalars of a tiled-sCOLA plan: background, growth factors, COLA time factors
// and the sigma_8 normalisation of the initial power spectrum.
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace scola {

namespace {

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

template <typename F>
double integrate(F f, double a, double b, int panels, int order) {
  static thread_local std::vector<double> gx, gw;
  static thread_local int cached = 0;
  if (cached != order) {
    gauss_legendre(order, gx, gw);
    cached = order;
  }
  const double h = (b - a) / panels;
  double sum = 0.0;
  for (int p = 0; p < panels; ++p) {
    const double c = a + (p + 0.5) * h;
    double s = 0.0;
    for (int i = 0; i < order; ++i) s += gw[i] * f(c + 0.5 * h * gx[i]);
    sum += 0.5 * h * s;
  }
  return sum;
}

}  // namespace

double Background::E(double a) const {
  return std::sqrt(Om / (a * a * a) + 1.0 - Om);
}

// Growth ODEs of App. A: V[D1] = D1, V[D2] = D2 - D1^2 with V[.] = -(1/K) d/da((1/D) d./da).
// State y = {D1, P1, D2, P2}, P = a^3 E dD/da, integrated in x = ln a with classic RK4 from
// the matter-dominated growing mode (D1 = a, D2 = -3/7 a^2) at a = 1e-6.
void Background::growth(const std::vector<double>& a_query, std::vector<double>& D1,
                        std::vector<double>& dD1, std::vector<double>& D2,
                        std::vector<double>& dD2) const {
  const size_t n = a_query.size();
  std::vector<size_t> order(n);
  for (size_t i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(),
            [&](size_t i, size_t j) { return a_query[i] < a_query[j]; });
  D1.assign(n, 0.0);
  dD1.assign(n, 0.0);
  D2.assign(n, 0.0);
  dD2.assign(n, 0.0);
  auto rhs = [&](double x, const double* y, double* f) {
    const double a = std::exp(x);
    const double e = E(a);
    f[0] = y[1] / (a * a * e);
    f[1] = 1.5 * Om * y[0] / (a * e);
    f[2] = y[3] / (a * a * e);
    f[3] = 1.5 * Om * (y[2] - y[0] * y[0]) / (a * e);
  };
  const double a0 = 1e-6;
  double y[4] = {a0, a0 * a0 * a0 * E(a0), -3.0 / 7.0 * a0 * a0,
                 a0 * a0 * a0 * E(a0) * (-6.0 / 7.0 * a0)};
  double x = std::log(a0);
  const double hmax = 1.0 / 4096.0;
  for (size_t qi = 0; qi < n; ++qi) {
    const size_t idx = order[qi];
    const double xt = std::log(a_query[idx]);
    const double span = xt - x;
    if (span > 0.0) {
      const long steps = std::max(1L, (long)std::ceil(span / hmax));
      const double h = span / steps;
      for (long s = 0; s < steps; ++s) {
        double k1[4], k2[4], k3[4], k4[4], t[4];
        rhs(x, y, k1);
        for (int c = 0; c < 4; ++c) t[c] = y[c] + 0.5 * h * k1[c];
        rhs(x + 0.5 * h, t, k2);
        for (int c = 0; c < 4; ++c) t[c] = y[c] + 0.5 * h * k2[c];
        rhs(x + 0.5 * h, t, k3);
        for (int c = 0; c < 4; ++c) t[c] = y[c] + h * k3[c];
        rhs(x + h, t, k4);
        for (int c = 0; c < 4; ++c) y[c] += h / 6.0 * (k1[c] + 2 * k2[c] + 2 * k3[c] + k4[c]);
        x += h;
      }
      x = xt;
    }
    const double a = a_query[idx];
    const double inv = 1.0 / (a * a * a * E(a));
    D1[idx] = y[0];
    dD1[idx] = y[1] * inv;
    D2[idx] = y[2];
    dD2[idx] = y[3] * inv;
  }
}

// App. B, modified discretisation with u(a) = a^n: alpha~ = a_K^-n int a^(n-2)/H_conf da.
double Background::alpha_tilde(double ai, double af, double aK, double n) const {
  const double v = integrate([&](double a) { return std::pow(a, n - 2.0) / (a * E(a)); },
                             ai, af, 16, 16);
  return v / std::pow(aK, n);
}

// App. B: beta~ = -3/2 Omega_m (af^n - ai^n) / (n aD^n H_conf(aD)).
double Background::beta_tilde(double ai, double af, double aD, double n) const {
  return -1.5 * Om * (std::pow(af, n) - std::pow(ai, n)) / (n * std::pow(aD, n) * aD * E(aD));
}

// App. B eq. alpha-beta-standard (t = a): alpha = int da / (a^2 H_conf), beta = -3/2 Omega_m
// int da / (a H_conf), with H_conf = a E(a).
double Background::alpha_standard(double ai, double af) const {
  return integrate([&](double a) { return 1.0 / (a * a * a * E(a)); }, ai, af, 16, 16);
}

double Background::beta_standard(double ai, double af) const {
  return -1.5 * Om * integrate([&](double a) { return 1.0 / (a * a * E(a)); }, ai, af, 16, 16);
}

// sigma^2(8 Mpc/h) of k^n_s T(k)^2 with the top-hat window, as an integral over ln k.
double Background::sigma8_unnormalised() const {
  auto f = [&](double lnk) {
    const double k = std::exp(lnk);
    const double x = 8.0 * k;
    const double W = 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
    const double T = eh_nowiggle_transfer(k, Om, Ob, h, Tcmb);
    return k * k * k * std::pow(k, ns) * T * T * W * W / (2.0 * M_PI * M_PI);
  };
  return integrate(f, std::log(1e-6), std::log(1e3), 8000, 8);
}

double Background::power(double k) const {
  if (k <= 0.0) return 0.0;
  const double T = eh_nowiggle_transfer(k, Om, Ob, h, Tcmb);
  return amplitude * std::pow(k, ns) * T * T;
}

void Background::normalise() {
  amplitude = sigma8 * sigma8 / sigma8_unnormalised();
}

}  // namespace scola
