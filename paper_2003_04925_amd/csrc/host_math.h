// Host FP64 scalars: flat LambdaCDM background, growth factors, COLA time factors and the
// normalised initial power spectrum.
#pragma once

#include <vector>

namespace scola {

struct Background {
  double Om = 0.31, Ob = 0.0486, h = 0.6774, ns = 0.9667, sigma8 = 0.81, Tcmb = 2.7255;
  double amplitude = 0.0;   // P(k) = amplitude k^ns T(k)^2 at a = 1

  double E(double a) const;  // H(a)/H0, Omega_L = 1 - Omega_m, no radiation
  // Unnormalised growing-mode D1, dD1/da, D2, dD2/da (D1 -> a, D2 -> -3/7 a^2 at a -> 0).
  void growth(const std::vector<double>& a, std::vector<double>& D1, std::vector<double>& dD1,
              std::vector<double>& D2, std::vector<double>& dD2) const;
  double alpha_tilde(double ai, double af, double aK, double n) const;
  double beta_tilde(double ai, double af, double aD, double n) const;
  double alpha_standard(double ai, double af) const;
  double beta_standard(double ai, double af) const;
  double sigma8_unnormalised() const;
  void normalise();
  double power(double k) const;  // P_lin(k, a = 1), (Mpc/h)^3, k in h/Mpc
};

}  // namespace scola
