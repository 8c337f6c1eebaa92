// Host-side quadrature rules of the plan (see quadrature.cpp).
#pragma once
#include <vector>

namespace bzq {

// n Gauss-Legendre nodes x (increasing) and weights w on [0, R]
void gauss_legendre(int n, double R, std::vector<double>& x, std::vector<double>& w);

// n-point Gauss rule for \int_0^1 t^{-s} (1-t)^{-r} g(t) dt; false if s >= 1 or r >= 1
bool gauss_jacobi01(int n, double s, double r, std::vector<double>& t, std::vector<double>& w);

// n-point Gauss-Laguerre rule for \int_0^inf e^{-u} g(u) du (long double)
void gauss_laguerre(int n, std::vector<long double>& u, std::vector<long double>& w);

// Rule for \int_{t_c}^1 |log(2 sqrt t)| (1-t)^{-1/2} g(t) dt, t_c = sin^2(theta_cut/2)
// (the Debye-Yukawa weight of Section 5.6 in t = sin^2(theta/2)); g smooth.
// Composite: Gauss-Jacobi for (1-t)^{-1/2} on [1/4, 1] (64 nodes), Gauss-
// Legendre panels on [t0, 1/4] shrinking by 8 (32, 24, then 16 nodes), and for
// theta_cut = 0 Gauss-Laguerre (20 nodes) on [0, t0 = 1e-6] after t = t0 e^{-u}.
// false unless 0 <= theta_cut < pi/3.
bool debye_rule(double theta_cut, std::vector<double>& t, std::vector<double>& w);

// M-point Lebedev rule as rows (x, y, z, weight); false if no rule of size M
bool lebedev_rule(int M, std::vector<double>& xyzw);

// The half of the rule whose first non-zero coordinate is positive, each
// point's antipode checked to exist with an equal weight.  Returns M/2, or -1
// if the rule is not centrally symmetric.
int lebedev_half(const std::vector<double>& xyzw, std::vector<double>& half);

}  // namespace bzq
