// Host-side quadrature rules of the plan (see quadrature.cpp).
#pragma once
#include <vector>

namespace bzq {

// n Gauss-Legendre nodes x (increasing) and weights w on [0, R]
void gauss_legendre(int n, double R, std::vector<double>& x, std::vector<double>& w);

// n-point Gauss rule for \int_0^1 t^{-s} (1-t)^{-r} g(t) dt; false if s >= 1 or r >= 1
bool gauss_jacobi01(int n, double s, double r, std::vector<double>& t, std::vector<double>& w);

// M-point Lebedev rule as rows (x, y, z, weight); false if no rule of size M
bool lebedev_rule(int M, std::vector<double>& xyzw);

// The half of the rule whose first non-zero coordinate is positive, each
// point's antipode checked to exist with an equal weight.  Returns M/2, or -1
// if the rule is not centrally symmetric.
int lebedev_half(const std::vector<double>& xyzw, std::vector<double>& half);

}  // namespace bzq
