// Host construction of the pole sets of eq. dFOP (see poles.cpp).
#pragma once

#include <complex>
#include <vector>

namespace pomm {

// Projector onto eigenvalues in [lo, homo] versus [lumo, inf), lo < homo < lumo.
void elliptic_poles(double lo, double homo, double lumo, int p, std::vector<std::complex<double>>& z,
                    std::vector<std::complex<double>>& w);

// exp(-pi K' p / (4K)) of the elliptic rule for the window (lo, homo, lumo).
double elliptic_rate(double lo, double homo, double lumo, int p);

void circle_poles(double center, double radius, int p, std::vector<std::complex<double>>& z,
                  std::vector<std::complex<double>>& w);

}  // namespace pomm
