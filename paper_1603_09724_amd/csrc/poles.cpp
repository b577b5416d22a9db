// Pole expansion of the Fermi projector (Section 3.1, eqs. FOP and dFOP), host side.
//
// Pi = (1/2 pi i) oint (zI - H)^{-1} dz over a contour around the occupied
// spectrum [lo, homo]; a p-point quadrature gives Pi ~= sum_j w_j (H - z_j I)^{-1}.
//
// Elliptic rule (conformal map in the spirit of Hale, Higham & Trefethen 2008,
// the quadrature the paper cites).  The Moebius map w = 1/(lumo - z) sends the
// occupied interval [lo, homo] to [wl, wh] = [1/(lumo-lo), 1/(lumo-homo)] and
// the unoccupied half line [lumo, inf) to (-inf, 0).  With
// k = (sqrt(wh/wl) - 1)/(sqrt(wh/wl) + 1) and complete elliptic integrals
// K = K(k), K' = K(sqrt(1-k^2)), the function
//   w(u) = sqrt(wl wh) (1 + k sn(u)) / (1 - k sn(u))
// maps the line Im u = K'/2 (one period, Re u in [-K, 3K)) to a closed curve
// around [wl, wh] that separates it from (-inf, 0]; z(u) = lumo - 1/w(u) is a
// closed curve around [lo, homo] avoiding [lumo, inf).  The p-point trapezoid
// rule in u gives
//   z_j = z(u_j),  w_j = (4K/(2 pi i p)) dz/du(u_j),  u_j = -K + (j - 1/2) 4K/p + i K'/2.
//
// Circle rule: trapezoid on |z - c| = rho, c = lo, rho = homo + (lumo-homo)/2 - lo,
// z_j = c + rho e^{i t_j}, t_j = 2 pi (j - 1/2)/p, w_j = -rho e^{i t_j}/p.
//
// Jacobi functions are computed by the arithmetic-geometric mean with the
// descending Landen transformation (Abramowitz & Stegun 16.4) for real
// arguments and the addition theorem with Jacobi's imaginary transformation
// (A&S 16.21) for complex ones.
#include <cmath>
#include <complex>
#include <vector>

#include "poles.h"

namespace pomm {

namespace {

using cd = std::complex<double>;

// K(m) = pi / (2 AGM(1, sqrt(1 - m))), parameter m = k^2 in [0, 1).
double ellip_k(double m) {
    double a = 1.0, b = std::sqrt(1.0 - m);
    for (int i = 0; i < 64 && std::fabs(a - b) > 1e-17 * a; ++i) {
        const double an = 0.5 * (a + b);
        b = std::sqrt(a * b);
        a = an;
    }
    return M_PI / (2.0 * a);
}

// sn, cn, dn of real u with parameter m (descending Landen / AGM).
void ellip_real(double u, double m, double& sn, double& cn, double& dn) {
    if (m < 1e-300) {
        sn = std::sin(u);
        cn = std::cos(u);
        dn = 1.0;
        return;
    }
    double a[40], c[40];
    a[0] = 1.0;
    double b = std::sqrt(1.0 - m);
    c[0] = std::sqrt(m);
    int N = 0;
    while (N < 38 && std::fabs(c[N]) > 1e-17) {
        a[N + 1] = 0.5 * (a[N] + b);
        c[N + 1] = 0.5 * (a[N] - b);
        b = std::sqrt(a[N] * b);
        ++N;
    }
    double phi = std::ldexp(a[N] * u, N);
    double phi_prev = phi;
    for (int i = N; i > 0; --i) {
        phi_prev = phi;
        phi = 0.5 * (phi + std::asin(c[i] / a[i] * std::sin(phi)));
    }
    sn = std::sin(phi);
    cn = std::cos(phi);
    dn = N > 0 ? cn / std::cos(phi_prev - phi) : 1.0;
}

void ellip_complex(double x, double y, double m, cd& sn, cd& cn, cd& dn) {
    double s, c, d, s1, c1, d1;
    ellip_real(x, m, s, c, d);
    ellip_real(y, 1.0 - m, s1, c1, d1);
    const double den = c1 * c1 + m * s * s * s1 * s1;
    sn = cd(s * d1, c * d * s1 * c1) / den;
    cn = cd(c * c1, -s * d * s1 * d1) / den;
    dn = cd(d * c1 * d1, -m * s * c * s1) / den;
}

}  // namespace

void elliptic_poles(double lo, double homo, double lumo, int p, std::vector<std::complex<double>>& z,
                    std::vector<std::complex<double>>& w) {
    const double wl = 1.0 / (lumo - lo), wh = 1.0 / (lumo - homo);
    const double q = std::sqrt(wh / wl);
    const double k = (q - 1.0) / (q + 1.0);
    const double m = k * k;
    const double K = ellip_k(m), Kp = ellip_k(1.0 - m);
    const double scale = std::sqrt(wl * wh);
    z.resize(p);
    w.resize(p);
    for (int j = 0; j < p; ++j) {
        const double x = -K + (j + 0.5) * 4.0 * K / p;
        cd sn, cn, dn;
        ellip_complex(x, 0.5 * Kp, m, sn, cn, dn);
        const cd den = 1.0 - k * sn;
        const cd ww = scale * (1.0 + k * sn) / den;
        const cd dw = scale * 2.0 * k * cn * dn / (den * den);
        z[j] = lumo - 1.0 / ww;
        const cd dz = dw / (ww * ww);
        w[j] = (4.0 * K / (2.0 * M_PI * p)) * dz / cd(0.0, 1.0);
    }
}

double elliptic_rate(double lo, double homo, double lumo, int p) {
    const double wl = 1.0 / (lumo - lo), wh = 1.0 / (lumo - homo);
    const double q = std::sqrt(wh / wl);
    const double k = (q - 1.0) / (q + 1.0);
    const double K = ellip_k(k * k), Kp = ellip_k(1.0 - k * k);
    return std::exp(-M_PI * Kp * p / (4.0 * K));
}

void circle_poles(double center, double radius, int p, std::vector<std::complex<double>>& z,
                  std::vector<std::complex<double>>& w) {
    z.resize(p);
    w.resize(p);
    for (int j = 0; j < p; ++j) {
        const double t = 2.0 * M_PI * (j + 0.5) / p;
        const cd e(std::cos(t), std::sin(t));
        z[j] = center + radius * e;
        w[j] = -radius * e / (double)p;
    }
}

}  // namespace pomm
