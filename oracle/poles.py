"""Pole expansion of the Fermi projector (Section 3.1, eqs. FOP and dFOP).

Pi = (1/2 pi i) oint_Gamma (zI - H)^{-1} dz projects onto the eigenvalues inside
Gamma; a quadrature of the contour gives Pi ~= sum_j w_j (H - z_j I)^{-1}.  The
paper uses the conformal-map quadrature of Hale, Higham and Trefethen (2008)
and defers its details; the construction below is derived from that published
mathematics.

Elliptic (conformal-map) set.  Let the occupied eigenvalues lie in [lo, a] and
the unoccupied ones in [b, inf), lo < a < b.  The Moebius map w = 1/(b - z)
sends [lo, a] to [mw, Mw] = [1/(b - lo), 1/(b - a)], sends [b, inf) to
(-inf, 0) and infinity to 0, so the region between the two spectral pieces
becomes C \\ ((-inf, 0] U [mw, Mw]).  With k = (sqrt(Mw/mw) - 1)/(sqrt(Mw/mw) + 1)
and K, K' the complete elliptic integrals of moduli k and sqrt(1 - k^2),
    w(u) = sqrt(mw Mw) (1 + k sn(u|k^2)) / (1 - k sn(u|k^2))
maps the rectangle -K < Re u < K, 0 < Im u < K' onto the upper half plane with
(-K, K) -> [mw, Mw] and the top edge -> (-inf, 0].  The line Im u = K'/2
traversed over one real period 4K is a closed curve around [mw, Mw] (clockwise),
hence z(u) = b - 1/w(u) is a closed clockwise curve around [lo, a] that avoids
[b, inf).  The trapezoid rule with p nodes u_j = -K + (j - 1/2) 4K/p + i K'/2 on
Pi = -(1/2 pi i) int z'(u) (z(u) - H)^{-1} du gives
    z_j = z(u_j),   w_j = (4K / (2 pi i p)) z'(u_j).
Its error decays like exp(-pi K' p / (4K)), a function of the ratio
(b - lo)/(b - a) only: the kinetic width of the unoccupied spectrum does not
enter.

Circle set.  Trapezoid rule on a circle of centre c, radius rho:
z_j = c + rho e^{i theta_j}, theta_j = 2 pi (j - 1/2)/p, w_j = -rho e^{i theta_j}/p;
its filter is exactly r(lambda) = 1/(1 + ((lambda - c)/rho)^p).

Nodes come in complex-conjugate pairs (p even), so r(lambda) is real on the
real axis.  Index j runs 1..p: the paper prints both sum_{j=0}^{p} and
j = 1..p; p = 30 poles are used (Section 4).
"""

from __future__ import annotations

import numpy as np
from scipy.special import ellipj, ellipk


def _sn_cn_dn_complex(x, y, m):
    """Jacobi sn, cn, dn at u = x + i y with parameter m = k^2 (real x, y).

    Addition formulas with Jacobi's imaginary transformation (Abramowitz &
    Stegun 16.21): the real-argument functions at (x | m) and (y | 1 - m)."""
    s, c, d, _ = ellipj(x, m)
    s1, c1, d1, _ = ellipj(y, 1.0 - m)
    den = c1 * c1 + m * s * s * s1 * s1
    sn = (s * d1 + 1j * c * d * s1 * c1) / den
    cn = (c * c1 - 1j * s * d * s1 * d1) / den
    dn = (d * c1 * d1 - 1j * m * s * c * s1) / den
    return sn, cn, dn


def elliptic_poles(lo: float, a: float, b: float, p: int = 30):
    """Conformal-map pole set for the projector onto [lo, a] versus [b, inf).

    Returns (z, w) with Pi ~= sum_j w_j (H - z_j I)^{-1}."""
    if not (lo < a < b):
        raise ValueError("need lo < a < b")
    mw, Mw = 1.0 / (b - lo), 1.0 / (b - a)
    q = np.sqrt(Mw / mw)
    k = (q - 1.0) / (q + 1.0)
    m = k * k
    K = ellipk(m)
    Kp = ellipk(1.0 - m)
    j = np.arange(1, p + 1)
    x = -K + (j - 0.5) * 4.0 * K / p
    y = np.full(p, 0.5 * Kp)
    sn, cn, dn = _sn_cn_dn_complex(x, y, m)
    scale = np.sqrt(mw * Mw)
    w = scale * (1.0 + k * sn) / (1.0 - k * sn)
    dw = scale * 2.0 * k * cn * dn / (1.0 - k * sn) ** 2
    z = b - 1.0 / w
    dz = dw / (w * w)
    weights = (4.0 * K / (2j * np.pi * p)) * dz
    return z, weights


def circle_poles(center: float, radius: float, p: int = 30):
    """Trapezoid rule on the circle |z - center| = radius."""
    theta = 2.0 * np.pi * (np.arange(1, p + 1) - 0.5) / p
    e = np.exp(1j * theta)
    return center + radius * e, -radius * e / p


def circle_filter_closed_form(lam, center, radius, p):
    """1/(1 + ((lambda - c)/rho)^p): the exact filter of the circle rule."""
    zeta = (np.asarray(lam, dtype=float) - center) / radius
    return 1.0 / (1.0 + zeta ** p)


def filter_function(lam, z, w):
    """r(lambda) = sum_j w_j / (lambda - z_j), the scalar action of the pole sum."""
    lam = np.asarray(lam, dtype=float)
    return np.sum(w[None, :] / (lam[:, None] - z[None, :]), axis=1)


def elliptic_error_rate(lo: float, a: float, b: float, p: int) -> float:
    """exp(-pi K' p / (4K)), the geometric rate of the elliptic rule."""
    mw, Mw = 1.0 / (b - lo), 1.0 / (b - a)
    q = np.sqrt(Mw / mw)
    k = (q - 1.0) / (q + 1.0)
    K, Kp = ellipk(k * k), ellipk(1.0 - k * k)
    return float(np.exp(-np.pi * Kp * p / (4.0 * K)))


def auto_npoles(lo: float, a: float, b: float, tol: float = 1e-9, floor: int = 30, cap: int = 64) -> int:
    """Smallest even p >= floor (the paper's 30) with elliptic_error_rate <= tol (capped)."""
    p = floor
    while p < cap and elliptic_error_rate(lo, a, b, p) > tol:
        p += 2
    return p
