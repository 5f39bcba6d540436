"""Closed forms used only as pins (oracle side).

Test infrastructure only (see ``oracle/__init__``).

* ``eq11_influence``: the hypergeometric closed form of K printed as Eq. 11.
  Evaluated as printed it agrees with the integral of Eq. 9 only for
  elements that do not straddle a coordinate axis (|di|, |dj| >= 1); it is
  singular at k = 0.  Used as a pin for those elements only.
* ``love_influence``: Love's closed form for uniform pressure on a rectangle
  of a homogeneous half-space (the k = 0 case, cited in Section 2.1):
  corner function x asinh(y/x) + y asinh(x/y).
* Hertz-type parabolic indentation (Section 2.2): contact radius from
  Eq. 15, exterior displacement Eq. 14 (free of alpha).  For the force, Eq. 16
  as printed is off from Hertz by pi^2 at k = 0; the reading used here
  places alpha Gamma((1+k)/2) Gamma((1-k)/2) in the denominator:
  F = 4 E0 a^(3+k) / (X (k+1)^2 (k+3) (1-nu^2) c0^k R),  X = alpha Gamma Gamma.
  It follows from superposing flat punches with the stiffness below, and is
  Hertz's 4 E* a^3 / (3 R) at k = 0.
* Flat punch: stiffness 2 E0 a^(1+k) / (X (1+k) (1-nu^2) c0^k) (Boussinesq
  2 E* a at k = 0).  Adhesive flat punch (Section 3.2): Eq. 25 for d_crit as
  printed; Eq. 26 read with X in the denominator, F_crit = stiffness * d_crit.
* JKR-type parabolic adhesion: Hertz-type solution plus a flat punch held
  at d_crit(a).  Minimum force -(3+k) pi gamma R / 2, the JKR -3 pi gamma R / 2
  at k = 0.
"""
import math

import numpy as np
from scipy import special

from .material import X_factor


def eq11_influence(di, dj, dx, dy, k):
    """Eq. 11 as printed, for offset (di, dj) = (i - i', j - j')."""
    p = (-di + 0.5) * dx
    q = (-di - 0.5) * dx
    m = (-dj + 0.5) * dy
    n = (-dj - 0.5) * dy
    e = (1.0 - k) / 2.0

    def F1(z):
        return special.hyp2f1(0.5, 1.0, (k + 2.0) / 2.0, z)

    def F2(z):
        return special.hyp2f1(1.0, 1.0 - k / 2.0, 1.5, z)

    s = (-n * p * (m * m + p * p) ** e * F1(-p * p / (m * m))
         + m * p * (n * n + p * p) ** e * F1(-p * p / (n * n))
         + n * q * (m * m + q * q) ** e * F1(-q * q / (m * m))
         - m * q * (n * n + q * q) ** e * F1(-q * q / (n * n))
         + k * n * p * (m * m + p * p) ** e * F2(-p * p / (m * m))
         - k * m * p * (n * n + p * p) ** e * F2(-p * p / (n * n))
         - k * n * q * (m * m + q * q) ** e * F2(-q * q / (m * m))
         + k * m * q * (n * n + q * q) ** e * F2(-q * q / (n * n)))
    return s / (m * n * (k - k * k))


def _love_corner(x, y):
    """Love's corner function for k = 0, odd in each argument."""
    if x == 0.0 or y == 0.0:
        return 0.0
    sx, sy = math.copysign(1.0, x), math.copysign(1.0, y)
    x, y = abs(x), abs(y)
    return sx * sy * (x * math.asinh(y / x) + y * math.asinh(x / y))


def love_influence(di, dj, dx, dy):
    """k = 0 element integral from Love's corner function."""
    a0, a1 = (di - 0.5) * dx, (di + 0.5) * dx
    b0, b1 = (dj - 0.5) * dy, (dj + 0.5) * dy
    return (_love_corner(a1, b1) - _love_corner(a0, b1)
            - _love_corner(a1, b0) + _love_corner(a0, b0))


def centred_square_integral(s, k):
    """Integral of r^-(1+k) over the square [-s, s]^2, by polar coordinates
    over its eight symmetric triangles: 8 s^(1-k)/(1-k) int_0^{pi/4} sec^(1-k).
    At k = 0 this is 8 s ln(1 + sqrt 2)."""
    from scipy import integrate
    v, _ = integrate.quad(lambda t: (1.0 / math.cos(t)) ** (1.0 - k), 0.0, math.pi / 4,
                          epsabs=0.0, epsrel=2e-14)
    return 8.0 * s ** (1.0 - k) / (1.0 - k) * v


def hertz_radius(k, R, d):
    """Eq. 15 solved for a."""
    return math.sqrt((1.0 + k) * R * d)


def hertz_force(k, nu, R, a, E0=1.0, c0=1.0):
    """Hertz-type force at contact radius a (reading of Eq. 16, see module doc)."""
    X = X_factor(k, nu)
    return 4.0 * E0 * a ** (3.0 + k) / (X * (k + 1.0) ** 2 * (k + 3.0)
                                        * (1.0 - nu * nu) * c0 ** k * R)


def hertz_force_printed(k, nu, R, a, E0=1.0, c0=1.0):
    """Eq. 16 exactly as printed (kept to document the discrepancy)."""
    from .material import alpha
    G = special.gamma((1.0 + k) / 2.0) * special.gamma((1.0 - k) / 2.0)
    return (4.0 * alpha(k, nu) / (G * (k + 1.0) ** 2 * (k + 3.0))
            * E0 / ((1.0 - nu * nu) * c0 ** k) * a ** (3.0 + k) / R)


def hertz_uz(r, a, R, k):
    """Eq. 14: surface deflection inside and outside the contact radius.
    B(x; a, b) is the non-regularised incomplete Beta function."""
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    inside = r < a
    out[inside] = (1.0 / (k + 1.0) - r[inside] ** 2 / (2.0 * a * a)) * a * a / R
    ro = r[~inside]
    x = (a / ro) ** 2

    def B(xx, aa, bb):
        return special.betainc(aa, bb, xx) * special.beta(aa, bb)

    val = math.cos(k * math.pi / 2.0) / (math.pi * (k + 1.0)) * (
        B(x, (1.0 + k) / 2.0, (1.0 - k) / 2.0)
        - ro ** 2 / a ** 2 * B(x, (3.0 + k) / 2.0, (1.0 - k) / 2.0))
    out[~inside] = val * a * a / R
    return out


def flat_punch_stiffness(k, nu, a, E0=1.0, c0=1.0):
    """F / d of a rigid flat circular punch of radius a."""
    return 2.0 * E0 * a ** (1.0 + k) / (X_factor(k, nu) * (1.0 + k) * (1.0 - nu * nu) * c0 ** k)


def flat_punch_dcrit(k, nu, gamma12, a, E0=1.0, c0=1.0):
    """Eq. 25."""
    return math.sqrt(X_factor(k, nu) * 2.0 * math.pi * (1.0 - nu * nu) * gamma12
                     * a ** (1.0 - k) * c0 ** k / E0)


def flat_punch_Fcrit(k, nu, gamma12, a, E0=1.0, c0=1.0):
    """Eq. 26 read with X in the denominator: stiffness times d_crit."""
    return flat_punch_stiffness(k, nu, a, E0, c0) * flat_punch_dcrit(k, nu, gamma12, a, E0, c0)


def jkr_curve(k, nu, gamma12, R, a, E0=1.0, c0=1.0):
    """Indentation and force of the JKR-type parabolic contact at radius a."""
    dH = a * a / ((1.0 + k) * R)
    dc = flat_punch_dcrit(k, nu, gamma12, a, E0, c0)
    F = hertz_force(k, nu, R, a, E0, c0) - flat_punch_stiffness(k, nu, a, E0, c0) * dc
    return dH - dc, F


def jkr_min_force(k, gamma12, R):
    """Minimum of the JKR-type force curve: -(3+k) pi gamma R / 2."""
    return -(3.0 + k) * math.pi * gamma12 * R / 2.0
