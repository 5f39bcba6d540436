"""Material constants of the power-law graded half-space (oracle).

Test infrastructure only (see ``oracle/__init__``).

Section 2.1: modulus E(z) = E0 (z/c0)^k with -1 < k < 1 (Eq. 1); the surface
deflection under a point force is alpha(k,nu)(1-nu^2) c0^k F / (E0 r^(1+k))
(Eq. 2) with alpha and beta given by Eqs. 3-4.

Section 3.1: the mesh-dependent detachment stress p_crit (Eq. 24), which
uses the dimensionless coefficient c1(k).  The paper gives c1 both as the
four-fold integral of Eq. 23 and, for use in the simulations, as the
"corrected" values of Table 1; p_crit here uses Table 1.

Pins (tests/test_oracle_material.py):
* alpha(0, nu) = 1/pi for every nu (Eq. 2 reduces to Boussinesq at k = 0);
* k -> 1 at nu = 1/2: the compliance of a uniformly loaded large region
  tends to Gibson's incompressible linearly-graded half-space, u = p / (2 m)
  with shear modulus m z  (a limit that exercises every Gamma factor and
  the nu-term of beta);
* c1 of Eq. 23 at k = 0 equals the classical closed form
  4 ln(1 + sqrt 2) - (4/3)(sqrt 2 - 1), and at k < 0 a brute-force
  Monte-Carlo estimate of the original four-fold integral;
* Table 1 values are reproduced exactly at the tabulated k.
"""
import math

import numpy as np
from scipy import integrate, interpolate, special


def check_k(k):
    """Section 2.1, Eq. 1: the power must satisfy -1 < k < 1."""
    if not (-1.0 < k < 1.0):
        raise ValueError("power-law exponent k must satisfy -1 < k < 1")


def beta(k, nu):
    """Eq. 4."""
    check_k(k)
    return math.sqrt((1.0 + k) * (1.0 - k * nu / (1.0 - nu)))


def alpha(k, nu):
    """Eq. 3 (Gamma-function prefactor of the point-force solution)."""
    b = beta(k, nu)
    g = special.gamma
    num = (2.0 ** k) * b * math.sin(b * math.pi / 2.0) \
        * g((3.0 + k + b) / 2.0) * g((3.0 + k - b) / 2.0)
    den = math.sqrt(math.pi) * (1.0 + k) * math.cos(k * math.pi / 2.0) \
        * g(2.0 + k) * g(1.0 + k / 2.0) * g((1.0 - k) / 2.0)
    return num / den


def compliance(k, nu, E0=1.0, c0=1.0):
    """Prefactor C = alpha (1 - nu^2) c0^k / E0 of Eqs. 2, 5, 7 and 12."""
    return alpha(k, nu) * (1.0 - nu * nu) * c0 ** k / E0


def X_factor(k, nu):
    """alpha(k,nu) Gamma((1+k)/2) Gamma((1-k)/2): the combination that appears in
    Eqs. 16, 17, 25 and 26."""
    return alpha(k, nu) * special.gamma((1.0 + k) / 2.0) * special.gamma((1.0 - k) / 2.0)


# Table 1: corrected coefficient c1(k), k = -0.9 ... 0.9 in steps of 0.1.
TABLE1_K = np.round(np.arange(-9, 10) * 0.1, 10)
TABLE1_C1 = np.array([0.14, 0.31, 0.495, 0.71, 0.96, 1.24, 1.58, 1.97, 2.43,
                      2.97,
                      3.66, 4.52, 5.62, 7.10, 9.15, 12.25, 17.50, 27.65, 58.00])


def c1_corrected(k):
    """Corrected c1(k) of Table 1.

    Exactly the tabulated value at the 19 tabulated k.  Between them the paper
    gives nothing; this oracle takes a natural cubic spline of ln c1 over k
    (ln c1 is close to linear in k, so the spline is well behaved).  Outside
    [-0.9, 0.9] the end cubic pieces are extrapolated.
    """
    check_k(k)
    hit = np.nonzero(np.abs(TABLE1_K - k) < 1e-12)[0]
    if hit.size:
        return float(TABLE1_C1[hit[0]])
    spline = interpolate.CubicSpline(TABLE1_K, np.log(TABLE1_C1), bc_type="natural")
    return float(math.exp(spline(k)))


def c1_eq23(k):
    """c1(k) as the four-fold unit-square integral of Eq. 23, with the
    integrand read as |r - r'|^-(1+k) (the squares are lost in the printed
    formula; Eq. 19 fixes the meaning).

    Steps: (i) integrating over the two unit intervals of a and a' at fixed
    difference u = a - a' leaves the weight (1 - |u|) on u in [-1, 1] (same
    for b); by the symmetry of the weights the integral is
    4 * int_0^1 int_0^1 (1-u)(1-v)(u^2+v^2)^-(1+k)/2 du dv;
    (ii) in polar coordinates over the two triangles u > v and u < v (equal
    by symmetry) the radial integral is elementary and the angular one is
    done by adaptive quadrature.
    """
    check_k(k)

    def radial(theta):
        c, s = math.cos(theta), math.sin(theta)
        R = 1.0 / c                     # edge u = 1 of the triangle u >= v
        return (R ** (1 - k) / (1 - k) - (c + s) * R ** (2 - k) / (2 - k)
                + c * s * R ** (3 - k) / (3 - k))

    val, _ = integrate.quad(radial, 0.0, math.pi / 4.0, epsabs=0.0, epsrel=2e-14, limit=200)
    return 8.0 * val


def p_crit(k, nu, gamma12, dx, E0=1.0, c0=1.0, c1=None):
    """Critical detachment stress of Eq. 24 for square elements of side dx.

    c1 defaults to the corrected Table 1 value.  An element in contact whose
    tensile stress exceeds this value detaches (Section 3.1).
    """
    if c1 is None:
        c1 = c1_corrected(k)
    return math.sqrt(2.0 * E0 * gamma12
                     / (alpha(k, nu) * (1.0 - nu * nu) * c1 * c0 ** k * dx ** (1.0 - k)))
