"""Pins of oracle/material.py against values fixed by the paper or by
mathematics independent of the oracle's formulas."""
import math
import os

import numpy as np
import pytest

from oracle import material as m

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("nu", [0.0, 0.25, 0.3, 0.45])
def test_alpha_boussinesq_at_k0(nu):
    # Eq. 2 at k = 0 must be Boussinesq's (1 - nu^2) F / (pi E r).
    assert m.beta(0.0, nu) == 1.0
    assert m.alpha(0.0, nu) == pytest.approx(1.0 / math.pi, rel=1e-15)


def test_alpha_gibson_limit():
    # k -> 1 at nu = 1/2: E(z) = E0 z / c0 is Gibson's incompressible soil,
    # shear modulus G(z) = m z with m = E0 / (3 c0), whose surface behaves as
    # a Winkler bed u = p / (2 m) = 1.5 p c0 / E0.  A uniform pressure p on a
    # disk of radius rho gives, at the centre, C p 2 pi rho^(1-k) / (1 - k)
    # (Eq. 5); as k -> 1 this tends to the local compliance
    # alpha (1 - nu^2) 2 pi / (1 - k) times p.
    for eps in (1e-6, 1e-8):
        k = 1.0 - eps
        local = m.alpha(k, 0.5) * (1.0 - 0.25) * 2.0 * math.pi / (1.0 - k)
        assert local == pytest.approx(1.5, rel=1e-5)


def test_alpha_positive_and_finite_over_domain():
    for k in np.linspace(-0.95, 0.95, 39):
        for nu in (0.0, 0.2, 0.3, 0.49):
            a = m.alpha(float(k), nu)
            assert np.isfinite(a) and a > 0


def test_check_k_domain():
    for bad in (-1.0, 1.0, 1.5, -2.0):
        with pytest.raises(ValueError):
            m.alpha(bad, 0.3)


def test_c1_eq23_closed_form_k0():
    # Eq. 23 at k = 0 is the classical self-potential of the unit square,
    # 4 ln(1 + sqrt 2) - (4/3)(sqrt 2 - 1) = 2.9732...
    exact = 4.0 * math.log(1.0 + math.sqrt(2.0)) - 4.0 / 3.0 * (math.sqrt(2.0) - 1.0)
    assert m.c1_eq23(0.0) == pytest.approx(exact, rel=1e-13)
    # and Table 1 prints 2.97 there
    assert m.c1_corrected(0.0) == pytest.approx(exact, abs=0.005)


@pytest.mark.parametrize("k", [-0.5, -0.3])
def test_c1_eq23_brute_force_monte_carlo(k):
    # The original four-fold integral over two independent points of the unit
    # square, sampled directly (finite variance for k < 0).
    rng = np.random.default_rng(23)
    n = 4_000_000
    a, b, a2, b2 = (rng.random(n) for _ in range(4))
    r = np.hypot(a - a2, b - b2)
    vals = r ** (-(1.0 + k))
    est = vals.mean()
    err = vals.std() / math.sqrt(n)
    assert abs(m.c1_eq23(k) - est) < 5.0 * err


def test_table1_matches_golden():
    rows = np.loadtxt(os.path.join(GOLDEN, "table1_c1.txt"))
    for k, c1 in rows:
        assert m.c1_corrected(float(k)) == c1


def test_c1_interpolation_between_table_points():
    ks = np.linspace(-0.9, 0.9, 181)
    vals = np.array([m.c1_corrected(float(k)) for k in ks])
    assert np.all(np.diff(vals) > 0)             # c1 increases with k
    # a point between two table entries lies between them
    assert 2.97 < m.c1_corrected(0.05) < 3.66


def _piece(i):
    """The cubic that ln c1 follows on [k_i, k_i+1], fitted through four
    interior points (exact interpolation when ln c1 is a cubic there)."""
    a, b = m.TABLE1_K[i], m.TABLE1_K[i + 1]
    x = np.linspace(a, b, 6)[1:-1]
    y = np.log([m.c1_corrected(float(t)) for t in x])
    return np.poly1d(np.polyfit(x - a, y, 3)), a, b


def test_c1_interpolant_is_the_natural_cubic_spline_of_ln_c1():
    # Between the Table 1 entries (Section 3.1) the reading is a natural
    # cubic spline of ln c1 over k.  Such a spline is fixed uniquely by four
    # properties, each checked here from values of c1_corrected alone:
    # (i) ln c1 is a cubic on every interval (its fourth difference on
    #     equally spaced points vanishes; a spline of c1 itself would leave
    #     a non-zero one),
    # (ii) it passes through the 19 tabulated values,
    # (iii) value, slope and curvature are continuous at the 17 interior
    #     knots (the cubics fitted on either side agree there),
    # (iv) the curvature is zero at k = -0.9 and 0.9 (natural ends; a
    #     clamped or not-a-knot end would not give zero).
    ks = m.TABLE1_K
    for i in range(len(ks) - 1):
        x = np.linspace(ks[i], ks[i + 1], 7)[1:-1]
        y = np.log([m.c1_corrected(float(t)) for t in x])
        d4 = y[0] - 4 * y[1] + 6 * y[2] - 4 * y[3] + y[4]
        assert abs(d4) < 1e-13, (i, d4)
    pieces = [_piece(i) for i in range(len(ks) - 1)]
    for i, (P, a, b) in enumerate(pieces):
        assert P(0.0) == pytest.approx(math.log(m.TABLE1_C1[i]), abs=1e-12)
        assert P(b - a) == pytest.approx(math.log(m.TABLE1_C1[i + 1]), abs=1e-12)
    for i in range(1, len(pieces)):
        L, aL, bL = pieces[i - 1]
        R, aR, _ = pieces[i]
        for der in (1, 2):
            left = L.deriv(der)(bL - aL)
            right = R.deriv(der)(0.0)
            assert left == pytest.approx(right, rel=1e-7, abs=1e-7), (i, der)
    first, a0, _ = pieces[0]
    last, aN, bN = pieces[-1]
    scale = max(abs(P.deriv(2)(0.0)) for P, _, _ in pieces)
    assert abs(first.deriv(2)(0.0)) < 1e-7 * scale
    assert abs(last.deriv(2)(bN - aN)) < 1e-7 * scale


def test_p_crit_scaling():
    # Eq. 24: p_crit ~ sqrt(gamma) * dx^-(1-k)/2 * sqrt(E0)
    k, nu = 0.3, 0.3
    base = m.p_crit(k, nu, 1e-3, 0.01)
    assert m.p_crit(k, nu, 4e-3, 0.01) == pytest.approx(2.0 * base, rel=1e-14)
    assert m.p_crit(k, nu, 1e-3, 0.04) == pytest.approx(base * 4.0 ** (-(1 - k) / 2), rel=1e-14)
    assert m.p_crit(k, nu, 1e-3, 0.01, E0=9.0) == pytest.approx(3.0 * base, rel=1e-14)


def test_p_crit_energy_balance():
    # Eqs. 19-22 with p^2: the self-energy of one loaded square element,
    # (1/2) C p^2 dx^(3-k) c1, equals gamma dx^2 exactly at p = p_crit.
    k, nu, gam, dx = -0.4, 0.25, 2e-3, 1.0 / 300
    pc = m.p_crit(k, nu, gam, dx)
    C = m.compliance(k, nu)
    U_el = 0.5 * C * pc * pc * dx ** (3 - k) * m.c1_corrected(k)
    assert U_el == pytest.approx(gam * dx * dx, rel=1e-13)
