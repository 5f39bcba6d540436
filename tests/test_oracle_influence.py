"""Pins of oracle/influence.py (Eqs. 8-11) against closed forms."""
import math

import numpy as np
import pytest

from oracle import analytic as an
from oracle import influence as inf


@pytest.mark.parametrize("dx,dy", [(1.0, 1.0), (0.02, 0.02), (0.5, 0.2)])
def test_love_closed_form_k0(dx, dy):
    # k = 0: Love's rectangle solution for a homogeneous half-space.
    Kq = inf.influence_quarter(12, 9, dx, dy, 0.0)
    for dj in range(9):
        for di in range(12):
            ref = an.love_influence(di, dj, dx, dy)
            assert Kq[dj, di] == pytest.approx(ref, rel=2e-13)


@pytest.mark.parametrize("k", [-0.8, -0.5, -0.3, 0.3, 0.5, 0.8])
def test_eq11_off_axis_elements(k):
    # Eq. 11 holds for elements that do not straddle a coordinate axis.
    dx, dy = 0.7, 1.3
    Kq = inf.influence_quarter(40, 40, dx, dy, k)
    for (di, dj) in [(1, 1), (2, 3), (3, 1), (10, 7), (1, 25), (39, 39), (33, 2)]:
        ref = an.eq11_influence(di, dj, dx, dy, k)
        assert Kq[dj, di] == pytest.approx(ref, rel=2e-11)


@pytest.mark.parametrize("k", [-0.7, 0.0, 0.4])
def test_additivity_over_centred_block(k):
    # Sum of element integrals over the (2R+1)^2 block centred at the origin
    # equals the integral of r^-(1+k) over that square (separate polar form).
    R = 20
    Kq = inf.influence_quarter(R + 1, R + 1, 1.0, 1.0, k)
    total = inf.influence_full(Kq).sum()
    ref = an.centred_square_integral(R + 0.5, k)
    assert total == pytest.approx(ref, rel=1e-13)
    if k == 0.0:
        assert ref == pytest.approx(8 * (R + 0.5) * math.log(1 + math.sqrt(2)), rel=1e-14)


@pytest.mark.parametrize("k", [-0.5, 0.5])
def test_homogeneity(k):
    # The integrand has degree -(1+k) over a 2-D element: K scales as s^(1-k).
    K1 = inf.influence_quarter(6, 6, 1.0, 1.0, k)
    s = 1.0 / 256
    Ks = inf.influence_quarter(6, 6, s, s, k)
    np.testing.assert_allclose(Ks, s ** (1 - k) * K1, rtol=1e-13)


def test_square_symmetry_and_positivity():
    Kq = inf.influence_quarter(30, 30, 0.1, 0.1, 0.3)
    np.testing.assert_allclose(Kq, Kq.T, rtol=1e-14)
    assert np.all(Kq > 0)
    # decreasing away from the loaded element
    assert np.all(np.diff(Kq[0]) < 0) and np.all(np.diff(np.diag(Kq)) < 0)


def test_wrap_layout():
    Kq = inf.influence_quarter(5, 4, 1.0, 1.0, 0.2)
    W = inf.influence_wrap(Kq, 10, 8)
    full = inf.influence_full(Kq)
    for dj in range(-3, 4):
        for di in range(-4, 5):
            assert W[dj % 8, di % 10] == full[dj + 3, di + 4]
    # the unused middle row/column stay zero
    assert np.all(W[4, :] == 0) and np.all(W[:, 5] == 0)
    with pytest.raises(ValueError):
        inf.influence_wrap(Kq, 8, 8)
