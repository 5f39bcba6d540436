"""Influence coefficients of a rectangular element (oracle).

Test infrastructure only (see ``oracle/__init__``).

Section 2.1, Eqs. 6-10: with constant pressure on each Dx x Dy element and
collocation at element centres, the displacement at element (i, j) caused by
unit pressure on element (i', j') is C * K, where K is the integral of the
point-force kernel r^-(1+k) over the loaded element (Eq. 9):

    K(di, dj) = int_{(di-1/2)Dx}^{(di+1/2)Dx} int_{(dj-1/2)Dy}^{(dj+1/2)Dy}
                (a^2 + b^2)^(-(1+k)/2) db da,     di = i - i', dj = j - j'.

The printed integrands of Eqs. 6 and 8 lose the squares and use Dx for the
y-limits; Eq. 9 fixes both (squared distance, separate Dx and Dy).  K
depends only on the offset, the element size and k (Eq. 10) and is even in
each offset, so only the quarter 0 <= di < nx, 0 <= dj < ny is computed.

Quadrature rules (chosen to differ from the GPU library's rules, so that
agreement between the two is meaningful):
* max(|di|, |dj|) <= 2: the element is split at the coordinate axes into
  pieces lying in one quadrant, each mirrored into the first quadrant.  A
  piece with the singular point at its corner is reduced exactly by polar
  coordinates (the radial integral of r^-(1+k) * r is elementary) to a
  smooth one-dimensional angular integral, done by adaptive quadrature; any
  other piece is integrated by nested adaptive quadrature.
* 2 < max(|di|, |dj|) <= 32: 20 x 20 tensor Gauss-Legendre on the element.
* beyond: 10 x 10 tensor Gauss-Legendre.
The integrand is analytic on every element of the last two groups; the
Gauss-Legendre error there is far below double-precision rounding.

Pins (tests/test_oracle_influence.py): Love's closed-form corner function at
k = 0; the hypergeometric closed form of Eq. 11 for elements that do not
straddle a coordinate axis; additivity (the sum over a centred square block
of elements equals the integral over the block, evaluated by a separate
polar formula); homogeneity K(s Dx, s Dy) = s^(1-k) K(Dx, Dy); symmetry.
"""
import math

import numpy as np
from scipy import integrate

from .material import check_k

NEAR = 2
MID = 32


def _corner_piece(X, Y, k):
    """int_0^X int_0^Y (a^2+b^2)^(-(1+k)/2) db da for X, Y > 0, via polar
    coordinates: the ray at angle theta leaves the rectangle at radius
    X/cos(theta) (theta below atan(Y/X)) or Y/sin(theta) (above), and
    int_0^R r^-(1+k) r dr = R^(1-k)/(1-k)."""
    th0 = math.atan2(Y, X)
    e = 1.0 - k
    lo, _ = integrate.quad(lambda t: (X / math.cos(t)) ** e, 0.0, th0,
                           epsabs=0.0, epsrel=2e-14, limit=200)
    hi, _ = integrate.quad(lambda t: (Y / math.sin(t)) ** e, th0, math.pi / 2.0,
                           epsabs=0.0, epsrel=2e-14, limit=200)
    return (lo + hi) / e


def _regular_piece(x0, x1, y0, y1, k):
    """Nested adaptive quadrature on a first-quadrant rectangle that does
    not have the origin as its corner (the integrand is then smooth on it)."""
    s = -(1.0 + k) / 2.0

    def inner(a):
        v, _ = integrate.quad(lambda b: (a * a + b * b) ** s, y0, y1,
                              epsabs=0.0, epsrel=5e-14, limit=200)
        return v

    v, _ = integrate.quad(inner, x0, x1, epsabs=0.0, epsrel=5e-14, limit=200)
    return v


def _split_axis(lo, hi):
    """Pieces of [lo, hi] on either side of 0, mirrored to non-negative
    intervals (the integrand is even in each coordinate)."""
    if lo >= 0.0:
        return [(lo, hi)]
    if hi <= 0.0:
        return [(-hi, -lo)]
    return [(0.0, -lo), (0.0, hi)]


def element_integral(a0, a1, b0, b1, k):
    """Adaptive-quadrature integral of (a^2+b^2)^(-(1+k)/2) over the
    rectangle [a0, a1] x [b0, b1] (Eq. 9 with general limits)."""
    check_k(k)
    total = 0.0
    for (x0, x1) in _split_axis(a0, a1):
        for (y0, y1) in _split_axis(b0, b1):
            if x1 <= x0 or y1 <= y0:
                continue
            if x0 == 0.0 and y0 == 0.0:
                total += _corner_piece(x1, y1, k)
            else:
                total += _regular_piece(x0, x1, y0, y1, k)
    return total


def _gauss_row(dj, dx, dy, k, order, di):
    """Tensor Gauss-Legendre value of K(di, dj) for a vector of di."""
    xg, wg = np.polynomial.legendre.leggauss(order)
    a = (di[:, None] + 0.5 * xg[None, :]) * dx            # (n, G)
    b = (dj + 0.5 * xg) * dy                              # (G,)
    f = (a[:, :, None] ** 2 + b[None, None, :] ** 2) ** (-(1.0 + k) / 2.0)
    return 0.25 * dx * dy * np.einsum("g,h,igh->i", wg, wg, f)


def influence_quarter(nx, ny, dx, dy, k):
    """K(di, dj) for 0 <= di < nx, 0 <= dj < ny as an (ny, nx) array
    (row index dj, column index di)."""
    check_k(k)
    if nx <= 0 or ny <= 0 or dx <= 0 or dy <= 0:
        raise ValueError("grid sizes and element sizes must be positive")
    Kq = np.empty((ny, nx))
    di_all = np.arange(nx, dtype=np.float64)
    for dj in range(ny):
        ring = np.maximum(np.arange(nx), dj)
        mid = ring <= MID
        if mid.any():
            Kq[dj, mid] = _gauss_row(dj, dx, dy, k, 20, di_all[mid])
        if (~mid).any():
            Kq[dj, ~mid] = _gauss_row(dj, dx, dy, k, 10, di_all[~mid])
    for dj in range(min(ny, NEAR + 1)):
        for di in range(min(nx, NEAR + 1)):
            Kq[dj, di] = element_integral((di - 0.5) * dx, (di + 0.5) * dx,
                                          (dj - 0.5) * dy, (dj + 0.5) * dy, k)
    return Kq


def influence_at(di, dj, dx, dy, k):
    """K at arbitrary offsets (arrays di, dj), with the same rules as
    ``influence_quarter`` (for sampled checks on grids too large to tabulate)."""
    check_k(k)
    di = np.abs(np.asarray(di, dtype=np.int64)).ravel()
    dj = np.abs(np.asarray(dj, dtype=np.int64)).ravel()
    out = np.empty(di.shape)
    ring = np.maximum(di, dj)
    for order, sel in ((20, (ring > NEAR) & (ring <= MID)), (10, ring > MID)):
        for j in np.unique(dj[sel]):
            rows = sel & (dj == j)
            out[rows] = _gauss_row(int(j), dx, dy, k, order, di[rows].astype(np.float64))
    for idx in np.nonzero(ring <= NEAR)[0]:
        a, b = int(di[idx]), int(dj[idx])
        out[idx] = element_integral((a - 0.5) * dx, (a + 0.5) * dx, (b - 0.5) * dy, (b + 0.5) * dy, k)
    return out


def influence_full(Kq):
    """The (2ny-1) x (2nx-1) array of K over all offsets, centred at
    (ny-1, nx-1): K is even in each offset (Eq. 10)."""
    ny, nx = Kq.shape
    jj = np.abs(np.arange(-(ny - 1), ny))
    ii = np.abs(np.arange(-(nx - 1), nx))
    return Kq[jj[:, None], ii[None, :]]


def influence_wrap(Kq, Mx, My):
    """K laid out for an My x Mx circular convolution: offset (di, dj) at
    index (dj mod My, di mod Mx); offsets beyond the grid stay zero.  With
    My >= 2ny-1 and Mx >= 2nx-1 no two offsets share an index."""
    ny, nx = Kq.shape
    if Mx < 2 * nx - 1 or My < 2 * ny - 1:
        raise ValueError("padded size must be at least 2n-1 in each direction")
    W = np.zeros((My, Mx))
    for dj in range(-(ny - 1), ny):
        for_row = Kq[abs(dj)]
        W[dj % My, np.arange(nx)] = for_row
        W[dj % My, (-np.arange(1, nx)) % Mx] = for_row[1:]
    return W
