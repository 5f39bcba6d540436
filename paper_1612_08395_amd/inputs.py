"""Seeded synthetic inputs: grids, indenter gap profiles, rough surfaces.

This module holds no arithmetic of the contact method itself (no influence
coefficients, convolution or solver step).  It only builds the input arrays
that both the GPU library and its test oracle consume, so that the two are
fed identical data.

Geometry follows the problem statement of Section 2.2 / 3.2 of Li & Popov
(arXiv:1612.08395): a square domain of side L is cut into n x n square
elements; element centres sit at x_i = -L/2 + (i + 1/2) L / n, so for even n
the domain centre (the indenter axis) is an element corner and a centred
axisymmetric indenter has the four-fold symmetry of the grid.

The rough surface generator draws a Gaussian random field with an isotropic
power spectrum C(q) that is flat below the roll-off wavenumber q0, falls as
q^(-2(1+H)) between q0 and the cut-off q1 and is zero above q1 (the
self-affine surface family of the paper's Fig. 4 example, whose actual
surface is not published).
"""
import math

import numpy as np


def grid(n, L):
    """Element-centre coordinates (X, Y), each n x n, row index = y."""
    c = -L / 2.0 + (np.arange(n) + 0.5) * (L / n)
    return np.meshgrid(c, c, indexing="xy")


def radius(n, L):
    X, Y = grid(n, L)
    return np.hypot(X, Y)


def parabolic(n, L, R):
    """Gap of a rigid paraboloid of radius R: h = r^2 / (2R)."""
    r = radius(n, L)
    return r * r / (2.0 * R)


def cone(n, L, slope):
    """Gap of a rigid cone: h = slope * r."""
    return slope * radius(n, L)


def flat_punch(n, L, a, outside=None):
    """Rigid flat cylindrical punch of radius a: h = 0 under the punch and a
    large gap (never closed) outside."""
    r = radius(n, L)
    big = 10.0 * L if outside is None else outside
    return np.where(r <= a, 0.0, big)


def square_punch(n, L, half_side, angle_deg, outside=None):
    """Rigid flat square punch of half-side s rotated by angle_deg."""
    X, Y = grid(n, L)
    t = math.radians(angle_deg)
    xr = X * math.cos(t) + Y * math.sin(t)
    yr = -X * math.sin(t) + Y * math.cos(t)
    big = 10.0 * L if outside is None else outside
    inside = (np.abs(xr) <= half_side) & (np.abs(yr) <= half_side)
    return np.where(inside, 0.0, big)


def fractal_surface(n, L, H, q0, q1, rms, seed):
    """Gaussian self-affine height field z (n x n, float64) with zero mean and
    the given rms height.

    White Gaussian noise from numpy's default_rng(seed) is filtered in
    Fourier space by sqrt(C(q)), C(q) = q0^-2(1+H) for 0 < q < q0,
    q^-2(1+H) for q0 <= q <= q1, 0 above q1 and at q = 0, then transformed
    back and rescaled to the requested rms.
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n))
    W = np.fft.rfft2(w)
    qx = 2.0 * math.pi * np.fft.rfftfreq(n, d=L / n)
    qy = 2.0 * math.pi * np.fft.fftfreq(n, d=L / n)
    q = np.hypot(qx[None, :], qy[:, None])
    expo = -2.0 * (1.0 + H)
    C = np.where(q < q0, q0 ** expo, np.where(q <= q1, np.maximum(q, 1e-300) ** expo, 0.0))
    C[0, 0] = 0.0
    z = np.fft.irfft2(W * np.sqrt(C), s=(n, n))
    z -= z.mean()
    z *= rms / math.sqrt(np.mean(z * z))
    return z


def fractal_gap(n, L, H, q0, q1, rms, seed):
    """Gap of a rough rigid surface against a flat half-space: h = max(z) - z,
    zero at the highest summit."""
    z = fractal_surface(n, L, H, q0, q1, rms, seed)
    return z.max() - z


def random_pressure(n_y, n_x, seed, scale=1.0):
    """Non-negative random pressure field for convolution tests."""
    rng = np.random.default_rng(seed)
    return scale * rng.random((n_y, n_x))
