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
    C = np.where(q <= q1, np.maximum(q, q0) ** expo, 0.0)
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


def serving_requests(count, seed, nu=0.3, mu_tabor=5.0, continuous_k=False):
    """A stream of independent solve requests of mixed size, material and
    indenter (all seeded):

    * grid n = round(2^U(6, 10)) snapped to a multiple of 16, side L = 1;
    * k uniform on the 0.05 grid inside (-0.8, 0.8) (so influence operators
      can be reused), nu fixed;
    * indenter, uniformly: paraboloid R = 1 with target contact radius
      a ~ U(0.1, 0.25) (depth a^2 / ((1+k) R), Eq. 15 of the paper), cone of
      slope 0.1 with d ~ U(0.005, 0.02), flat punch of radius L/4 with
      d ~ U(1e-3, 1e-2), or a rough surface (H ~ U(0.5, 0.9), q0 =
      min(8, n/16) 2 pi / L, q1 = (n/4) 2 pi / L, rms 1e-3, depth at the 5 %
      height quantile);
    * half of the requests adhesive: work of adhesion from a Tabor-like
      parameter mu = (R gamma^2 / (E*^2 dx^3))^(1/3) = 5 with R = 1 and the
      grid spacing as interaction range; non-adhesive preload to d0, then one
      pull-off solve at d0 / 2.
    continuous_k: the same stream with every k moved by U(-0.025, 0.025)
    (drawn from a generator of its own, so that the other draws are those of
    the 0.05-grid stream): no two requests share an influence operator.
    Returns a list of dicts (n, k, shape, h, d, d_preload, gamma).
    """
    rng = np.random.default_rng(seed)
    rng_k = np.random.default_rng(seed + 1)
    ks = np.round(np.arange(-15, 16) * 0.05, 10)
    estar = 1.0 / (1.0 - nu * nu)
    surfaces = {}
    out = []
    for i in range(count):
        n = int(round(2.0 ** rng.uniform(6.0, 10.0) / 16.0)) * 16
        n = max(64, min(1024, n))
        k = float(rng.choice(ks))
        if continuous_k:
            k = float(np.clip(k + rng_k.uniform(-0.025, 0.025), -0.795, 0.795))
        shape = ["parabolic", "cone", "punch", "rough"][int(rng.integers(0, 4))]
        L = 1.0
        if shape == "parabolic":
            a = rng.uniform(0.1, 0.25)
            h = parabolic(n, L, 1.0)
            d = a * a / ((1.0 + k) * 1.0)
        elif shape == "cone":
            h = cone(n, L, 0.1)
            d = rng.uniform(0.005, 0.02)
        elif shape == "punch":
            h = flat_punch(n, L, L / 4)
            d = rng.uniform(1e-3, 1e-2)
        else:
            key = (n, int(rng.integers(0, 8)))
            if key not in surfaces:
                H = 0.5 + 0.4 * ((key[1] + 0.5) / 8.0)
                surfaces[key] = fractal_gap(n, L, H, min(8.0, n / 16.0) * 2 * math.pi / L,
                                            (n / 4.0) * 2 * math.pi / L, 1e-3 * L, 7919 * n + key[1])
            h = surfaces[key]
            d = float(np.quantile(h, 0.05))
        adhesive = bool(rng.integers(0, 2))
        req = {"n": n, "k": k, "shape": shape, "h": h}
        if adhesive:
            dx = L / n
            req.update(d=0.5 * d, d_preload=d,
                       gamma=math.sqrt(mu_tabor ** 3 * estar * estar * dx ** 3 / 1.0))
        else:
            req.update(d=d, d_preload=0.0, gamma=0.0)
        out.append(req)
    return out
