"""Pressure -> surface displacement (oracle).

Test infrastructure only (see ``oracle/__init__``).

Eq. 7 / Eq. 12: u(i, j) = C * sum_{i', j'} K(i - i', j - j') p(i', j').

* ``conv_direct`` is that double sum written out, O(N^4); small grids only.
* ``FFTConvolver`` is Eq. 13: the same sum as a product of discrete Fourier
  transforms.  Eq. 13 as printed drops the factor (1 - nu^2) that Eqs. 7 and
  12 carry; C here is the full prefactor of Eq. 12.  A bare DFT product is a
  circular (periodic) convolution, so p is zero-padded to My x Mx with
  My >= 2ny - 1, Mx >= 2nx - 1 and K is laid out wrap-around
  (``influence_wrap``); the first ny x nx outputs of the circular product are
  then exactly the non-periodic half-space sum of Eq. 7.

Pins (tests/test_oracle_convolution.py): direct sum == FFT form to 1e-13 on
grids up to 32 x 32; independence of the padded size; a uniform pressure on
the whole grid gives, at a grid point, C times the integral of r^-(1+k) over
the loaded square (separate polar formula; Love's closed form at k = 0).
"""
import numpy as np
from scipy import fft

from .influence import influence_wrap


def conv_direct(Kq, p, C):
    """Eq. 7 as an explicit sum over all loaded elements."""
    ny, nx = p.shape
    u = np.empty_like(p, dtype=np.float64)
    jj = np.arange(ny)
    ii = np.arange(nx)
    for j in range(ny):
        rows = np.abs(j - jj)
        for i in range(nx):
            cols = np.abs(i - ii)
            u[j, i] = C * np.sum(Kq[rows[:, None], cols[None, :]] * p)
    return u


class FFTConvolver:
    """Eq. 13 with zero padding (see module docstring)."""

    def __init__(self, Kq, C, Mx=None, My=None, workers=None):
        ny, nx = Kq.shape
        self.nx, self.ny = nx, ny
        self.Mx = int(Mx) if Mx else 2 * nx
        self.My = int(My) if My else 2 * ny
        self.C = float(C)
        self.workers = workers
        self.Khat = fft.rfft2(influence_wrap(Kq, self.Mx, self.My), workers=workers)

    def __call__(self, p):
        P = fft.rfft2(np.asarray(p, dtype=np.float64), s=(self.My, self.Mx),
                      workers=self.workers)
        u = fft.irfft2(P * self.Khat, s=(self.My, self.Mx), workers=self.workers)
        return self.C * u[:self.ny, :self.nx]
