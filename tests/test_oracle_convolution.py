"""Pins of oracle/convolution.py (Eqs. 7, 12, 13)."""
import numpy as np
import pytest

from oracle import analytic as an
from oracle import influence as inf
from oracle import material as m
from oracle.convolution import FFTConvolver, conv_direct
from paper_1612_08395_amd import inputs


@pytest.mark.parametrize("ny,nx,k", [(32, 32, 0.3), (17, 23, -0.5), (9, 31, 0.8), (1, 12, 0.0)])
def test_direct_sum_equals_fft(ny, nx, k):
    Kq = inf.influence_quarter(nx, ny, 1.0 / nx, 1.3 / nx, k)
    C = m.compliance(k, 0.3)
    p = inputs.random_pressure(ny, nx, seed=ny * 100 + nx) - 0.3   # mixed signs
    u_d = conv_direct(Kq, p, C)
    u_f = FFTConvolver(Kq, C)(p)
    assert np.max(np.abs(u_f - u_d)) <= 1e-13 * np.max(np.abs(u_d))


def test_padded_size_does_not_matter():
    n = 20
    Kq = inf.influence_quarter(n, n, 0.05, 0.05, -0.2)
    p = inputs.random_pressure(n, n, seed=5)
    ref = FFTConvolver(Kq, 1.0)(p)
    for (Mx, My) in [(2 * n - 1, 2 * n - 1), (64, 40), (3 * n, 4 * n)]:
        np.testing.assert_allclose(FFTConvolver(Kq, 1.0, Mx, My)(p), ref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("k", [-0.6, 0.0, 0.5])
def test_uniform_load_centre_displacement(k):
    # Uniform p on an odd (2R+1)^2 grid: at the centre element u equals
    # C p times the integral of r^-(1+k) over the whole loaded square.
    R = 15
    n = 2 * R + 1
    dx = 0.01
    Kq = inf.influence_quarter(n, n, dx, dx, k)
    C = m.compliance(k, 0.3)
    u = FFTConvolver(Kq, C)(np.full((n, n), 2.0))
    ref = C * 2.0 * an.centred_square_integral((R + 0.5) * dx, k)
    assert u[R, R] == pytest.approx(ref, rel=1e-12)
    # and the field is four-fold symmetric
    np.testing.assert_allclose(u, u[::-1, :], rtol=1e-13)
    np.testing.assert_allclose(u, u.T, rtol=1e-13)


@pytest.mark.parametrize("k", [-0.9, -0.5, 0.0, 0.8])
def test_influence_matrix_spd_and_real_spectrum(k):
    # K is real and even, so the DFT of its wrap-around layout is real.  The
    # N^2 x N^2 matrix of Eq. 12 itself is symmetric positive definite (brute
    # force eigenvalues), so the non-adhesive contact solution is unique.
    # (The circulant embedding of size (2N)^2 is indefinite for k < 0; it is
    # only ever used as a product, never inverted.)
    n = 16
    Kq = inf.influence_quarter(n, n, 1.0 / n, 1.0 / n, k)
    Kh = np.fft.fft2(inf.influence_wrap(Kq, 2 * n, 2 * n))
    assert np.max(np.abs(Kh.imag)) <= 1e-13 * np.max(np.abs(Kh.real))
    full = inf.influence_full(Kq)
    idx = np.arange(n)
    J = idx[:, None, None, None] - idx[None, None, :, None] + n - 1
    I = idx[None, :, None, None] - idx[None, None, None, :] + n - 1
    A = full[J, I].reshape(n * n, n * n)
    np.testing.assert_allclose(A, A.T, rtol=0, atol=0)
    ev = np.linalg.eigvalsh(A)
    assert ev[0] > 1e-6 * ev[-1]
