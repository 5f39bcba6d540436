"""GPU influence coefficients (Eqs. 8-10) and scalars against the oracle."""
import numpy as np
import pytest

from oracle import influence as inf
from oracle import material as m
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nx,ny,dx,dy,k,nu", [
    (1, 1, 1.0, 1.0, 0.5, 0.3),
    (7, 5, 0.3, 0.2, -0.5, 0.25),
    (40, 40, 1.0 / 64, 1.0 / 64, 0.5, 0.3),
    (33, 60, 0.01, 0.013, -0.8, 0.0),
    (64, 64, 1.0, 1.0, 0.0, 0.45),
    (50, 20, 1.0 / 256, 1.0 / 256, 0.9, 0.3),
])
def test_coefficients_match_oracle(nx, ny, dx, dy, k, nu):
    from paper_1612_08395_amd import bem
    announce("influence", nx, ny, dx, dy, k, nu)
    K = bem.bem_influence_ex(nx, ny, dx, dy, k, nu)
    got = bem.bem_influence_coeffs(K)
    ref = inf.influence_full(inf.influence_quarter(nx, ny, dx, dy, k))
    np.testing.assert_allclose(got, ref, rtol=2e-13, atol=0)
    info = bem.bem_influence_info(K)
    assert info.alpha == pytest.approx(m.alpha(k, nu), rel=1e-14)
    assert info.C == pytest.approx(m.compliance(k, nu), rel=1e-14)
    assert info.K00 == pytest.approx(ref[ny - 1, nx - 1], rel=2e-13)
    assert info.Mx >= 2 * nx and info.My >= 2 * ny
    K.free()


@pytest.mark.parametrize("n,k", [(2048, 0.3), (4096, -0.3)])
def test_coefficients_full_size_sampled(n, k):
    from paper_1612_08395_amd import bem
    announce("influence-full", n, k)
    dx = 1.0 / n
    K = bem.bem_influence(n, n, dx, k, 0.3)
    got = bem.bem_influence_coeffs(K)
    K.free()
    rng = np.random.default_rng(n)
    di = np.concatenate([np.arange(6), rng.integers(0, n, 400), [n - 1]])
    dj = np.concatenate([np.arange(6)[::-1], rng.integers(0, n, 400), [n - 1]])
    ref = inf.influence_at(di, dj, dx, dx, k)
    np.testing.assert_allclose(got[dj + n - 1, di + n - 1], ref, rtol=2e-13, atol=0)
    # evenness in both offsets
    np.testing.assert_array_equal(got[n - 1 - dj, n - 1 - di], got[dj + n - 1, di + n - 1])
