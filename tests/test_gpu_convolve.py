"""GPU convolution u = C K * p (Eqs. 7, 12, 13) against the oracle."""
import numpy as np
import pytest

from oracle import influence as inf
from oracle import material as m
from oracle.convolution import FFTConvolver, conv_direct
from paper_1612_08395_amd import inputs
from tests.gpu_util import announce, rel_max

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-13     # max error / max |u|
FP32_TOL = 3e-6


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("ny,nx,k", [(1, 1, 0.3), (1, 9, 0.5), (17, 23, -0.5), (32, 32, 0.8)])
def test_fp64_matches_direct_sum(ny, nx, k):
    from paper_1612_08395_amd import bem
    announce("conv-direct", ny, nx, k)
    dx, dy = 1.0 / nx, 1.3 / nx
    K = bem.bem_influence_ex(nx, ny, dx, dy, k, 0.3)
    p = inputs.random_pressure(ny, nx, seed=nx * 7 + ny) - 0.25
    u = bem.bem_convolve(K, p)
    Kq = inf.influence_quarter(nx, ny, dx, dy, k)
    ref = conv_direct(Kq, p, m.compliance(k, 0.3))
    assert rel_max(u, ref) <= FP64_TOL
    K.free()


@pytest.mark.parametrize("ny,nx,k", [(128, 128, 0.5), (100, 37, -0.3), (301, 512, 0.0),
                                     (1024, 1024, -0.8), (63, 2048, 0.3), (1500, 700, 0.2),
                                     (2100, 130, -0.4), (2048, 2048, 0.3), (37, 1500, 0.6)])
def test_fp64_and_fp32_match_oracle_fft(ny, nx, k):
    from paper_1612_08395_amd import bem
    torch = _torch()
    announce("conv-fft", ny, nx, k)
    dx = 2.0 / max(nx, ny)
    K = bem.bem_influence(nx, ny, dx, k, 0.3)
    p = inputs.random_pressure(ny, nx, seed=ny + 3 * nx)
    Kq = inf.influence_quarter(nx, ny, dx, dx, k)
    ref = FFTConvolver(Kq, m.compliance(k, 0.3), workers=-1)(p)
    u64 = bem.bem_convolve(K, p)
    assert rel_max(u64, ref) <= FP64_TOL
    pd = torch.tensor(p, dtype=torch.float32, device="cuda")
    ud = torch.empty_like(pd)
    bem.bem_convolve_dev(K, bem.BEM_MIXED, pd, ud)
    torch.cuda.synchronize()
    assert rel_max(ud.cpu().numpy(), ref) <= FP32_TOL
    # device FP64 path, aliased in/out
    pd64 = torch.tensor(p, dtype=torch.float64, device="cuda")
    bem.bem_convolve_dev(K, bem.BEM_FP64, pd64, pd64)
    torch.cuda.synchronize()
    assert rel_max(pd64.cpu().numpy(), ref) <= FP64_TOL
    K.free()


@pytest.mark.parametrize("n,k", [(2048, 0.3), (4096, -0.3)])
def test_full_size_sparse_sources_sampled(n, k):
    # At full size the oracle evaluates sampled outputs one by one:
    # u(i, j) = C sum_s K(i - i_s, j - j_s) p_s for a few point loads.
    from paper_1612_08395_amd import bem
    torch = _torch()
    announce("conv-full", n, k)
    dx = 1.0 / n
    K = bem.bem_influence(n, n, dx, k, 0.3)
    rng = np.random.default_rng(n + 1)
    ns = 40
    si, sj = rng.integers(0, n, ns), rng.integers(0, n, ns)
    si[:4] = [0, n - 1, 0, n - 1]
    sj[:4] = [0, 0, n - 1, n - 1]
    ps = rng.random(ns) + 0.5
    p = np.zeros((n, n))
    np.add.at(p, (sj, si), ps)
    oi = np.concatenate([rng.integers(0, n, 120), [0, n - 1]])
    oj = np.concatenate([rng.integers(0, n, 120), [n - 1, 0]])
    C = m.compliance(k, 0.3)
    Kv = inf.influence_at((oi[:, None] - si[None, :]).ravel(), (oj[:, None] - sj[None, :]).ravel(),
                          dx, dx, k).reshape(len(oi), ns)
    ref = C * Kv @ ps
    scale = C * inf.influence_at([0], [0], dx, dx, k)[0] * ps.max()   # near-field magnitude
    for prec, dt, tol in ((bem.BEM_FP64, torch.float64, FP64_TOL), (bem.BEM_MIXED, torch.float32, 5e-6)):
        pd = torch.tensor(p, dtype=dt, device="cuda")
        ud = torch.empty_like(pd)
        bem.bem_convolve_dev(K, prec, pd, ud)
        torch.cuda.synchronize()
        got = ud.cpu().numpy()[oj, oi].astype(np.float64)
        err = np.max(np.abs(got - ref)) / scale
        assert err <= tol, (prec, err)
    K.free()
