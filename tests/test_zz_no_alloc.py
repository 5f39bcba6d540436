"""The allocation-free convolution entry point (bem_convolve_dev_noalloc)
against the allocating one (bem_convolve_dev): same kernels, so the same
displacements bit for bit, on two calls in a row, the second on a smaller
grid than the first (the fixed scratch array keeps the first call's
contents), in both precisions; and the size limit."""
import numpy as np
import pytest

from paper_1612_08395_amd import inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _pair(bem, torch, nx, ny, k, precision, seed):
    dt = torch.float64 if precision == bem.BEM_FP64 else torch.float32
    K = bem.bem_influence(nx, ny, 1.0 / nx, k, 0.3)
    p = torch.tensor(inputs.random_pressure(ny, nx, seed), dtype=dt, device="cuda")
    u_ref = torch.full_like(p, float("nan"))
    u_na = torch.full_like(p, float("nan"))
    bem.bem_convolve_dev(K, precision, p, u_ref)
    bem.bem_convolve_dev_noalloc(K, precision, p, u_na)
    torch.cuda.synchronize()
    return K, p, u_ref, u_na


@pytest.mark.parametrize("prec_name", ["FP64", "MIXED"])
def test_noalloc_convolution_equals_allocating_one(prec_name):
    import torch
    from paper_1612_08395_amd import bem
    precision = getattr(bem, f"BEM_{prec_name}")
    # first call on the largest grid the array holds in this precision, then
    # a smaller, ragged one: 1024 x 1024 (FP64) / 2048 x 1024 (FP32), then 200 x 136
    big = (1024, 1024) if precision == bem.BEM_FP64 else (2048, 1024)
    for (nx, ny), k, seed in ((big, 0.3, 1), ((200, 136), -0.4, 2)):
        announce("noalloc", prec_name, nx, ny)
        K, p, u_ref, u_na = _pair(bem, torch, nx, ny, k, precision, seed)
        assert torch.isfinite(u_ref).all()
        assert torch.equal(u_na, u_ref), (nx, ny)
        K.free()


def test_noalloc_rejects_grids_beyond_its_array():
    import torch
    from paper_1612_08395_amd import bem
    announce("noalloc-limit")
    # FP32 2048 x 1200: 1200 rows of 2048 complex floats = 19.7 MB > 16 MiB
    K = bem.bem_influence(2048, 1200, 1.0 / 2048, 0.3, 0.3)
    p = torch.zeros((1200, 2048), dtype=torch.float32, device="cuda")
    u = torch.empty_like(p)
    with pytest.raises(bem.BemError) as e:
        bem.bem_convolve_dev_noalloc(K, bem.BEM_MIXED, p, u)
    assert e.value.code == bem.BEM_EUNSUPPORTED
    assert "scratch" in bem.bem_last_error()
    bem.bem_convolve_dev(K, bem.BEM_MIXED, p, u)      # the allocating entry point serves it
    torch.cuda.synchronize()
    assert not u.abs().max().item()
    K.free()
    with pytest.raises(bem.BemError) as e:
        bem.bem_convolve_dev_noalloc(_Null(), bem.BEM_FP64, p, u)
    assert e.value.code == bem.BEM_EINVAL


class _Null:
    handle = None
