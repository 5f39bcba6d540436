"""Force (load) control on the GPU against the FP64 oracle's load-controlled
solve (same seeded inputs), and against the GPU's own displacement control."""
import math

import numpy as np
import pytest

from oracle import influence as inf
from oracle import material as m
from oracle import solver as so
from paper_1612_08395_amd import inputs
from tests.gpu_util import announce, rel_l2

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10     # relative L2 pressure error, all-FP64 path
MIXED_TOL = 2e-5     # relative L2 pressure error, mixed path


def _bem():
    from paper_1612_08395_amd import bem
    return bem


def _force_params(bem, F, precision, **kw):
    return bem.bem_params_init(control=bem.BEM_CTRL_FORCE, F=F, precision=precision, **kw)


CASES = [
    # (nx, ny, side, k, shape, force)
    (64, 64, 1.0, 0.3, "parabolic", 2e-3),
    (37, 50, 1.0, -0.5, "parabolic", 1.5e-3),      # ragged, non-square grid
    (96, 96, 1.0, 0.2, "rough", None),              # force from a 5 % quantile depth
    (2200, 24, 1.0, -0.3, "parabolic", None),       # 4096-point row transforms
]


def _profile(nx, ny, L, shape):
    if shape == "parabolic":
        x = -L / 2 + (np.arange(nx) + 0.5) * (L / nx)
        y = -L * ny / nx / 2 + (np.arange(ny) + 0.5) * (L / nx)
        X, Y = np.meshgrid(x, y)
        return (X * X + Y * Y) / 2.0
    return inputs.fractal_gap(nx, L, 0.7, 4 * 2 * math.pi, nx / 4 * 2 * math.pi, 1e-3, 23)


@pytest.mark.parametrize("nx,ny,L,k,shape,F", CASES)
def test_force_control_parity(nx, ny, L, k, shape, F):
    bem = _bem()
    announce(f"force-parity {nx}x{ny} k={k} {shape}")
    dx = L / nx
    h = _profile(nx, ny, L, shape)
    Kq = inf.influence_quarter(nx, ny, dx, dx, k)
    C = m.compliance(k, 0.3)
    if F is None:
        d = float(np.quantile(h, 0.05))
        F = so.force(so.solve_nonadhesive(Kq, C, h, d, tol=1e-12).p, dx, dx)
    ref = so.solve_force(Kq, C, h, F, dx, dx, tol=1e-12)
    assert ref.converged
    K = bem.bem_influence_ex(nx, ny, dx, dx, k, 0.3)
    for prec, tol in ((bem.BEM_FP64, FP64_TOL), (bem.BEM_MIXED, MIXED_TOL)):
        rc, res, p, c, u = bem.bem_solve(K, h, _force_params(bem, F, prec), want_u=True)
        assert rc == 0 and res.status == 0
        assert rel_l2(p, ref.p) <= tol
        assert res.d == pytest.approx(ref.d, rel=10 * tol)
        assert res.F == pytest.approx(F, rel=1e-12 if prec == bem.BEM_FP64 else 1e-6)
        assert abs(int(c.sum()) - int(ref.contact.sum())) <= max(1, 1e-3 * ref.contact.sum())
        # u returned is the displacement; u + h - d vanishes on the contact
        assert np.max(np.abs((u + h - res.d)[c > 0])) <= 100 * tol * res.d
    K.free()


def test_force_and_displacement_control_agree_on_gpu():
    bem = _bem()
    announce("force-vs-displacement")
    n, k = 128, -0.3
    h = inputs.fractal_gap(n, 1.0, 0.8, 4 * 2 * math.pi, 32 * 2 * math.pi, 1e-3, 31)
    d = float(np.quantile(h, 0.1))
    K = bem.bem_influence(n, n, 1.0 / n, k, 0.3)
    _, rd, pd, cd, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d))
    _, rf, pf, cf, _ = bem.bem_solve(K, h, _force_params(bem, rd.F, bem.BEM_FP64))
    K.free()
    assert rf.d == pytest.approx(d, rel=1e-9)
    assert rel_l2(pf, pd) <= 1e-9
    assert np.array_equal(cf, cd)


def test_zero_load_and_force_sweep():
    bem = _bem()
    announce("force-zero-and-sweep")
    n = 64
    h = inputs.parabolic(n, 1.0, 1.0) + 1e-4          # min h = 1e-4 + the centre cells' r^2/2
    K = bem.bem_influence(n, n, 1.0 / n, 0.4, 0.3)
    rc, res, p, c, _ = bem.bem_solve(K, h, _force_params(bem, 0.0, bem.BEM_FP64))
    assert rc == 0 and not p.any() and not c.any()
    assert res.d == h.min() and res.F == 0.0
    forces = [4e-4, 8e-4, 1.6e-3, 8e-4]              # loading, then unloading
    st = bem.bem_state_create(K)
    rc, sweep = bem.bem_sweep(K, h, _force_params(bem, 0.0, bem.BEM_FP64), forces, state=st)
    st.free()
    assert rc == 0
    # the same loads through the device-h entry point as two concurrent chains
    import torch
    h_dev = torch.tensor(h, dtype=torch.float64, device="cuda")
    rc2, chained = bem.bem_sweep_dev(K, h_dev, _force_params(bem, 0.0, bem.BEM_FP64), forces,
                                     chains=2)
    assert rc2 == 0
    for F, r, r2 in zip(forces, sweep, chained):
        _, cold, _, _, _ = bem.bem_solve(K, h, _force_params(bem, F, bem.BEM_FP64))
        for x in (r, r2):
            assert x.F == pytest.approx(F, rel=1e-12)
            assert x.d == pytest.approx(cold.d, rel=1e-10)
            assert x.n_contact == cold.n_contact
    K.free()


def test_force_control_2048_mixed_vs_fp64():
    """Full size: rough 2048^2 surface under the load of 10 % contact area;
    the mixed path against the FP64 path, and the load constraint."""
    import torch
    bem = _bem()
    announce("force-2048")
    n = 2048
    h = inputs.fractal_gap(n, 1.0, 0.7, 8 * 2 * math.pi, 512 * 2 * math.pi, 1e-3, 1612)
    h_dev = torch.tensor(h, dtype=torch.float64, device="cuda")
    K = bem.bem_influence(n, n, 1.0 / n, 0.3, 0.3)
    _, rd = bem.bem_solve_dev(K, h_dev, bem.bem_params_init(d=0.004669638031382314))
    out = {}
    for prec in (bem.BEM_FP64, bem.BEM_MIXED):
        p = torch.empty((n, n), dtype=torch.float64, device="cuda")
        _, r = bem.bem_solve_dev(K, h_dev, _force_params(bem, rd.F, prec), p_out=p)
        assert r.status == 0
        out[prec] = (r, p)
    K.free()
    r64, p64 = out[bem.BEM_FP64]
    r32, p32 = out[bem.BEM_MIXED]
    assert r64.d == pytest.approx(0.004669638031382314, rel=1e-9)
    assert r64.F == pytest.approx(rd.F, rel=1e-12)
    err = float(torch.linalg.norm(p32 - p64) / torch.linalg.norm(p64))
    assert err <= MIXED_TOL
    assert r32.d == pytest.approx(r64.d, rel=1e-5)
    assert abs(r32.n_contact - r64.n_contact) <= 1e-3 * r64.n_contact
