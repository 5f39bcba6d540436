"""Parity at the full workload sizes.

The oracle cannot run whole solves at 2048^2 / 4096^2 within a test, so here:
* the KKT conditions of the GPU pressure are checked with the oracle's own
  convolution (a property that holds at any size);
* the mixed path is compared with the all-FP64 path on the same inputs;
* 256^2 crops of the 4096^2 surface, at identical statistics, are solved by
  both the GPU (mixed) and the oracle (spot checks);
* the 512^2 adhesive sweep is compared step transition by step transition.
"""
import math

import numpy as np
import pytest

from oracle import analytic as an
from oracle import influence as inf
from oracle import material as m
from oracle import solver as so
from oracle.convolution import FFTConvolver
from paper_1612_08395_amd import inputs
from tests.gpu_util import announce, rel_l2

pytestmark = pytest.mark.gpu

TWO_PI = 2.0 * math.pi


def _rough(n, H, q0, q1, seed, L=1.0):
    return inputs.fractal_gap(n, L, H, q0 * TWO_PI / L, q1 * TWO_PI / L, 1e-3 * L, seed)


def _kkt(Kq, C, h, d, p, conv, gtol):
    g = conv(p) + h - d
    contact = p > 0
    assert p.min() >= 0.0
    assert g.min() >= -gtol                        # no interpenetration
    assert np.max(np.abs(g[contact])) <= gtol     # gap closed where loaded
    return contact.sum()


def test_rough_2048_kkt_and_mixed_vs_fp64():
    import torch
    from paper_1612_08395_amd import bem
    n, k, nu = 2048, 0.3, 0.3
    announce("rough-2048", n, k)
    h = _rough(n, 0.7, 8.0, 512.0, 1612)
    dx = 1.0 / n
    K = bem.bem_influence(n, n, dx, k, nu)
    h_dev = torch.tensor(h, dtype=torch.float64, device="cuda")
    d = float(np.quantile(h, 0.08))            # a few percent contact
    p64 = torch.empty_like(h_dev)
    p32 = torch.empty_like(h_dev)
    _, r64 = bem.bem_solve_dev(K, h_dev, bem.bem_params_init(d=d), p_out=p64)
    _, r32 = bem.bem_solve_dev(K, h_dev, bem.bem_params_init(d=d, precision=bem.BEM_MIXED),
                               p_out=p32)
    torch.cuda.synchronize()
    assert r64.status == 0
    P64, P32 = p64.cpu().numpy(), p32.cpu().numpy()
    Kq = inf.influence_quarter(n, n, dx, dx, k)
    conv = FFTConvolver(Kq, m.compliance(k, nu), workers=-1)
    nc = _kkt(Kq, m.compliance(k, nu), h, d, P64, conv, gtol=1e-9 * d)
    assert nc == r64.n_contact
    err = rel_l2(P32, P64)
    print(f"[rough-2048] contact {nc / n / n:.4f}, mixed vs fp64 rel L2 {err:.3e}, "
          f"iters {r32.iters}/{r64.iters}", flush=True)
    assert err <= 2e-5
    assert abs(r32.n_contact - r64.n_contact) <= 1e-3 * r64.n_contact
    K.free()


def test_rough_4096_crops_mixed_vs_oracle():
    # 256^2 windows cut from the 4096^2 surface at the quadrant centres, each
    # solved as its own 256^2 problem (k = -0.3, nu = 0.25).
    from paper_1612_08395_amd import bem
    n, k, nu = 4096, -0.3, 0.25
    announce("crops-4096")
    h = _rough(n, 0.7, 8.0, 512.0, 8395)           # q1 = 1/4 of Nyquist at 4096
    w = 256
    dx = 1.0 / n
    Kq = inf.influence_quarter(w, w, dx, dx, k)
    C = m.compliance(k, nu)
    conv = FFTConvolver(Kq, C, workers=-1)
    K = bem.bem_influence(w, w, dx, k, nu)
    for cy, cx in ((n // 4, n // 4), (n // 4, 3 * n // 4), (3 * n // 4, n // 4),
                   (3 * n // 4, 3 * n // 4)):
        hw = h[cy - w // 2: cy + w // 2, cx - w // 2: cx + w // 2].copy()
        hw -= hw.min()
        d = float(np.quantile(hw, 0.1))
        ref = so.solve_nonadhesive(Kq, C, hw, d, tol=1e-12, conv=conv)
        _, res, p, c, _ = bem.bem_solve(K, hw, bem.bem_params_init(d=d, precision=bem.BEM_MIXED))
        err = rel_l2(p, ref.p)
        print(f"[crop {cy},{cx}] mixed rel L2 {err:.3e} contact {c.sum()} vs {ref.contact.sum()}",
              flush=True)
        assert err <= 2e-5
        assert abs(int(c.sum()) - int(ref.contact.sum())) <= max(1, 1e-3 * ref.contact.sum())
        _, res, p, c, _ = bem.bem_solve(K, hw, bem.bem_params_init(d=d))
        assert rel_l2(p, ref.p) <= 1e-10
    K.free()


@pytest.mark.parametrize("k", [-0.5, 0.0, 0.5])
def test_adhesive_512_step_transitions(k):
    # 512^2, side 2, R = 1, nu = 0.3, gamma12 = 2.9995e-3: preload, then the
    # first pull-off steps compared with the oracle's own steps.
    from paper_1612_08395_amd import bem
    n, L, nu, R, gam = 512, 2.0, 0.3, 1.0, 2.9995e-3
    announce("adhesive-512", k)
    dx = L / n
    aF = {-0.5: 0.116, 0.0: 0.213, 0.5: 0.352}[k]
    dj = {-0.5: -0.0198, 0.0: -0.0314, 0.5: -0.0626}[k]
    d0 = (1.5 * aF) ** 2 / ((1 + k) * R)
    dd = (d0 - dj) / 95.0
    h = inputs.parabolic(n, L, R)
    Kq = inf.influence_quarter(n, n, dx, dx, k)
    C = m.compliance(k, nu)
    conv = FFTConvolver(Kq, C, workers=-1)
    pc = m.p_crit(k, nu, gam, dx)
    ref = so.solve_nonadhesive(Kq, C, h, d0, tol=1e-12, conv=conv)
    K = bem.bem_influence(n, n, dx, k, nu)
    st = bem.bem_state_create(K)
    _, res, p, c, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d0), state=st)
    assert rel_l2(p, ref.p) <= 1e-10
    A, pr, d = ref.contact, ref.p, d0
    for s in range(3):
        d -= dd * 8          # jump eight sweep steps at a time
        step = so.adhesive_step(Kq, C, h, d, A, pr, pc, tol=1e-12, conv=conv)
        _, res, p, c, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d, gamma=gam), state=st)
        same = np.array_equal(c.astype(bool), step.contact)
        print(f"[adh-512 k={k}] step {s} d={d:.5f} contact {c.sum()} vs {step.contact.sum()} "
              f"rounds {res.detach_rounds}/{step.rounds}", flush=True)
        if not same:
            assert abs(int(c.sum()) - int(step.contact.sum())) <= max(1, 1e-3 * step.contact.sum())
            break
        assert rel_l2(p, step.p) <= 1e-10
        A, pr = step.contact, step.p
    st.free()
    K.free()


@pytest.mark.parametrize("k", [-0.5, 0.0, 0.5])
def test_adhesive_512_full_sweep_pulloff(k):
    # 100 loading + 100 unloading steps on the GPU (FP64); the smallest force
    # of the sweep against the JKR-type pull-off -(3+k) pi gamma R / 2.
    from paper_1612_08395_amd import bem
    n, L, nu, R, gam = 512, 2.0, 0.3, 1.0, 2.9995e-3
    announce("adhesive-512-sweep", k)
    dx = L / n
    aF = {-0.5: 0.116, 0.0: 0.213, 0.5: 0.352}[k]
    dj = {-0.5: -0.0198, 0.0: -0.0314, 0.5: -0.0626}[k]
    d0 = (1.5 * aF) ** 2 / ((1 + k) * R)
    dd = (d0 - dj) / 95.0
    ds = list(np.linspace(d0 / 100, d0, 100)) + [d0 - dd * (s + 1) for s in range(100)]
    h = inputs.parabolic(n, L, R)
    K = bem.bem_influence(n, n, dx, k, nu)
    _, res = bem.bem_sweep(K, h, bem.bem_params_init(gamma=gam), ds)
    F = np.array([r.F for r in res])
    Fmin = F[100:].min()
    ref = an.jkr_min_force(k, gam, R)
    print(f"[sweep-512 k={k}] Fmin {Fmin:.6e} vs JKR-type {ref:.6e} ratio {Fmin / ref:.4f}; "
          f"final contact {res[-1].n_contact}", flush=True)
    assert res[-1].n_contact == 0                  # pulled off within the sweep
    assert all(r.n_penetrating == 0 for r in res[100:])
    # The mesh-dependent criterion converges about as 1 / (elements across
    # the pull-off radius): the oracle's mesh study at k = -0.5
    # (tests/test_oracle_adhesion.py) bounds the overshoot by 2.1 / (a_F / dx),
    # which is 7.1 %, 3.9 % and 2.3 % at the 30, 55 and 90 elements of this
    # grid for k = -0.5, 0 and 0.5.
    tol = 2.1 / (aF / dx)
    assert Fmin == pytest.approx(ref, rel=tol)
    # loading branch: Hertz-type force at the preload depth
    a = an.hertz_radius(k, R, d0)
    assert res[99].F == pytest.approx(an.hertz_force(k, nu, R, a), rel=1e-2)
    K.free()


@pytest.mark.parametrize("q,gam", [(0, 1e-5), (1, 3e-5), (2, 1e-4), (3, 3e-4)])
def test_rough_4096_adhesive_crops_step_transitions(q, gam):
    # The adhesive rough-surface configuration: the 4096^2 surface (seed
    # 8395, k = -0.3, nu = 0.25) with the work of adhesion swept over
    # {1, 3, 10, 30} 1e-5 E0 L.  A 256^2 window at quadrant centre q, as its
    # own 256^2 problem with the full grid's element size: a non-adhesive load
    # to the depth of 10 % of the window below it, then three pull-off steps
    # (Section 3.1).  Each step is compared as a transition: the GPU state is
    # set to the oracle's previous step (bem_state_set), so both start from
    # the same contact set and pressure and must reach the same new set
    # (counts within 0.1 %, at least one element) and pressure (MIXED 2e-5,
    # FP64 1e-10 relative L2).
    from paper_1612_08395_amd import bem
    n, k, nu, w = 4096, -0.3, 0.25, 256
    announce("adhesive-crops-4096", q, gam)
    h = _rough(n, 0.7, 8.0, 512.0, 8395)
    cy, cx = ((n // 4, n // 4), (n // 4, 3 * n // 4), (3 * n // 4, n // 4),
              (3 * n // 4, 3 * n // 4))[q]
    hw = h[cy - w // 2: cy + w // 2, cx - w // 2: cx + w // 2].copy()
    hw -= hw.min()
    dx = 1.0 / n
    Kq = inf.influence_quarter(w, w, dx, dx, k)
    C = m.compliance(k, nu)
    conv = FFTConvolver(Kq, C, workers=-1)
    pc = m.p_crit(k, nu, gam, dx)
    d0 = float(np.quantile(hw, 0.1))
    load = so.solve_nonadhesive(Kq, C, hw, d0, tol=1e-12, conv=conv)
    K = bem.bem_influence(w, w, dx, k, nu)
    A, pr = load.contact, load.p
    detached = 0
    for s in (1, 2, 3):
        d = d0 * (1.0 - 0.25 * s)
        step = so.adhesive_step(Kq, C, hw, d, A, pr, pc, tol=1e-12, conv=conv)
        for prec, tol in ((bem.BEM_MIXED, 2e-5), (bem.BEM_FP64, 1e-10)):
            st = bem.bem_state_create(K)
            bem.bem_state_set(st, pr, A.astype(np.uint8))
            _, res, p, c, _ = bem.bem_solve(K, hw, bem.bem_params_init(d=d, gamma=gam,
                                                                      precision=prec), state=st)
            st.free()
            cg, co = int(c.sum()), int(step.contact.sum())
            print(f"[adh-crop q={q} gam={gam:g} prec={prec}] step {s} d={d:.4e} contact "
                  f"{A.sum()} -> {cg} (oracle {co}), rounds {res.detach_rounds}/{step.rounds}",
                  flush=True)
            assert res.p_crit == pytest.approx(pc, rel=1e-14)
            assert res.n_penetrating == 0
            assert abs(cg - co) <= max(1, 1e-3 * co)
            if np.array_equal(c.astype(bool), step.contact):
                assert rel_l2(p, step.p) <= tol
        detached += int(A.sum()) - int(step.contact.sum())
        A, pr = step.contact, step.p
    assert detached > 0                            # the steps do pull elements off
    K.free()
