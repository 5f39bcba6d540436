"""GPU contact solves against the FP64 oracle (same seeded inputs)."""
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

FP64_TOL = 1e-10     # relative L2 pressure error, all-FP64 path
MIXED_TOL = 2e-5     # relative L2 pressure error, mixed path


def _bem():
    from paper_1612_08395_amd import bem
    return bem


def _oracle(n, L, k, nu, ny=None, L_y=None):
    ny = ny or n
    dx = L / n
    Kq = inf.influence_quarter(n, ny, dx, dx, k)
    C = m.compliance(k, nu)
    return dx, Kq, C, FFTConvolver(Kq, C, workers=-1)


def _count_close(a, b, frac=1e-3):
    return abs(int(a) - int(b)) <= max(1, frac * max(a, b))


def test_config1_hertz_type_fp64_and_mixed():
    # 128 x 128, side 2, k = 0.5, nu = 0.3, R = 1, d = 0.01, FP64, tol 1e-12
    bem = _bem()
    n, L, k, nu, R, d = 128, 2.0, 0.5, 0.3, 1.0, 0.01
    announce("config1", n, k)
    dx, Kq, C, conv = _oracle(n, L, k, nu)
    h = inputs.parabolic(n, L, R)
    ref = so.solve_nonadhesive(Kq, C, h, d, tol=1e-12, conv=conv)
    K = bem.bem_influence(n, n, dx, k, nu)
    rc, res, p, c, u = bem.bem_solve(K, h, bem.bem_params_init(d=d), want_u=True)
    assert rc == bem.BEM_OK and res.status == 0
    assert rel_l2(p, ref.p) <= FP64_TOL
    assert np.array_equal(c.astype(bool), ref.contact)
    assert res.n_contact == ref.contact.sum()
    assert res.F == pytest.approx(so.force(ref.p, dx, dx), rel=1e-10)
    assert rel_l2(u, ref.u) <= 1e-10
    # closed forms of Section 2.2 (Eq. 15, reading of Eq. 16)
    a = an.hertz_radius(k, R, d)
    assert res.F == pytest.approx(an.hertz_force(k, nu, R, a), rel=2e-2)
    assert abs(math.sqrt(res.area / math.pi) - a) < dx
    # mixed path
    rc, rm, pm, cm, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d, precision=bem.BEM_MIXED))
    assert rm.status in (0, bem.BEM_EFLOOR)
    assert rel_l2(pm, ref.p) <= MIXED_TOL
    assert _count_close(rm.n_contact, ref.contact.sum())
    K.free()


@pytest.mark.parametrize("ny,nx,k,shape", [(37, 50, -0.5, "parabolic"), (64, 64, 0.0, "cone"),
                                           (33, 33, 0.8, "parabolic"), (1, 16, 0.2, "parabolic")])
def test_ragged_and_degenerate_grids(ny, nx, k, shape):
    bem = _bem()
    announce("ragged", ny, nx, k, shape)
    nu, L = 0.3, 1.0
    dx = L / max(nx, ny)
    Kq = inf.influence_quarter(nx, ny, dx, dx, k)
    C = m.compliance(k, nu)
    xs = (np.arange(nx) + 0.5) * dx - 0.45 * L
    ys = (np.arange(ny) + 0.5) * dx - 0.55 * L * ny / max(nx, ny)
    r = np.hypot(xs[None, :], ys[:, None])
    h = r * r / 2.0 if shape == "parabolic" else 0.1 * r
    d = float(np.quantile(h, 0.15))
    ref = so.solve_nonadhesive(Kq, C, h, d, tol=1e-12)
    K = bem.bem_influence(nx, ny, dx, k, nu)
    rc, res, p, c, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d))
    assert rel_l2(p, ref.p) <= FP64_TOL
    assert np.array_equal(c.astype(bool), ref.contact)
    K.free()


@pytest.mark.parametrize("ny,nx,k", [(41, 1300, 0.3), (32, 2048, 0.2), (2100, 48, 0.1)])
def test_wide_and_tall_grids_mixed(ny, nx, k):
    # 1024 < nx <= 2048: the row spectrum has 2048 columns, so the mixed loop
    # runs its C2R sweeps on the wave-FFT kernels (ragged nx, odd ny: a row
    # pair with one row); 2048 < ny <= 4096: the column sweeps run on the
    # quarter-sequence wave kernels (Ly = 4096)
    bem = _bem()
    announce("wide-mixed", ny, nx, k)
    nu, L = 0.3, 1.0
    dx = L / nx
    Kq = inf.influence_quarter(nx, ny, dx, dx, k)
    C = m.compliance(k, nu)
    xs = (np.arange(nx) + 0.5) * dx - 0.5 * L
    ys = (np.arange(ny) + 0.5) * dx - 0.5 * ny * dx
    h = (xs[None, :] ** 2 + 4.0 * ys[:, None] ** 2) / 2.0
    d = float(np.quantile(h, 0.2))
    ref = so.solve_nonadhesive(Kq, C, h, d, tol=1e-12, conv=FFTConvolver(Kq, C, workers=-1))
    K = bem.bem_influence(nx, ny, dx, k, nu)
    _, rm, pm, cm, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d, precision=bem.BEM_MIXED))
    assert rm.status in (0, bem.BEM_EFLOOR)
    assert rel_l2(pm, ref.p) <= MIXED_TOL
    assert _count_close(rm.n_contact, ref.contact.sum())
    K.free()


def test_rows_longer_than_2048():
    # 2048 < nx <= 4096: the CG loop runs 4096-point row transforms (Stockham,
    # 512 threads a row pair, the direction prologue held to 128 VGPRs).
    # Displacement-controlled solves in both precisions, then one pull-off
    # step with adhesion (fixed-set solves; gamma chosen so that one detach
    # round takes 4 elements out of the contact set).
    bem = _bem()
    ny, nx, k, nu, L, gam = 24, 2200, -0.3, 0.25, 1.0, 2.5e-4
    announce("long-rows", ny, nx, k)
    dx = L / nx
    Kq = inf.influence_quarter(nx, ny, dx, dx, k)
    C = m.compliance(k, nu)
    conv = FFTConvolver(Kq, C, workers=-1)
    xs = (np.arange(nx) + 0.5) * dx - 0.5 * L
    ys = (np.arange(ny) + 0.5) * dx - 0.5 * ny * dx
    h = (xs[None, :] ** 2 + 4.0 * ys[:, None] ** 2) / 2.0
    d0 = float(np.quantile(h, 0.3))
    ref = so.solve_nonadhesive(Kq, C, h, d0, tol=1e-12, conv=conv)
    K = bem.bem_influence(nx, ny, dx, k, nu)
    _, rm, pm, cm, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d0, precision=bem.BEM_MIXED))
    assert rm.status in (0, bem.BEM_EFLOOR)
    assert rel_l2(pm, ref.p) <= MIXED_TOL
    assert _count_close(rm.n_contact, ref.contact.sum())
    st = bem.bem_state_create(K)
    _, r64, p64, c64, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d0), state=st)
    assert rel_l2(p64, ref.p) <= FP64_TOL
    assert np.array_equal(c64.astype(bool), ref.contact)
    d1 = 0.8 * d0
    step = so.adhesive_step(Kq, C, h, d1, ref.contact, ref.p, m.p_crit(k, nu, gam, dx),
                            tol=1e-12, conv=conv)
    assert step.rounds == 1 and step.contact.sum() == ref.contact.sum() - 4
    _, ra, pa, ca, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d1, gamma=gam), state=st)
    assert ra.detach_rounds == step.rounds
    assert np.array_equal(ca.astype(bool), step.contact)
    assert rel_l2(pa, step.p) <= FP64_TOL
    st.free()
    K.free()


def test_no_contact_and_full_contact():
    bem = _bem()
    announce("degenerate-contact")
    n, L, k, nu = 32, 1.0, 0.3, 0.3
    dx, Kq, C, conv = _oracle(n, L, k, nu)
    K = bem.bem_influence(n, n, dx, k, nu)
    h = inputs.parabolic(n, L, 1.0)
    # indenter above the surface: no contact, zero pressure
    rc, res, p, c, _ = bem.bem_solve(K, h + 0.01, bem.bem_params_init(d=0.0))
    assert res.n_contact == 0 and np.all(p == 0) and res.F == 0.0
    # flat rigid plane pushed in everywhere: whole grid in contact
    flat = np.zeros((n, n))
    ref = so.solve_nonadhesive(Kq, C, flat, 1e-3, tol=1e-12, conv=conv)
    rc, res, p, c, _ = bem.bem_solve(K, flat, bem.bem_params_init(d=1e-3))
    assert res.n_contact == n * n == ref.contact.sum()
    assert rel_l2(p, ref.p) <= FP64_TOL
    K.free()


def test_warm_start_state_roundtrip_and_sweep():
    bem = _bem()
    announce("warm-start")
    n, L, k, nu, R = 96, 1.0, -0.3, 0.25, 1.0
    dx, Kq, C, conv = _oracle(n, L, k, nu)
    h = inputs.parabolic(n, L, R)
    K = bem.bem_influence(n, n, dx, k, nu)
    st = bem.bem_state_create(K)
    ds = [0.004, 0.008, 0.012]
    refs = [so.solve_nonadhesive(Kq, C, h, d, tol=1e-12, conv=conv) for d in ds]
    iters = []
    for d, ref in zip(ds, refs):
        rc, res, p, c, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d), state=st)
        assert rel_l2(p, ref.p) <= FP64_TOL
        iters.append(res.iters)
    # export / import of the state
    p_s, c_s = bem.bem_state_get(st)
    assert rel_l2(p_s, refs[-1].p) <= FP64_TOL
    st2 = bem.bem_state_create(K)
    bem.bem_state_set(st2, p_s, c_s)
    rc, res2, p2, c2, _ = bem.bem_solve(K, h, bem.bem_params_init(d=ds[-1]), state=st2)
    assert rel_l2(p2, refs[-1].p) <= FP64_TOL
    assert res2.iters <= 2
    # the sweep entry point gives the same forces
    rc, sw = bem.bem_sweep(K, h, bem.bem_params_init(), ds)
    for r, ref in zip(sw, refs):
        assert r.F == pytest.approx(so.force(ref.p, dx, dx), rel=1e-10)
    st.free()
    st2.free()
    K.free()


@pytest.mark.parametrize("chains", [1, 2, 3])
def test_sweep_dev_concurrent_chains(chains):
    # bem_sweep_dev: h read on the device, steps split over concurrent
    # warm-start chains; every step against the oracle, and the caller's
    # state left with the last step's solution
    import torch
    bem = _bem()
    announce("sweep-dev", chains)
    n, L, k, nu = 96, 1.0, 0.4, 0.3
    dx, Kq, C, conv = _oracle(n, L, k, nu)
    h = inputs.fractal_gap(n, L, 0.8, 4 * 2 * math.pi / L, 32 * 2 * math.pi / L, 1e-3 * L, 77)
    ds = [float(np.quantile(h, q)) for q in (0.02, 0.04, 0.06, 0.08, 0.10, 0.12, 0.14)]
    refs = [so.solve_nonadhesive(Kq, C, h, d, tol=1e-12, conv=conv) for d in ds]
    K = bem.bem_influence(n, n, dx, k, nu)
    h_dev = torch.tensor(h, dtype=torch.float64, device="cuda")
    st = bem.bem_state_create(K)
    rc, sw = bem.bem_sweep_dev(K, h_dev, bem.bem_params_init(), ds, chains=chains, state=st)
    assert rc == 0
    for r, ref in zip(sw, refs):
        assert r.status == 0
        assert r.F == pytest.approx(so.force(ref.p, dx, dx), rel=1e-10)
        assert r.n_contact == int(ref.contact.sum())
    p_s, c_s = bem.bem_state_get(st)
    assert rel_l2(p_s, refs[-1].p) <= FP64_TOL
    assert np.array_equal(c_s.astype(bool), refs[-1].contact)
    # mixed precision through the same chains
    rc, swm = bem.bem_sweep_dev(K, h_dev, bem.bem_params_init(precision=bem.BEM_MIXED), ds,
                                chains=chains)
    for r, ref in zip(swm, refs):
        assert r.status in (0, bem.BEM_EFLOOR)
        assert r.F == pytest.approx(so.force(ref.p, dx, dx), rel=2e-5)
        assert _count_close(r.n_contact, ref.contact.sum())
    st.free()
    K.free()


def test_sweep_state_from_another_profile():
    # Sweep steps after the first start from the previous step's gap shifted
    # to the new depth.  A state whose last solve was on another gap profile
    # must not hand its gap to a sweep: every step against the oracle, in
    # both precisions, then a second sweep on the same state.
    bem = _bem()
    announce("sweep-other-profile")
    n, L, k, nu = 80, 1.0, 0.2, 0.3
    dx, Kq, C, conv = _oracle(n, L, k, nu)
    h = inputs.parabolic(n, L, 1.0)
    h2 = inputs.fractal_gap(n, L, 0.7, 4 * 2 * math.pi / L, 20 * 2 * math.pi / L, 1e-3 * L, 5)
    ds = [0.002, 0.004, 0.006, 0.008]
    refs = [so.solve_nonadhesive(Kq, C, h, d, tol=1e-12, conv=conv) for d in ds]
    K = bem.bem_influence(n, n, dx, k, nu)
    for prec, tol in ((bem.BEM_FP64, FP64_TOL), (bem.BEM_MIXED, MIXED_TOL)):
        st = bem.bem_state_create(K)
        d2 = float(np.quantile(h2, 0.1))
        bem.bem_solve(K, h2, bem.bem_params_init(d=d2, precision=prec), state=st)
        for _ in range(2):
            rc, sw = bem.bem_sweep(K, h, bem.bem_params_init(precision=prec), ds, state=st)
            for r, ref in zip(sw, refs):
                assert r.status in (0, bem.BEM_EFLOOR)
                assert r.F == pytest.approx(so.force(ref.p, dx, dx), rel=max(tol, 1e-10))
                assert _count_close(r.n_contact, ref.contact.sum())
        p_s, _ = bem.bem_state_get(st)
        assert rel_l2(p_s, refs[-1].p) <= tol
        st.free()
    K.free()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_sweep_matches_separate_warm_solves(prec):
    # A sweep step takes its first gap from the previous step's (a shift by
    # the change of d); separate bem_solve calls on a warm state recompute it
    # by convolution.  Same pressures (to rounding) and iteration counts.
    bem = _bem()
    announce("sweep-vs-solves", prec)
    precision = bem.BEM_FP64 if prec == "fp64" else bem.BEM_MIXED
    n, L, k, nu = 128, 1.0, 0.3, 0.3
    dx = L / n
    h = inputs.fractal_gap(n, L, 0.7, 4 * 2 * math.pi / L, 32 * 2 * math.pi / L, 1e-3 * L, 41)
    ds = [float(np.quantile(h, q)) for q in (0.02, 0.04, 0.06, 0.08, 0.10)]
    K = bem.bem_influence(n, n, dx, k, nu)
    st = bem.bem_state_create(K)
    rc, sw = bem.bem_sweep(K, h, bem.bem_params_init(precision=precision), ds, state=st)
    p_sweep, _ = bem.bem_state_get(st)
    st2 = bem.bem_state_create(K)
    for d, r in zip(ds, sw):
        _, res, p, c, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d, precision=precision),
                                        state=st2)
        assert abs(res.iters - r.iters) <= 1
        assert res.n_contact == r.n_contact if prec == "fp64" else _count_close(res.n_contact,
                                                                                r.n_contact)
        assert res.F == pytest.approx(r.F, rel=1e-12 if prec == "fp64" else 1e-6)
    assert rel_l2(p, p_sweep) <= (1e-12 if prec == "fp64" else 1e-6)
    st.free()
    st2.free()
    K.free()


def test_sweep_dev_argument_errors():
    import torch
    bem = _bem()
    announce("sweep-dev-errors")
    n = 32
    K = bem.bem_influence(n, n, 1.0 / n, 0.0, 0.3)
    h_dev = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    for chains in (0, 9):
        with pytest.raises(bem.BemError):
            bem.bem_sweep_dev(K, h_dev, bem.bem_params_init(), [0.01], chains=chains)
    with pytest.raises(bem.BemError):   # adhesive sweeps depend on their path
        bem.bem_sweep_dev(K, h_dev, bem.bem_params_init(gamma=1e-3), [0.01, 0.0], chains=2)
    with pytest.raises(bem.BemError):
        bem.bem_sweep_dev(K, h_dev, bem.bem_params_init(), [0.01, float("nan")], chains=2)
    K.free()


def test_adhesive_step_transitions_parity():
    # Section 3.1: non-adhesive preload, then pull-off steps with the
    # detachment criterion; each step compared with the oracle's own step.
    bem = _bem()
    announce("adhesive-transitions")
    n, L, k, nu, R, gam = 96, 1.0, 0.5, 0.3, 1.0, 5e-4
    dx, Kq, C, conv = _oracle(n, L, k, nu)
    h = inputs.parabolic(n, L, R)
    pc = m.p_crit(k, nu, gam, dx)
    assert bem.bem_p_crit(k, nu, gam, dx) == pytest.approx(pc, rel=1e-14)
    d0 = 0.02
    ref = so.solve_nonadhesive(Kq, C, h, d0, tol=1e-12, conv=conv)
    K = bem.bem_influence(n, n, dx, k, nu)
    st = bem.bem_state_create(K)
    rc, res, p, c, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d0), state=st)
    assert rel_l2(p, ref.p) <= FP64_TOL
    A, pr = ref.contact, ref.p
    compared = 0
    d = d0
    for s in range(12):
        d -= 0.004
        step = so.adhesive_step(Kq, C, h, d, A, pr, pc, tol=1e-12, conv=conv)
        rc, res, p, c, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d, gamma=gam), state=st)
        assert res.p_crit == pytest.approx(pc, rel=1e-14)
        if not np.array_equal(c.astype(bool), step.contact):
            # a near-tie detachment decision: compare counts only, then stop
            assert _count_close(res.n_contact, step.contact.sum())
            break
        assert rel_l2(p, step.p) <= FP64_TOL
        assert res.F == pytest.approx(so.force(step.p, dx, dx), rel=1e-9, abs=1e-12)
        assert np.all(-p[c.astype(bool)] <= pc * (1 + 1e-12))
        assert res.n_penetrating == 0
        compared += 1
        A, pr = step.contact, step.p
        if not A.any():
            break
    assert compared >= 5
    st.free()
    K.free()


def test_solver_clock_accounts_every_launch():
    """The solver clock sees six launches per CG iteration: all six for the
    iterations worked on, the first three at the stopping iteration (the
    direction kernel there only takes the decision), and every launch queued
    after it as skipped."""
    bem = _bem()
    announce("solver-clock")
    n = 64
    K = bem.bem_influence(n, n, 1.0 / n, 0.3, 0.3)
    h = inputs.parabolic(n, 1.0, 1.0)
    total = 0
    bem.bem_clock_start()
    for d in (0.002, 0.004):
        _, res, _, _, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d, precision=bem.BEM_MIXED))
        total += res.iters
    c = bem.bem_clock_stop()
    K.free()
    assert c.iterations == total
    assert list(c.launches) == [total + 2] * 3 + [total] * 3
    assert c.skipped % 6 == 0 and c.skipped >= 6   # two solves, three skipped at each stop
    assert all(x > 0 for x in c.ms)


def test_error_paths():
    bem = _bem()
    announce("errors")
    K = bem.bem_influence_ex(16, 16, 0.1, 0.12, 0.3, 0.3)
    h = np.zeros((16, 16))
    with pytest.raises(bem.BemError) as e:      # force control is non-adhesive only
        bem.bem_solve(K, h, bem.bem_params_init(control=bem.BEM_CTRL_FORCE, F=1.0, gamma=1e-3))
    assert e.value.code == bem.BEM_EUNSUPPORTED
    with pytest.raises(bem.BemError) as e:
        bem.bem_solve(K, h, bem.bem_params_init(control=bem.BEM_CTRL_FORCE, F=-1.0))
    assert e.value.code == bem.BEM_EINVAL
    with pytest.raises(bem.BemError) as e:      # adhesion on non-square elements
        bem.bem_solve(K, h, bem.bem_params_init(d=0.01, gamma=1e-3))
    assert e.value.code == bem.BEM_EUNSUPPORTED
    hb = h.copy()
    hb[3, 4] = np.nan
    with pytest.raises(bem.BemError) as e:
        bem.bem_solve(K, hb, bem.bem_params_init(d=0.01))
    assert e.value.code == bem.BEM_EINVAL
    with pytest.raises(bem.BemError) as e:
        bem.bem_solve(K, h, bem.bem_params_init(d=float("inf")))
    assert e.value.code == bem.BEM_EINVAL
    # iteration limit: warning status, last iterate returned
    Kq = bem.bem_influence(64, 64, 1 / 64, 0.0, 0.3)
    rc, res, p, c, _ = bem.bem_solve(Kq, inputs.parabolic(64, 1.0, 1.0),
                                     bem.bem_params_init(d=0.01, max_iter=3))
    assert rc == bem.BEM_ENOCONV and res.status == bem.BEM_ENOCONV and res.iters == 3
    assert np.all(np.isfinite(p))
    K.free()
    Kq.free()


@pytest.mark.parametrize("k", [0.05, -0.35, 0.75, -0.87, 0.5])
def test_library_c1_and_p_crit_match_oracle(k):
    # Table 1 between its entries (natural cubic spline of ln c1) and Eq. 24:
    # the library's own C implementation against the oracle's scipy spline.
    bem = _bem()
    announce("c1/p_crit", k)
    assert bem.bem_c1(k) == pytest.approx(m.c1_corrected(k), rel=1e-14)
    for nu, gam, dx, E0, c0 in ((0.3, 2e-3, 1 / 256, 1.0, 1.0), (0.25, 7e-5, 0.013, 2.5, 0.6)):
        assert bem.bem_p_crit(k, nu, gam, dx, E0, c0) == pytest.approx(
            m.p_crit(k, nu, gam, dx, E0=E0, c0=c0), rel=1e-14)


def test_adhesive_step_at_off_table_k():
    # k = 0.35 lies between Table 1 entries, so p_crit comes from the spline
    # branch of both sides (library: bem_p_crit inside bem_solve; oracle:
    # c1_corrected); c0 != 1 enters through C and c0^k in Eq. 24.
    bem = _bem()
    n, L, k, nu, R, gam, c0 = 96, 1.0, 0.35, 0.3, 1.0, 3e-5, 0.7
    announce("adhesive-off-table", n, k)
    dx = L / n
    Kq = inf.influence_quarter(n, n, dx, dx, k)
    C = m.compliance(k, nu, c0=c0)
    conv = FFTConvolver(Kq, C, workers=-1)
    h = inputs.parabolic(n, L, R)
    pc = m.p_crit(k, nu, gam, dx, c0=c0)
    load = so.solve_nonadhesive(Kq, C, h, 0.015, tol=1e-12, conv=conv)
    step = so.adhesive_step(Kq, C, h, 0.005, load.contact, load.p, pc, tol=1e-12, conv=conv)
    assert step.rounds >= 2 and 0 < step.contact.sum() < load.contact.sum()
    K = bem.bem_influence_ex(n, n, dx, dx, k, nu, 1.0, c0)
    st = bem.bem_state_create(K)
    bem.bem_solve(K, h, bem.bem_params_init(d=0.015), state=st)
    _, res, p, c, _ = bem.bem_solve(K, h, bem.bem_params_init(d=0.005, gamma=gam), state=st)
    assert res.p_crit == pytest.approx(pc, rel=1e-14)
    assert np.array_equal(c.astype(bool), step.contact)
    assert rel_l2(p, step.p) <= FP64_TOL
    assert res.detach_rounds == step.rounds
    st.free()
    K.free()
