"""Pins of oracle/solver.py: contact-mechanics facts that do not depend on
how the oracle is written (KKT conditions, uniqueness, symmetry, Hertz,
Boussinesq, the Hertz-type and flat-punch closed forms of the paper)."""
import math

import numpy as np
import pytest

from oracle import analytic as an
from oracle import influence as inf
from oracle import material as m
from oracle import solver as so
from oracle.convolution import FFTConvolver, conv_direct
from paper_1612_08395_amd import inputs


def _setup(n, L, k, nu=0.3):
    dx = L / n
    Kq = inf.influence_quarter(n, n, dx, dx, k)
    C = m.compliance(k, nu)
    return dx, Kq, C


@pytest.mark.parametrize("k", [-0.5, 0.3])
def test_kkt_with_direct_sum_residual(k):
    n, L, R, d = 40, 1.0, 1.0, 0.03
    dx, Kq, C = _setup(n, L, k)
    h = inputs.parabolic(n, L, R)
    res = so.solve_nonadhesive(Kq, C, h, d, tol=1e-13)
    assert res.converged
    p = res.p
    g = conv_direct(Kq, p, C) + h - d          # independent residual
    scale = d
    assert p.min() >= 0.0
    assert g.min() >= -1e-10 * scale            # no interpenetration
    assert np.max(np.abs(g[p > 0])) <= 1e-10 * scale   # closed gap in contact
    assert np.sum(p * np.abs(g)) <= 1e-10 * scale * np.sum(p)
    assert 50 < np.count_nonzero(p) < n * n / 2


def test_cold_and_warm_start_agree():
    n, L, R, d, k = 64, 1.0, 1.0, 0.02, 0.2
    dx, Kq, C = _setup(n, L, k)
    h = inputs.parabolic(n, L, R)
    a = so.solve_nonadhesive(Kq, C, h, d, tol=1e-13)
    rng = np.random.default_rng(0)
    warm = a.p * (1.0 + 0.5 * rng.random(a.p.shape)) + 0.1 * rng.random(a.p.shape) * a.p.max()
    b = so.solve_nonadhesive(Kq, C, h, d, tol=1e-13, p_init=warm)
    assert np.linalg.norm(a.p - b.p) <= 1e-10 * np.linalg.norm(a.p)
    assert np.array_equal(a.contact, b.contact)


def test_fourfold_symmetry():
    n, L, R, d, k = 64, 1.0, 1.0, 0.02, -0.3
    dx, Kq, C = _setup(n, L, k)
    p = so.solve_nonadhesive(Kq, C, inputs.parabolic(n, L, R), d, tol=1e-13).p
    for q in (p[::-1, :], p[:, ::-1], p.T):
        assert np.max(np.abs(q - p)) <= 1e-10 * p.max()


def test_hertz_k0():
    # Classical Hertz: a = sqrt(R d), F = 4 E* a^3 / (3 R).
    n, L, R, d, nu = 128, 2.0, 1.0, 0.01, 0.3
    dx, Kq, C = _setup(n, L, 0.0, nu)
    res = so.solve_nonadhesive(Kq, C, inputs.parabolic(n, L, R), d)
    F = so.force(res.p, dx, dx)
    a = math.sqrt(R * d)
    Estar = 1.0 / (1 - nu * nu)
    assert F == pytest.approx(4 * Estar * a ** 3 / (3 * R), rel=3e-3)
    a_num = math.sqrt(res.contact.sum() * dx * dx / math.pi)
    assert abs(a_num - a) < dx


@pytest.mark.parametrize("k", [-0.5, 0.5, 0.8])
def test_hertz_type_power_law(k):
    # Section 2.2: a from Eq. 15, F from the reading of Eq. 16.
    n, L, R, d, nu = 128, 2.0, 1.0, 0.01, 0.3
    dx, Kq, C = _setup(n, L, k, nu)
    res = so.solve_nonadhesive(Kq, C, inputs.parabolic(n, L, R), d)
    a = an.hertz_radius(k, R, d)
    F = so.force(res.p, dx, dx)
    assert F == pytest.approx(an.hertz_force(k, nu, R, a), rel=1e-2)
    # the printed Eq. 16 is far off, which is why the reading is needed
    assert abs(F / an.hertz_force_printed(k, nu, R, a) - 1) > 1.0
    a_num = math.sqrt(res.contact.sum() * dx * dx / math.pi)
    assert abs(a_num - a) < dx


@pytest.mark.parametrize("k", [-0.5, 0.0, 0.5])
def test_exterior_displacement_eq14(k):
    # Eq. 14 (free of alpha): surface deflection outside the contact.
    n, L, R, d, nu = 128, 2.0, 1.0, 0.01, 0.3
    dx, Kq, C = _setup(n, L, k, nu)
    res = so.solve_nonadhesive(Kq, C, inputs.parabolic(n, L, R), d)
    r = inputs.radius(n, L)
    a = an.hertz_radius(k, R, d)
    ring = (r > 1.3 * a) & (r < 3.0 * a)
    ref = an.hertz_uz(r[ring], a, R, k)
    assert np.max(np.abs(res.u[ring] - ref)) <= 1.5e-2 * d


@pytest.mark.parametrize("k", [-0.5, 0.0, 0.5])
def test_flat_punch_stiffness(k):
    # Rigid flat circular punch: F / d = 2 E0 a^(1+k) / (X (1+k)(1-nu^2) c0^k)
    # (Boussinesq's 2 E* a at k = 0), with a the radius of a disk of the same
    # area as the discrete punch.
    n, L, nu, a = 96, 1.0, 0.3, 0.25
    dx, Kq, C = _setup(n, L, k, nu)
    h = inputs.flat_punch(n, L, a)
    A = h == 0.0
    res = so.solve_fixed_set(Kq, C, h, 1e-3, A)
    a_eq = math.sqrt(A.sum() * dx * dx / math.pi)
    kfp = so.force(res.p, dx, dx) / 1e-3
    assert kfp == pytest.approx(an.flat_punch_stiffness(k, nu, a_eq), rel=1.5e-2)


def test_fixed_set_solution_properties():
    # p = 0 off A, u = d - h on A (to tolerance), tensile pressure allowed.
    n, L, R, k = 48, 1.0, 1.0, 0.2
    dx, Kq, C = _setup(n, L, k)
    h = inputs.parabolic(n, L, R)
    A = inputs.radius(n, L) < 0.15
    d = 0.005                                   # smaller than the Hertz depth for A
    res = so.solve_fixed_set(Kq, C, h, d, A, tol=1e-13)
    assert np.all(res.p[~A] == 0)
    g = conv_direct(Kq, res.p, C) + h - d
    assert np.max(np.abs(g[A])) <= 1e-10 * d
    assert res.p.min() < 0                      # edge is in tension


def test_adhesive_detach_loop_invariants():
    n, L, R, k, nu, gam = 64, 1.0, 1.0, 0.0, 0.3, 2e-4
    dx, Kq, C = _setup(n, L, k, nu)
    conv = FFTConvolver(Kq, C)
    h = inputs.parabolic(n, L, R)
    pc = m.p_crit(k, nu, gam, dx)
    load = so.solve_nonadhesive(Kq, C, h, 0.02, conv=conv)
    step = so.adhesive_step(Kq, C, h, 0.0, load.contact, load.p, pc, conv=conv)
    A = step.contact
    assert A.sum() < load.contact.sum()          # some elements detached
    assert np.all(A <= load.contact)             # the set only shrinks
    assert np.all(-step.p[A] <= pc)              # criterion met on A
    assert np.all(step.p[~A] == 0)
    assert step.g[~A].min() >= -1e-10            # no penetration off A
    assert step.rounds >= 1


def test_flat_punch_pulloff_k0_kendall():
    # Adhesive flat punch, k = 0 (Section 3.2, Eqs. 25-26 at k = 0 are
    # Kendall's F = sqrt(8 pi gamma E* a^3)).  Pull from d = 0 in small
    # steps; the largest tensile force before complete detachment is
    # compared to the closed form (mesh criterion, within a few percent).
    n, L, a, nu, gam = 96, 1.0, 0.25, 0.3, 1e-3
    dx, Kq, C = _setup(n, L, 0.0, nu)
    conv = FFTConvolver(Kq, C)
    h = inputs.flat_punch(n, L, a)
    A = h == 0.0
    a_eq = math.sqrt(A.sum() * dx * dx / math.pi)
    Fc = an.flat_punch_Fcrit(0.0, nu, gam, a_eq)
    dc = an.flat_punch_dcrit(0.0, nu, gam, a_eq)
    pc = m.p_crit(0.0, nu, gam, dx)
    p = np.zeros_like(h)
    Fmin = 0.0
    for s in range(1, 200):
        d = -dc * s / 100.0
        st = so.adhesive_step(Kq, C, h, d, A, p, pc, tol=1e-10, conv=conv)
        A, p = st.contact, st.p
        Fmin = min(Fmin, so.force(p, dx, dx))
        if not A.any():
            break
    assert not A.any()
    assert -Fmin == pytest.approx(Fc, rel=0.05)


# ---- load control ------------------------------------------------------------

@pytest.mark.parametrize("k", [-0.4, 0.3])
def test_force_control_kkt_with_direct_sum_residual(k):
    n, L, R = 40, 1.0, 1.0
    dx, Kq, C = _setup(n, L, k)
    h = inputs.parabolic(n, L, R)
    W = 6e-3
    res = so.solve_force(Kq, C, h, W, dx, dx, tol=1e-13)
    assert res.converged
    p, d = res.p, res.d
    assert so.force(p, dx, dx) == pytest.approx(W, rel=1e-13)   # the load constraint
    g = conv_direct(Kq, p, C) + h - d          # independent residual, d from the solve
    assert p.min() >= 0.0
    assert g.min() >= -1e-10 * d
    assert np.max(np.abs(g[p > 0])) <= 1e-10 * d
    assert 40 < np.count_nonzero(p) < n * n / 2


def test_force_control_hertz_k0():
    # Classical Hertz under a given load: a = (3 F R / (4 E*))^(1/3), d = a^2 / R.
    n, L, R, nu = 128, 2.0, 1.0, 0.3
    dx, Kq, C = _setup(n, L, 0.0, nu)
    Estar = 1.0 / (1 - nu * nu)
    a = 0.1
    W = 4 * Estar * a ** 3 / (3 * R)
    res = so.solve_force(Kq, C, inputs.parabolic(n, L, R), W, dx, dx)
    assert res.d == pytest.approx(a * a / R, rel=3e-3)
    a_num = math.sqrt(res.contact.sum() * dx * dx / math.pi)
    assert abs(a_num - a) < dx


@pytest.mark.parametrize("k", [-0.5, 0.5])
def test_force_control_hertz_type_power_law(k):
    # load from the reading of Eq. 16 at radius a; indentation from Eq. 15
    n, L, R, nu = 128, 2.0, 1.0, 0.3
    dx, Kq, C = _setup(n, L, k, nu)
    a = 0.1
    W = an.hertz_force(k, nu, R, a)
    res = so.solve_force(Kq, C, inputs.parabolic(n, L, R), W, dx, dx)
    assert res.d == pytest.approx(a * a / ((1 + k) * R), rel=1e-2)
    a_num = math.sqrt(res.contact.sum() * dx * dx / math.pi)
    assert abs(a_num - a) < dx


def test_force_and_displacement_control_agree():
    # the solution is unique: the load of a displacement-controlled solve,
    # prescribed, gives back its pressure and indentation
    n, L, k = 64, 1.0, 0.2
    dx, Kq, C = _setup(n, L, k)
    h = inputs.fractal_gap(n, L, 0.7, 4 * 2 * math.pi, 16 * 2 * math.pi, 1e-3, 11)
    d = float(np.quantile(h, 0.08))
    a = so.solve_nonadhesive(Kq, C, h, d, tol=1e-13)
    b = so.solve_force(Kq, C, h, so.force(a.p, dx, dx), dx, dx, tol=1e-13)
    assert b.d == pytest.approx(d, rel=1e-9)
    assert np.linalg.norm(a.p - b.p) <= 1e-8 * np.linalg.norm(a.p)
    assert np.array_equal(a.contact, b.contact)


def test_force_control_zero_load():
    n, L = 16, 1.0
    dx, Kq, C = _setup(n, L, 0.0)
    res = so.solve_force(Kq, C, inputs.parabolic(n, L, 1.0), 0.0, dx, dx)
    assert not res.p.any() and res.converged
