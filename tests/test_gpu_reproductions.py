"""Section 3.2 and 2.2 examples reproduced on the GPU against the closed forms
(the figure data itself is not published): flat-punch pull-off (Eqs. 25, 26,
Fig. 6), square punch in four orientations (Fig. 10), the Hertz-type
k-sweep at 512^2 (Eqs. 15, 16, Fig. 3), mesh independence of the
adhesive pull-off (256^2 vs 1024^2, Fig. 7), its independence of R / c0
(Fig. 8a), and Table 1 refitted from BEM pull-offs at every other tabulated k
(Section 3.1, Fig. 5)."""
import math

import numpy as np
import pytest

from oracle import analytic as an
from paper_1612_08395_amd import inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

NU, GAMMA = 0.3, 1e-3


def _punch_pulloff(bem, n, L, k, h, dref, max_steps=300):
    """Adhesive flat-stamp pull-off from zero indentation: the contact set
    starts as the stamp face and d decreases in steps of dref / 100.
    Returns forces, contact counts and depths, up to complete detachment."""
    K = bem.bem_influence(n, n, L / n, k, NU)
    st = bem.bem_state_create(K)
    bem.bem_state_set(st, None, (h == 0.0).astype(np.uint8))
    F, c, d = [], [], []
    for s in range(1, max_steps):
        ds = -dref * s / 100.0
        _, res, _, _, _ = bem.bem_solve(K, h, bem.bem_params_init(d=ds, gamma=GAMMA), state=st)
        assert res.n_penetrating == 0
        F.append(res.F)
        c.append(res.n_contact)
        d.append(ds)
        if res.n_contact == 0:
            break
    st.free()
    K.free()
    return np.array(F), np.array(c), np.array(d)


@pytest.mark.parametrize("k", [-0.5, 0.3])
def test_flat_punch_pulloff_eqs_25_26(k):
    """A flat cylindrical punch keeps its contact radius during pull-off and
    detaches at d_crit (Eq. 25) with the force F_crit (Eq. 26, read with X in
    the denominator); the mesh-dependent criterion (Eq. 24, Table 1) has to
    reproduce both.  a* = 0.25 L on 512^2 (128 elements across the radius);
    the step is d_crit / 100."""
    from paper_1612_08395_amd import bem
    announce(f"flat-punch k={k}")
    n, L, a = 512, 1.0, 0.25
    h = inputs.flat_punch(n, L, a)
    area = int((h == 0).sum())
    a_eq = math.sqrt(area * (L / n) ** 2 / math.pi)
    dc = an.flat_punch_dcrit(k, NU, GAMMA, a_eq)
    Fc = an.flat_punch_Fcrit(k, NU, GAMMA, a_eq)
    F, c, d = _punch_pulloff(bem, n, L, k, h, dc)
    assert c[-1] == 0                                   # pulled off
    assert -F.min() == pytest.approx(Fc, rel=0.01)
    assert 1.0 <= -d[-1] / dc <= 1.02                   # detaches within one step after d_crit
    assert c[-2] >= 0.98 * area                         # radius unchanged until then
    assert -d[int(np.argmin(F))] / dc == pytest.approx(1.0, abs=0.011)


def test_square_punch_orientation_independence():
    """Square punch (half side 0.2 L) at 0, 15, 30 and 45 degrees to the grid,
    k = 0.3, 512^2 (Fig. 10): the pull-off force does not depend on the
    orientation.  Normalised by the inscribed cylinder (radius = half side),
    it lies between 1 and the ratio for a cylinder of the square's area."""
    from paper_1612_08395_amd import bem
    announce("square-punch")
    n, L, k, s = 512, 1.0, 0.3, 0.2
    dc = an.flat_punch_dcrit(k, NU, GAMMA, s)
    Fc = an.flat_punch_Fcrit(k, NU, GAMMA, s)
    ratios = []
    for ang in (0, 15, 30, 45):
        h = inputs.square_punch(n, L, s, ang)
        F, c, _ = _punch_pulloff(bem, n, L, k, h, dc)
        assert c[-1] == 0
        ratios.append(-F.min() / Fc)
    ratios = np.array(ratios)
    print("[square punch] F_min / F_crit(inscribed):", np.round(ratios, 4), flush=True)
    assert ratios.max() / ratios.min() - 1.0 < 0.02
    equal_area = (2.0 / math.sqrt(math.pi)) ** ((3.0 + k) / 2.0)   # F_crit ~ a^((3+k)/2)
    assert np.all((ratios > 1.0) & (ratios < equal_area))


def test_hertz_type_k_sweep_512():
    """Non-adhesive parabolic indentation at 512^2 (side 2, R = 1, d = 0.01)
    for k from -0.8 to 0.8: force from the reading of Eq. 16 and contact
    radius from Eq. 15."""
    from paper_1612_08395_amd import bem
    announce("hertz-k-sweep")
    n, L, R, d = 512, 2.0, 1.0, 0.01
    dx = L / n
    h = inputs.parabolic(n, L, R)
    for k in (-0.8, -0.4, 0.0, 0.4, 0.8):
        K = bem.bem_influence(n, n, dx, k, NU)
        _, res, _, _, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d))
        K.free()
        a = an.hertz_radius(k, R, d)
        assert res.F == pytest.approx(an.hertz_force(k, NU, R, a), rel=1e-3)
        assert abs(math.sqrt(res.n_contact * dx * dx / math.pi) - a) < dx


def test_mesh_independence_of_pulloff():
    """Parabolic JKR-type pull-off, k = 0.5, side 2, R = 1, at 256^2 and
    1024^2 (Fig. 7): both meshes give the closed-form pull-off force
    -(3+k) pi gamma R / 2 and agree with each other."""
    from paper_1612_08395_amd import bem
    announce("mesh-independence")
    k, L, R, gam = 0.5, 2.0, 1.0, 2.9995e-3
    aF, dj = 0.352, -0.0626
    d0 = (1.5 * aF) ** 2 / ((1 + k) * R)
    dd = (d0 - dj) / 95.0
    ds = list(np.linspace(d0 / 100, d0, 100)) + [d0 - dd * (s + 1) for s in range(100)]
    ref = an.jkr_min_force(k, gam, R)
    Fmin = {}
    for n in (256, 1024):
        K = bem.bem_influence(n, n, L / n, k, NU)
        _, res = bem.bem_sweep(K, inputs.parabolic(n, L, R), bem.bem_params_init(gamma=gam), ds)
        K.free()
        assert res[-1].n_contact == 0
        Fmin[n] = min(r.F for r in res[100:])
    print(f"[mesh] Fmin/ref 256: {Fmin[256] / ref:.4f}, 1024: {Fmin[1024] / ref:.4f}", flush=True)
    assert Fmin[256] == pytest.approx(ref, rel=0.02)
    assert Fmin[1024] == pytest.approx(ref, rel=0.005)
    assert Fmin[256] == pytest.approx(Fmin[1024], rel=0.02)


def _jkr_points(k, nu, gam, R, c0=1.0):
    """Pull-off radius a_F (force minimum) and jump-off depth d_j (indentation
    minimum) of the JKR-type closed form, which set up the sweeps below."""
    from scipy import optimize
    opt = {"xatol": 1e-12}
    aF = optimize.minimize_scalar(lambda a: an.jkr_curve(k, nu, gam, R, a, 1.0, c0)[1],
                                  bounds=(1e-6, 10.0), method="bounded", options=opt).x
    aj = optimize.minimize_scalar(lambda a: an.jkr_curve(k, nu, gam, R, a, 1.0, c0)[0],
                                  bounds=(1e-6, 10.0), method="bounded", options=opt).x
    return aF, an.jkr_curve(k, nu, gam, R, aj, 1.0, c0)[0]


def _pulloff_sweep(bem, K, h, k, R, aF, dj, prm, no_penetration=True):
    """Preload to (1.5 a_F)^2 / ((1+k) R), then 100 pull-off steps of
    (d0 - d_j) / 95; returns the smallest force and the step results."""
    d0 = (1.5 * aF) ** 2 / ((1 + k) * R)
    dd = (d0 - dj) / 95.0
    ds = [d0] + [d0 - dd * (s + 1) for s in range(100)]
    _, res = bem.bem_sweep(K, h, prm, ds)
    assert res[-1].n_contact == 0                  # pulled off within the sweep
    if no_penetration:
        assert all(r.n_penetrating == 0 for r in res[1:])
    return min(r.F for r in res[1:]), res


# fitted c1 / Table 1 value at each tabulated k (filled in by the test below)
C1_FIT = {}


@pytest.mark.parametrize("k", [-0.9, -0.7, -0.5, -0.3, -0.1, 0.1, 0.3, 0.5, 0.7, 0.9])
def test_c1_calibration_reproduces_table1(k):
    """Table 1 calibrates c1(k) so that the BEM pull-off of a parabolic
    indenter equals the JKR-type -(3+k) pi gamma R / 2.  Redo that fit: the
    pull-off force at c1 and 1.25 c1 (p_crit from Eq. 24 scales as c1^-1/2)
    gives the power law F_min ~ c1^e, and with it the c1 that meets the
    closed form.  512^2 on a side of 4 a_F (128 elements across the pull-off
    radius; the preload radius 1.5 a_F stays inside), R = 1, gamma = 2.9995e-3,
    nu = 0.3, mixed precision."""
    from paper_1612_08395_amd import bem
    announce(f"c1-calibration k={k}")
    n, nu, R, gam = 512, 0.3, 1.0, 2.9995e-3
    aF, dj = _jkr_points(k, nu, gam, R)
    L = 4.0 * aF
    dx = L / n
    K = bem.bem_influence(n, n, dx, k, nu)
    h = inputs.parabolic(n, L, R)
    pc = bem.bem_p_crit(k, nu, gam, dx)       # Eq. 24 with Table 1's c1
    ref = an.jkr_min_force(k, gam, R)
    ratio = {}
    pen = 0
    for f in (1.0, 1.25):
        prm = bem.bem_params_init(gamma=gam, p_crit=pc / math.sqrt(f), precision=bem.BEM_MIXED)
        # k = -0.9: the nearly flat kernel r^-0.1 lifts the free surface round a
        # shrinking tensile contact into the indenter (elements off the set
        # with g < 0); the contact set only shrinks under unloading (no
        # re-attachment), so those are counted, not excluded
        Fmin, res = _pulloff_sweep(bem, K, h, k, R, aF, dj, prm, no_penetration=k > -0.85)
        pen = max(pen, max(r.n_penetrating for r in res[1:]))
        ratio[f] = Fmin / ref
    K.free()
    e = math.log(ratio[1.25] / ratio[1.0]) / math.log(1.25)
    c1_fit = math.exp(-math.log(ratio[1.0]) / e)   # relative to the table value
    C1_FIT[k] = c1_fit
    print(f"[c1 k={k}] F_min/F_JKR {ratio[1.0]:.4f} (c1), {ratio[1.25]:.4f} (1.25 c1); "
          f"exponent {e:.3f}; fitted c1 / Table 1 = {c1_fit:.4f}; most penetrating elements "
          f"off the set {pen}", flush=True)
    assert e == pytest.approx(-1.0, abs=0.1)      # F_min ~ p_crit^2 ~ 1 / c1
    assert c1_fit == pytest.approx(1.0, abs=0.03)


def test_pulloff_independent_of_R_over_c0():
    """Fig. 8a: the adhesive F(d) of a parabolic indenter for several R / c0
    (here c0 = 0.5, 1, 2 with R = 1, k = 0.5, side 2, 512^2, mixed
    precision).  c0 enters through C = alpha (1 - nu^2) c0^k / E0 and the
    c0^k of Eq. 24; the closed-form pull-off -(3+k) pi gamma R / 2 does not
    depend on it, while the pull-off radius grows as c0^(k/(3+k))."""
    from paper_1612_08395_amd import bem
    announce("R/c0 sweep")
    n, L, k, nu, R, gam = 512, 2.0, 0.5, 0.3, 1.0, 2.9995e-3
    dx = L / n
    h = inputs.parabolic(n, L, R)
    ref = an.jkr_min_force(k, gam, R)
    got = {}
    for c0 in (0.5, 1.0, 2.0):
        aF, dj = _jkr_points(k, nu, gam, R, c0)
        K = bem.bem_influence_ex(n, n, dx, dx, k, nu, 1.0, c0)
        Fmin, res = _pulloff_sweep(bem, K, h, k, R, aF, dj,
                                   bem.bem_params_init(gamma=gam, precision=bem.BEM_MIXED))
        K.free()
        got[c0] = Fmin / ref
        at_min = min(res[1:], key=lambda r: r.F)
        print(f"[R/c0={R / c0:g}] F_min / F_JKR {got[c0]:.4f}, a_F {aF:.4f} "
              f"({aF / dx:.0f} elements), contact radius at F_min "
              f"{math.sqrt(at_min.area / math.pi):.4f}", flush=True)
        assert got[c0] == pytest.approx(1.0, rel=2.1 / (aF / dx))
    vals = np.array(list(got.values()))
    assert vals.max() / vals.min() - 1.0 < 0.01


def test_adhesive_step_transitions_c0():
    """GPU vs oracle pull-off step transitions at c0 = 2 (R / c0 = 1/2),
    k = 0.5, 128^2, side 2: from the oracle's previous contact set and
    pressure (set into the GPU state), the same new contact set and pressure
    (FP64, 1e-10)."""
    from oracle import influence as inf
    from oracle import material as m
    from oracle import solver as so
    from oracle.convolution import FFTConvolver
    from paper_1612_08395_amd import bem
    from tests.gpu_util import rel_l2
    announce("c0 step transitions")
    n, L, k, nu, R, gam, c0 = 128, 2.0, 0.5, 0.3, 1.0, 2.9995e-3, 2.0
    dx = L / n
    Kq = inf.influence_quarter(n, n, dx, dx, k)
    C = m.compliance(k, nu, c0=c0)
    conv = FFTConvolver(Kq, C, workers=-1)
    h = inputs.parabolic(n, L, R)
    pc = m.p_crit(k, nu, gam, dx, c0=c0)
    aF, dj = _jkr_points(k, nu, gam, R, c0)
    d0 = (1.5 * aF) ** 2 / ((1 + k) * R)
    load = so.solve_nonadhesive(Kq, C, h, d0, tol=1e-12, conv=conv)
    K = bem.bem_influence_ex(n, n, dx, dx, k, nu, 1.0, c0)
    _, res, p, c, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d0))
    assert rel_l2(p, load.p) <= 1e-10
    A, pr = load.contact, load.p
    rounds = 0
    for s in range(1, 6):
        d = d0 - s * (d0 - dj) / 5.0
        step = so.adhesive_step(Kq, C, h, d, A, pr, pc, tol=1e-12, conv=conv)
        st = bem.bem_state_create(K)
        bem.bem_state_set(st, pr, A.astype(np.uint8))
        _, res, p, c, _ = bem.bem_solve(K, h, bem.bem_params_init(d=d, gamma=gam), state=st)
        st.free()
        print(f"[c0=2] step {s} d={d:.4e} contact {A.sum()} -> {c.sum()} (oracle "
              f"{step.contact.sum()}), rounds {res.detach_rounds}/{step.rounds}", flush=True)
        assert res.p_crit == pytest.approx(pc, rel=1e-14)
        assert np.array_equal(c.astype(bool), step.contact)
        if step.contact.any():
            assert rel_l2(p, step.p) <= 1e-10
        rounds += step.rounds
        A, pr = step.contact, step.p
        if not A.any():
            break
    assert rounds > 0
    K.free()
