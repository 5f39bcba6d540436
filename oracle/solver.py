"""Contact solves (oracle).

Test infrastructure only (see ``oracle/__init__``).

Sign conventions: p > 0 is compressive; u > 0 is surface displacement into
the half-space; h is the gap between the undeformed surfaces (h >= 0, zero
at the first point of contact); d is the indentation.  The gap after
deformation is g = u + h - d: contact means g = 0, separation g > 0.

Non-adhesive contact (Section 2.1).  The paper solves the inverse problem
(pressure from prescribed surface displacement in contact, p >= 0 outside
of it) with the constrained conjugate-gradient method it cites (Polonsky &
Keer; Pohrt & Li) and does not print the algorithm.  This oracle takes that
published method in its displacement-controlled form (d given; the mean-gap
shift and load rescaling of the load-controlled form are not used):

  repeat
    u = C K * p ;  g = u + h - d ;  Ic = {p > 0} ;  G = sum_Ic g^2
    t = g + delta (G / G_old) t  on Ic, 0 elsewhere ;  G_old = G
    r = C K * t ;  tau = sum_Ic g t / sum_Ic r t
    p <- p - tau t on Ic ;  p <- max(p, 0)
    Iol = {p = 0 and g < 0} ; delta = 1 if Iol is empty, else delta = 0 and
    p <- p - tau g on Iol
  until sqrt(G) <= tol ||(d - h)_Ic||, Iol is empty and
        sum |p_new - p_old| <= tol sum |p_new|

(the stopping test is made at the top of an iteration, so G belongs to the
iterate that is returned.)  The cold start is p = max(d - h, 0) / (C K(0,0)).
The non-adhesive solution is unique (K is symmetric positive definite), so
initial guess and iteration path do not change the answer.

Adhesive contact (Section 3.1).  With the contact set A held fixed, the
pressure on A follows from u = d - h on A and p = 0 off A: a symmetric
positive-definite linear system solved by the same iteration with Ic := A,
no clipping and no overlap step.  Then every element of A whose tensile
stress exceeds p_crit (-p > p_crit, strict) leaves A, all at once; the
solve is repeated on the reduced set until no element violates the
criterion.  Force F = Dx Dy sum p.

Load-controlled non-adhesive contact (the form of the cited method in
which the total force W is prescribed and the indentation is an unknown).
With gh = u + h (the gap up to the unknown rigid approach):

  repeat
    u = C K * p ;  Ic = {p > 0} ;  gbar = mean_Ic gh ;  g = gh - gbar
    G = sum_Ic g^2
    t = g + delta (G / G_old) t on Ic, 0 elsewhere ;  G_old = G
    r = C K * t ;  r <- r - mean_Ic r ;  tau = sum_Ic g t / sum_Ic r t
    p <- p - tau t on Ic ;  p <- max(p, 0) ;  overlap step as above
    p <- p W / (Dx Dy sum p)
  until sqrt(G) <= tol ||u_Ic||, Iol is empty and
        sum |p_new - p_old| <= tol sum |p_new|

The indentation is d = gbar: on Ic the gap u + h - d vanishes.  The cold
start is a uniform pressure carrying W.  (Reading: the stopping test is the
displacement-controlled one, with the contact displacement as its scale.)

Pins (tests/test_oracle_solver.py): KKT conditions with a direct-sum
residual; cold and warm starts agree; four-fold symmetry of a centred
indenter; Hertz (k = 0) force and radius; power-law Hertz-type radius
(Eq. 15) and force (reading of Eq. 16); exterior displacement (Eq. 14);
Boussinesq flat-punch stiffness; JKR pull-off force at k = 0 and its
power-law generalisation.
"""
import numpy as np

from .convolution import FFTConvolver


class SolveResult:
    def __init__(self, p, g, u, iters, converged, contact, rounds=0):
        self.p = p
        self.g = g
        self.u = u
        self.iters = iters
        self.converged = converged
        self.contact = contact
        self.rounds = rounds


def _cg(conv, h, d, p, tol, max_iter, fixed_set=None):
    """Shared loop.  fixed_set None: non-adhesive (Ic = {p > 0}, projection
    and overlap step).  fixed_set = boolean mask A: adhesive fixed-set solve."""
    f = d - h
    delta = 0.0
    G_old = 1.0
    t = np.zeros_like(p)
    n_ol, sum_dp, sum_p = 0, np.inf, 1.0
    it = 0
    converged = False
    while True:
        u = conv(p)
        g = u + h - d
        Ic = (p > 0) if fixed_set is None else fixed_set
        G = float(np.sum(g[Ic] ** 2))
        fnorm = float(np.sqrt(np.sum(f[Ic] ** 2)))
        if it > 0 and np.sqrt(G) <= tol * fnorm and n_ol == 0 and sum_dp <= tol * sum_p:
            converged = True
            break
        if it >= max_iter:
            break
        it += 1
        ratio = G / G_old if G_old > 0 else 0.0
        t = np.where(Ic, g + delta * ratio * t, 0.0)
        G_old = G
        r = conv(t)
        rt = float(np.sum(r[Ic] * t[Ic]))
        tau = float(np.sum(g[Ic] * t[Ic])) / rt if rt != 0.0 else 0.0
        p_old = p
        p = np.where(Ic, p - tau * t, p)
        if fixed_set is None:
            p = np.maximum(p, 0.0)
            ol = (p == 0.0) & (g < 0.0)
            n_ol = int(np.count_nonzero(ol))
            if n_ol == 0:
                delta = 1.0
            else:
                delta = 0.0
                p = np.where(ol, p - tau * g, p)
        else:
            delta = 1.0
        sum_dp = float(np.sum(np.abs(p - p_old)))
        sum_p = float(np.sum(np.abs(p)))
    return p, g, u, it, converged


def cold_start(Kq, C, h, d):
    """p = max(d - h, 0) / (C K(0, 0)): each element pushed alone to close its gap."""
    return np.maximum(d - h, 0.0) / (C * Kq[0, 0])


def solve_nonadhesive(Kq, C, h, d, tol=1e-12, max_iter=20000, p_init=None, conv=None):
    """Displacement-controlled non-adhesive solve (see module docstring)."""
    h = np.asarray(h, dtype=np.float64)
    conv = conv or FFTConvolver(Kq, C)
    if not np.any(h < d):
        z = np.zeros_like(h)
        u = z.copy()
        return SolveResult(z, u + h - d, u, 0, True, z > 0)
    p = cold_start(Kq, C, h, d) if p_init is None else np.maximum(np.asarray(p_init, float), 0.0)
    p, g, u, it, ok = _cg(conv, h, d, p, tol, max_iter)
    return SolveResult(p, g, u, it, ok, p > 0)


def solve_fixed_set(Kq, C, h, d, A, p_init=None, tol=1e-12, max_iter=20000, conv=None):
    """Pressure on the fixed contact set A with u = d - h on A, p = 0 off A."""
    h = np.asarray(h, dtype=np.float64)
    A = np.asarray(A, dtype=bool)
    conv = conv or FFTConvolver(Kq, C)
    if not A.any():
        z = np.zeros_like(h)
        u = z.copy()
        return SolveResult(z, u + h - d, u, 0, True, A.copy())
    p = np.zeros_like(h) if p_init is None else np.where(A, p_init, 0.0)
    p, g, u, it, ok = _cg(conv, h, d, p, tol, max_iter, fixed_set=A)
    return SolveResult(p, g, u, it, ok, A.copy())


def adhesive_step(Kq, C, h, d, A, p_init, pcrit, tol=1e-12, max_iter=20000, conv=None):
    """One pull-off step: fixed-set solve, detach all violators, re-solve
    until none is left (Section 3.1)."""
    conv = conv or FFTConvolver(Kq, C)
    A = np.asarray(A, dtype=bool).copy()
    p = np.where(A, p_init, 0.0)
    rounds = 0
    iters = 0
    while True:
        res = solve_fixed_set(Kq, C, h, d, A, p, tol, max_iter, conv)
        iters += res.iters
        V = A & (-res.p > pcrit)
        if not V.any():
            res.rounds = rounds
            res.iters = iters
            res.contact = A
            return res
        A = A & ~V
        p = np.where(A, res.p, 0.0)
        rounds += 1


def solve_force(Kq, C, h, W, dx, dy, tol=1e-12, max_iter=20000, p_init=None, conv=None):
    """Load-controlled non-adhesive solve (see module docstring).  Returns a
    SolveResult with the indentation in .d."""
    h = np.asarray(h, dtype=np.float64)
    conv = conv or FFTConvolver(Kq, C)
    if W <= 0.0:
        z = np.zeros_like(h)
        res = SolveResult(z, h - h.min(), z.copy(), 0, True, z > 0)
        res.d = float(h.min())
        return res
    P_target = W / (dx * dy)
    if p_init is None or not np.any(np.asarray(p_init) > 0):
        p = np.full_like(h, P_target / h.size)
    else:
        p = np.maximum(np.asarray(p_init, dtype=np.float64), 0.0)
        p = p * (P_target / np.sum(p))
    delta = 0.0
    G_old = 1.0
    t = np.zeros_like(p)
    n_ol, sum_dp, sum_p = 0, np.inf, 1.0
    it = 0
    converged = False
    while True:
        u = conv(p)
        gh = u + h
        Ic = p > 0
        gbar = float(np.mean(gh[Ic]))
        g = gh - gbar
        G = float(np.sum(g[Ic] ** 2))
        unorm = float(np.sqrt(np.sum(u[Ic] ** 2)))
        if it > 0 and np.sqrt(G) <= tol * unorm and n_ol == 0 and sum_dp <= tol * sum_p:
            converged = True
            break
        if it >= max_iter:
            break
        it += 1
        ratio = G / G_old if G_old > 0 else 0.0
        t = np.where(Ic, g + delta * ratio * t, 0.0)
        G_old = G
        r = conv(t)
        r = r - float(np.mean(r[Ic]))
        rt = float(np.sum(r[Ic] * t[Ic]))
        tau = float(np.sum(g[Ic] * t[Ic])) / rt if rt != 0.0 else 0.0
        p_old = p
        p = np.where(Ic, p - tau * t, p)
        p = np.maximum(p, 0.0)
        ol = (p == 0.0) & (g < 0.0)
        n_ol = int(np.count_nonzero(ol))
        if n_ol == 0:
            delta = 1.0
        else:
            delta = 0.0
            p = np.where(ol, p - tau * g, p)
        p = p * (P_target / np.sum(p))
        sum_dp = float(np.sum(np.abs(p - p_old)))
        sum_p = float(np.sum(np.abs(p)))
    res = SolveResult(p, g, u, it, converged, p > 0)
    res.d = gbar
    return res


def force(p, dx, dy):
    """Total normal force: element area times the sum of pressures."""
    return float(dx * dy * np.sum(p))
