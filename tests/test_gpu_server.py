"""Serving loop: continuous batching of independent solves on one GPU."""
import numpy as np
import pytest

from paper_1612_08395_amd import inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _mix(bem, rng, count):
    reqs = []
    for i in range(count):
        n = int(rng.choice([48, 64, 96, 128, 160, 256]))
        k = float(rng.choice([-0.5, -0.2, 0.0, 0.3, 0.6]))
        shape = i % 4
        L = 1.0
        if shape == 0:
            h = inputs.parabolic(n, L, 1.0)
            d = 0.1 ** 2 / ((1 + k) * 1.0)
        elif shape == 1:
            h = inputs.cone(n, L, 0.1)
            d = 0.01
        elif shape == 2:
            h = inputs.flat_punch(n, L, 0.25)
            d = 2e-3
        else:
            h = inputs.fractal_gap(n, L, 0.7, 8 * 2 * np.pi, n / 4 * 2 * np.pi, 1e-3, 100 + i)
            d = float(np.quantile(h, 0.05))
        prec = bem.BEM_FP64 if i % 3 else bem.BEM_MIXED
        if i % 2 and shape != 2:
            gam = float(np.sqrt(125.0 * (1 / (1 - 0.09)) ** 2 / n ** 3))
            prm = bem.bem_params_init(d=0.5 * d, d_preload=d, gamma=gam, precision=prec)
        else:
            prm = bem.bem_params_init(d=d, precision=prec)
        reqs.append((n, k, h, prm))
    return reqs


def _alone_vs_mix(bem, reqs, batch_slots, extra=()):
    srv = bem.bem_server_create_ex(budget_bytes=4 << 30, n_slots=4, batch_slots=batch_slots)
    ids = [srv.submit(n, n, 1.0 / n, k, 0.3, h, prm, want_p=True) for (n, k, h, prm) in reqs]
    got = [srv.poll(i) for i in ids]
    st = srv.stats()
    srv.free()
    assert st.completed == len(reqs) and st.failed == 0
    assert st.peak_running >= 2                 # requests overlapped on the device
    assert st.device_bytes_reserved <= 4 << 30  # both precisions share the pools
    assert st.p99_latency_s >= st.p50_latency_s > 0
    for (n, k, h, prm), (status, res, p, c) in zip(reqs, got):
        K = bem.bem_influence(n, n, 1.0 / n, k, 0.3)
        rc, ra, pa, ca, _ = bem.bem_solve(K, h, prm)
        K.free()
        assert status == rc
        assert np.array_equal(p, pa)            # bitwise: deterministic reductions
        assert np.array_equal(c, ca)
        assert res.F == ra.F and res.iters == ra.iters
        assert res.n_contact == ra.n_contact and res.detach_rounds == ra.detach_rounds
        assert res.residual == ra.residual and res.n_penetrating == ra.n_penetrating
    return st


def test_alone_and_in_the_mix_are_identical():
    # default server: every request here (48^2 ... 256^2, displacement
    # control) runs on the batched path, its CG kernels sharing launches with
    # the other requests of its geometry and precision
    from paper_1612_08395_amd import bem
    announce("server-mix batched")
    rng = np.random.default_rng(5)
    reqs = _mix(bem, rng, 24)
    st = _alone_vs_mix(bem, reqs, 16)
    assert st.batched == len(reqs)
    assert st.mean_batch_slots > 1.0            # launches did carry several solves
    print(f"[server-mix] mean solves per batched launch {st.mean_batch_slots:.2f}", flush=True)


def test_alone_and_in_the_mix_per_request_path():
    from paper_1612_08395_amd import bem
    announce("server-mix per-request")
    rng = np.random.default_rng(6)
    reqs = _mix(bem, rng, 12)
    st = _alone_vs_mix(bem, reqs, 0)
    assert st.batched == 0


def test_both_paths_together():
    # a batched geometry class next to requests of the per-request path: a
    # grid beyond the batched sweeps (1100 x 1100) and a load-controlled solve
    from paper_1612_08395_amd import bem
    announce("server both paths")
    srv = bem.bem_server_create_ex(budget_bytes=4 << 30, n_slots=2, batch_slots=8)
    reqs = []
    for i, n in enumerate((64, 64, 96, 1100, 64)):
        h = inputs.parabolic(n, 1.0, 1.0)
        if i == 4:
            prm = bem.bem_params_init(control=bem.BEM_CTRL_FORCE, F=2e-3)
        else:
            prm = bem.bem_params_init(d=0.01, precision=bem.BEM_MIXED if i % 2 else bem.BEM_FP64)
        reqs.append((n, 0.2, h, prm))
    ids = [srv.submit(n, n, 1.0 / n, k, 0.3, h, prm, want_p=True) for (n, k, h, prm) in reqs]
    got = [srv.poll(i) for i in ids]
    st = srv.stats()
    srv.free()
    assert st.completed == len(reqs) and st.failed == 0
    assert st.batched == 3
    for (n, k, h, prm), (status, res, p, c) in zip(reqs, got):
        K = bem.bem_influence(n, n, 1.0 / n, k, 0.3)
        rc, ra, pa, ca, _ = bem.bem_solve(K, h, prm)
        K.free()
        assert status == rc and np.array_equal(p, pa) and np.array_equal(c, ca)
        assert res.d == ra.d


def test_served_results_match_oracle():
    # a seeded sample of the serving stream (grids up to 128^2), served in
    # both precisions, against the oracle: non-adhesive solves, and adhesive
    # requests as the non-adhesive preload followed by the pull-off step
    from oracle import influence as inf
    from oracle import material as m
    from oracle import solver as so
    from oracle.convolution import FFTConvolver
    from paper_1612_08395_amd import bem
    from paper_1612_08395_amd.serving import run_stream
    from tests.gpu_util import rel_l2
    announce("served vs oracle")
    reqs = [r for r in inputs.serving_requests(200, 2024) if r["n"] <= 128][:10]
    assert len(reqs) == 10 and any(r["gamma"] > 0 for r in reqs)
    out = {prec: run_stream(reqs, prec, None, want_p=True)["results"]
           for prec in (bem.BEM_FP64, bem.BEM_MIXED)}
    for j, r in enumerate(reqs):
        n, k, nu = r["n"], r["k"], 0.3
        dx = 1.0 / n
        Kq = inf.influence_quarter(n, n, dx, dx, k)
        C = m.compliance(k, nu)
        conv = FFTConvolver(Kq, C)
        if r["gamma"] > 0:
            load = so.solve_nonadhesive(Kq, C, r["h"], max(r["d"], r["d_preload"]), conv=conv)
            ref = so.adhesive_step(Kq, C, r["h"], r["d"], load.contact, load.p,
                                   m.p_crit(k, nu, r["gamma"], dx), conv=conv)
        else:
            ref = so.solve_nonadhesive(Kq, C, r["h"], r["d"], conv=conv)
        for prec, tol in ((bem.BEM_FP64, 1e-10), (bem.BEM_MIXED, 2e-5)):
            status, res, p, c = out[prec][j]
            print(f"[served {j}] n={n} k={k} {r['shape']} gamma={r['gamma']:.2e} prec={prec} "
                  f"status {status} contact {int(c.sum())} vs {int(ref.contact.sum())}", flush=True)
            assert status in (0, bem.BEM_EFLOOR)
            nref = int(ref.contact.sum())
            assert abs(int(c.sum()) - nref) <= max(1, 1e-3 * nref)
            if np.array_equal(c.astype(bool), ref.contact) and np.abs(ref.p).max() > 0:
                assert rel_l2(p, ref.p) <= tol


def test_admission_under_a_tight_budget():
    from paper_1612_08395_amd import bem
    announce("server-budget")
    fi, fs = bem.bem_footprint(256, 256, bem.BEM_FP64)
    srv = bem.bem_server_create(budget_bytes=fi + fs + 1024, n_slots=4)
    rng = np.random.default_rng(9)
    ids = []
    for i in range(6):
        k = [0.1, 0.2][i % 2]                     # two keys alternate: forces evictions
        h = inputs.parabolic(256, 1.0, 1.0)
        ids.append(srv.submit(256, 256, 1 / 256, k, 0.3, h, bem.bem_params_init(d=0.005)))
    out = [srv.poll(i) for i in ids]
    st = srv.stats()
    assert all(o[0] == 0 for o in out)
    assert st.completed == 6 and st.peak_running == 1
    assert st.evictions >= 1
    assert st.device_bytes_reserved <= fi + fs + 1024
    with pytest.raises(bem.BemError) as e:       # can never fit
        srv.submit(512, 512, 1 / 512, 0.1, 0.3, inputs.parabolic(512, 1.0, 1.0),
                   bem.bem_params_init(d=0.005))
    assert e.value.code == bem.BEM_ENOMEM
    srv.free()


def _session_curve(bem, srv, sid, n, k, h, steps, prec, gam):
    # the steps of a load-unload curve as requests of one session: loading
    # steps non-adhesive, pull-off steps (below the previous step) adhesive
    ids, prev = [], None
    for d in steps:
        unloading = gam > 0 and prev is not None and d < prev
        prm = bem.bem_params_init(d=d, gamma=gam if unloading else 0.0, precision=prec)
        ids.append(srv.submit(n, n, 1.0 / n, k, 0.3, h, prm, want_p=True, session=sid))
        prev = d
    return ids


@pytest.mark.parametrize("n,k,prec,adhesive", [
    (64, 0.3, "fp64", False), (96, -0.4, "mixed", False), (64, 0.5, "fp64", True),
    (128, 0.0, "mixed", True), (288, 0.2, "mixed", False), (320, 0.5, "fp64", True)])
def test_session_requests_match_the_library_on_one_state(n, k, prec, adhesive):
    # one session's requests on one gap profile, while other clients'
    # requests run: grids up to 256^2 take the batched path, where each
    # request is bem_solve with the session's state; larger ones the
    # per-request path, where they are the steps of bem_sweep (iteration 0
    # from the previous gap shifted).  Forces, iteration counts, detach
    # rounds and the final pressure agree bitwise with those calls.
    from paper_1612_08395_amd import bem
    announce("server-session", n, k, prec, adhesive)
    P = bem.BEM_FP64 if prec == "fp64" else bem.BEM_MIXED
    h = inputs.parabolic(n, 1.0, 1.0)
    d3 = 0.15 ** 2 / (1 + k)
    gam = float(np.sqrt(125.0 * (1 / (1 - 0.09)) ** 2 / n ** 3)) if adhesive else 0.0
    steps = [d3 / 3, 2 * d3 / 3, d3, d3 / 2, 0.0] if adhesive else [d3 / 4, d3 / 2, d3, 1.5 * d3]
    srv = bem.bem_server_create_ex(budget_bytes=4 << 30, n_slots=4, batch_slots=16)
    sid = srv.session_open()
    ids = _session_curve(bem, srv, sid, n, k, h, steps, P, gam)
    others = [srv.submit(m, m, 1.0 / m, kk, 0.3, hh, pp, want_p=True)
              for (m, kk, hh, pp) in _mix(bem, np.random.default_rng(11), 8)]
    got = [srv.poll(i) for i in ids]
    for i in others:
        assert srv.poll(i)[0] >= 0
    srv.session_close(sid)
    st = srv.stats()
    srv.free()
    assert st.failed == 0 and st.device_bytes_reserved <= 4 << 30
    batched = n <= 256
    assert st.batched >= (len(steps) if batched else 0)
    K = bem.bem_influence(n, n, 1.0 / n, k, 0.3)
    S = bem.bem_state_create(K)
    if batched:
        res, prev = [], None
        for d in steps:
            unloading = gam > 0 and prev is not None and d < prev
            prm = bem.bem_params_init(d=d, gamma=gam if unloading else 0.0, precision=P)
            res.append(bem.bem_solve(K, h, prm, state=S)[1])
            prev = d
    else:
        rc, res = bem.bem_sweep(K, h, bem.bem_params_init(gamma=gam, precision=P), steps,
                                state=S)
    p_last, _ = bem.bem_state_get(S)
    S.free()
    K.free()
    for (status, r, p, c), ra in zip(got, res):
        assert status >= 0
        assert r.F == ra.F and r.iters == ra.iters and r.n_contact == ra.n_contact
        assert r.detach_rounds == ra.detach_rounds and r.residual == ra.residual
    assert np.array_equal(got[-1][2], p_last)
    print(f"[server-session] iterations per step {[r.iters for _, r, _, _ in got]}", flush=True)


def test_session_with_new_profile_warm_starts_to_the_same_solution():
    # a request whose gap profile differs from the session's previous one
    # starts from the previous pressure only; a non-adhesive solution is
    # unique, so it matches a cold solve to the CG tolerance
    from paper_1612_08395_amd import bem
    announce("server-session new profile")
    n, k = 96, 0.2
    h1 = inputs.parabolic(n, 1.0, 1.0)
    h2 = inputs.fractal_gap(n, 1.0, 0.7, 8 * 2 * np.pi, n / 4 * 2 * np.pi, 1e-3, 77) + h1
    d = 0.01
    srv = bem.bem_server_create_ex(budget_bytes=1 << 30, n_slots=2, batch_slots=0)
    sid = srv.session_open()
    prm = bem.bem_params_init(d=d)
    i1 = srv.submit(n, n, 1.0 / n, k, 0.3, h1, prm, want_p=True, session=sid)
    i2 = srv.submit(n, n, 1.0 / n, k, 0.3, h2, prm, want_p=True, session=sid)
    (_, r1, _, _), (s2, r2, p2, c2) = srv.poll(i1), srv.poll(i2)
    srv.session_close(sid)
    srv.free()
    K = bem.bem_influence(n, n, 1.0 / n, k, 0.3)
    rc, ra, pa, ca, _ = bem.bem_solve(K, h2, prm)
    K.free()
    assert s2 == rc == bem.BEM_OK
    assert np.linalg.norm(p2 - pa) <= 1e-8 * np.linalg.norm(pa)
    assert abs(r2.F - ra.F) <= 1e-10 * abs(ra.F)
    assert np.array_equal(c2, ca)


def test_session_errors_and_budget():
    from paper_1612_08395_amd import bem
    announce("server-session errors")
    n = 64
    h = inputs.parabolic(n, 1.0, 1.0)
    prm = bem.bem_params_init(d=0.005, precision=bem.BEM_MIXED)
    srv = bem.bem_server_create_ex(budget_bytes=1 << 30, n_slots=2, batch_slots=16)
    sid = srv.session_open()
    i1 = srv.submit(n, n, 1.0 / n, 0.3, 0.3, h, prm, session=sid)
    for bad in ((n + 1, 0.3, bem.BEM_MIXED), (n, 0.2, bem.BEM_MIXED), (n, 0.3, bem.BEM_FP64)):
        m, kk, pr = bad
        with pytest.raises(bem.BemError) as e:
            srv.submit(m, m, 1.0 / n, kk, 0.3, inputs.parabolic(m, 1.0, 1.0),
                       bem.bem_params_init(d=0.005, precision=pr), session=sid)
        assert e.value.code == bem.BEM_EINVAL
    assert srv.poll(i1)[0] == bem.BEM_OK
    reserved_open = srv.stats().device_bytes_reserved
    srv.session_close(sid)
    with pytest.raises(bem.BemError):
        srv.session_close(sid)
    with pytest.raises(bem.BemError):
        srv.submit(n, n, 1.0 / n, 0.3, 0.3, h, prm, session=sid)
    with pytest.raises(bem.BemError):
        srv.submit(n, n, 1.0 / n, 0.3, 0.3, h, prm, session=12345)
    # the closed session's state went back to the pool: the same grid runs on
    # the per-request path without reserving more memory
    sid2 = srv.session_open()
    i2 = srv.submit(n, n, 1.0 / n, 0.3, 0.3, h, prm, session=sid2)
    assert srv.poll(i2)[0] == bem.BEM_OK
    st = srv.stats()
    assert st.device_bytes_reserved == reserved_open and st.cache_hits >= 1
    srv.session_close(sid2)
    srv.free()


def test_server_free_with_open_sessions_and_queued_requests():
    # freeing the server drops queued requests and returns every session's
    # state, whether its requests ran or not
    from paper_1612_08395_amd import bem
    announce("server-session free")
    srv = bem.bem_server_create_ex(budget_bytes=1 << 30, n_slots=2, batch_slots=16)
    sids = [srv.session_open() for _ in range(3)]
    for j, (n, k) in enumerate(((64, 0.3), (320, 0.1), (128, -0.2))):
        h = inputs.parabolic(n, 1.0, 1.0)
        for d in (0.002, 0.004, 0.006):
            srv.submit(n, n, 1.0 / n, k, 0.3, h, bem.bem_params_init(d=d), session=sids[j])
    first = srv.submit(64, 64, 1.0 / 64, 0.3, 0.3, inputs.parabolic(64, 1.0, 1.0),
                       bem.bem_params_init(d=0.003))
    assert srv.poll(first)[0] == bem.BEM_OK
    srv.session_close(sids[0])
    srv.free()                                   # sessions 1 and 2 still open
