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


def test_alone_and_in_the_mix_are_identical():
    from paper_1612_08395_amd import bem
    announce("server-mix")
    rng = np.random.default_rng(5)
    reqs = _mix(bem, rng, 24)
    srv = bem.bem_server_create(budget_bytes=4 << 30, n_slots=4)
    ids = [srv.submit(n, n, 1.0 / n, k, 0.3, h, prm, want_p=True) for (n, k, h, prm) in reqs]
    got = [srv.poll(i) for i in ids]
    st = srv.stats()
    assert st.completed == len(reqs) and st.failed == 0
    assert st.peak_running >= 2                 # requests overlapped on the device
    assert st.device_bytes_reserved <= 4 << 30  # both precisions share the pools
    assert st.p99_latency_s >= st.p50_latency_s > 0
    srv.free()
    for (n, k, h, prm), (status, res, p, c) in zip(reqs, got):
        K = bem.bem_influence(n, n, 1.0 / n, k, 0.3)
        rc, ra, pa, ca, _ = bem.bem_solve(K, h, prm)
        K.free()
        assert status == rc
        assert np.array_equal(p, pa)            # bitwise: deterministic reductions
        assert np.array_equal(c, ca)
        assert res.F == ra.F and res.iters == ra.iters


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
