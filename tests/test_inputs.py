"""The seeded input generators (CPU): the serving stream and its variants,
the loading curves of serving.run_curves, the rough surface's statistics."""
import math

import numpy as np
import pytest

from paper_1612_08395_amd import inputs


def test_serving_stream_is_seeded_and_spans_the_configured_ranges():
    a = inputs.serving_requests(400, 2024)
    b = inputs.serving_requests(400, 2024)
    assert all(x["n"] == y["n"] and x["k"] == y["k"] and np.array_equal(x["h"], y["h"])
               for x, y in zip(a, b))
    ns = np.array([r["n"] for r in a])
    assert ns.min() >= 64 and ns.max() <= 1024 and np.all(ns % 16 == 0)
    ks = np.array([r["k"] for r in a])
    assert np.all(np.abs(ks) < 0.8)
    assert np.allclose(ks * 20, np.round(ks * 20))            # the 0.05 grid
    shapes = {r["shape"] for r in a}
    assert shapes == {"parabolic", "cone", "punch", "rough"}
    adh = [r for r in a if r["gamma"] > 0]
    assert 0.4 < len(adh) / len(a) < 0.6
    for r in adh:                                             # preload, then pull-off at d0 / 2
        assert r["d"] == pytest.approx(0.5 * r["d_preload"])


def test_continuous_k_moves_only_k():
    a = inputs.serving_requests(200, 7)
    b = inputs.serving_requests(200, 7, continuous_k=True)
    dk = np.array([y["k"] - x["k"] for x, y in zip(a, b)])
    assert np.all(np.abs(dk) <= 0.025 + 1e-12) and np.count_nonzero(dk) == len(dk)
    assert len({round(y["k"], 12) for y in b}) == len(b)      # no shared influence operator
    for x, y in zip(a, b):
        assert (x["n"], x["shape"], x["gamma"]) == (y["n"], y["shape"], y["gamma"])
        assert np.array_equal(x["h"], y["h"])


def test_curve_steps():
    from paper_1612_08395_amd.serving import curve_steps
    plain = {"n": 64, "d": 0.01, "d_preload": 0.0, "gamma": 0.0}
    st = curve_steps(plain, 8)
    assert [a for _, a in st] == [False] * 8
    assert [d for d, _ in st] == pytest.approx([0.01 * (j + 1) / 8 for j in range(8)])
    adh = {"n": 64, "d": 0.005, "d_preload": 0.01, "gamma": 1e-3}
    st = curve_steps(adh, 8)
    assert [a for _, a in st] == [False] * 4 + [True] * 4
    ds = [d for d, _ in st]
    assert ds[3] == pytest.approx(0.01) and ds[-1] == 0.0
    assert all(ds[i + 1] < ds[i] for i in range(3, 7))        # pull-off: decreasing


def test_rough_surface_statistics():
    n, L, H = 256, 1.0, 0.7
    h = inputs.fractal_gap(n, L, H, 8 * 2 * math.pi / L, 64 * 2 * math.pi / L, 1e-3 * L, 3)
    z = h.max() - h
    assert h.min() == 0.0
    assert np.sqrt(np.mean((z - z.mean()) ** 2)) == pytest.approx(1e-3 * L, rel=1e-9)
    # no power above q1: the spectrum vanishes beyond 64 waves per side
    F = np.abs(np.fft.rfft2(z - z.mean()))
    kx = np.fft.rfftfreq(n, 1.0 / n)
    ky = np.fft.fftfreq(n, 1.0 / n)
    q = np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)
    assert F[q > 64.5].max() <= 1e-9 * F.max()
