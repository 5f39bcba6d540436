"""Driver of the serving loop (bem_server_*): submits a request stream with
Poisson arrivals and collects latency / throughput.  Argument marshalling and
timing only; every solve runs in the library."""
import time

import numpy as np

from . import bem


def run_stream(requests, precision, qps=None, n_slots=4, budget_bytes=8 << 30, seed=0,
               nu=0.3):
    """Submit `requests` (dicts from inputs.serving_requests) to a fresh server.
    qps None: all at once (saturation).  Otherwise Poisson arrivals at rate qps.
    Returns a dict of statistics."""
    srv = bem.bem_server_create(budget_bytes, n_slots)
    rng = np.random.default_rng(seed)
    ids = []
    t0 = time.perf_counter()
    t_next = t0
    for r in requests:
        if qps is not None:
            t_next += rng.exponential(1.0 / qps)
            delay = t_next - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
        prm = bem.bem_params_init(d=r["d"], d_preload=r["d_preload"], gamma=r["gamma"],
                                  precision=precision)
        ids.append(srv.submit(r["n"], r["n"], 1.0 / r["n"], r["k"], nu, r["h"], prm))
    statuses = [srv.poll(i)[0] for i in ids]
    t1 = time.perf_counter()
    st = srv.stats().as_dict()
    srv.free()
    st["wall_s"] = t1 - t0
    st["offered_qps"] = qps
    st["status_counts"] = {int(s): statuses.count(s) for s in set(statuses)}
    return st
