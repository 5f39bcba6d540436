"""Driver of the serving loop (bem_server_*): submits a request stream with
Poisson arrivals and collects latency / throughput, and runs loading curves
with and without server sessions.  Argument marshalling and
timing only; every solve runs in the library.

    python -m paper_1612_08395_amd.serving --requests 10000 --out stream.json

runs the seeded request stream (inputs.serving_requests) at saturation for
both precisions, then with Poisson arrivals at 0.8 x the FP64 saturation
rate, and writes the statistics as JSON; --phase curves runs each request's
loading curve with and without server sessions instead.
"""
import argparse
import json
import sys
import time

import numpy as np

from . import bem


def run_stream(requests, precision, qps=None, n_slots=4, budget_bytes=8 << 30, seed=0,
               nu=0.3, batch_slots=16, want_p=False, progress=None):
    """Submit `requests` (dicts from inputs.serving_requests) to a fresh server.
    qps None: all at once (saturation).  Otherwise Poisson arrivals at rate qps.
    batch_slots: solves per batched launch group (0: every request is a solve
    of its own).  Returns a dict of statistics; with want_p also the list of
    (status, result, pressure, contact) per request under "results"."""
    srv = bem.bem_server_create_ex(budget_bytes, n_slots, batch_slots)
    rng = np.random.default_rng(seed)
    ids = []
    t0 = time.perf_counter()
    t_next = t0
    for j, r in enumerate(requests):
        if qps is not None:
            t_next += rng.exponential(1.0 / qps)
            delay = t_next - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
        prm = bem.bem_params_init(d=r["d"], d_preload=r["d_preload"], gamma=r["gamma"],
                                  precision=precision)
        ids.append(srv.submit(r["n"], r["n"], 1.0 / r["n"], r["k"], nu, r["h"], prm,
                              want_p=want_p))
        if progress and (j + 1) % progress == 0:
            print(f"[serving] submitted {j + 1}/{len(requests)}", file=sys.stderr, flush=True)
    polled = []
    for j, i in enumerate(ids):
        polled.append(srv.poll(i))
        if progress and (j + 1) % progress == 0:
            print(f"[serving] done {j + 1}/{len(ids)}", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    st = srv.stats().as_dict()
    srv.free()
    statuses = [p[0] for p in polled]
    st["wall_s"] = t1 - t0
    st["offered_qps"] = qps
    st["status_counts"] = {int(s): statuses.count(s) for s in set(statuses)}
    st["statuses"] = statuses
    if want_p:
        st["results"] = [(p[0], p[1], p[2], p[3]) for p in polled]
    return st


def curve_steps(r, steps=8):
    """The indentation steps of one request's loading curve: `steps` loading
    steps up to its depth d, or, for an adhesive request (gamma > 0), half as
    many loading steps up to d_preload and as many pull-off steps down from
    it.  Returns [(d, adhesive), ...]."""
    if r["gamma"] > 0:
        m = steps // 2
        d0 = r["d_preload"]
        return ([(d0 * (j + 1) / m, False) for j in range(m)] +
                [(d0 * (m - 1 - j) / m, True) for j in range(m)])
    return [(r["d"] * (j + 1) / steps, False) for j in range(steps)]


def run_curves(requests, precision, sessions, steps=8, n_slots=4, budget_bytes=8 << 30,
               batch_slots=16, nu=0.3):
    """Each request becomes a load(-unload) curve (curve_steps), all curves
    submitted at once.  sessions=True: one server session per curve, so each
    step starts from the previous step's state on the device; False: every
    step an independent request (cold start; a pull-off step then makes its
    contact set by a non-adhesive preload to the curve's deepest step, as a
    client without sessions would have to).  Returns a dict of statistics."""
    srv = bem.bem_server_create_ex(budget_bytes, n_slots, batch_slots)
    t0 = time.perf_counter()
    ids = []
    for r in requests:
        sid = srv.session_open() if sessions else None
        cs = curve_steps(r, steps)
        dmax = max(d for d, _ in cs)
        for d, adh in cs:
            prm = bem.bem_params_init(d=d, gamma=r["gamma"] if adh else 0.0,
                                      d_preload=0.0 if sessions else dmax, precision=precision)
            ids.append(srv.submit(r["n"], r["n"], 1.0 / r["n"], r["k"], nu, r["h"], prm,
                                  session=sid))
        if sessions:
            srv.session_close(sid)   # no more requests; released after its last one
    polled = [srv.poll(i) for i in ids]
    t1 = time.perf_counter()
    st = srv.stats().as_dict()
    srv.free()
    iters = [p[1].iters for p in polled]
    statuses = [p[0] for p in polled]
    return {"curves": len(requests), "solves": len(ids), "wall_s": t1 - t0,
            "solves_per_s": len(ids) / (t1 - t0), "mean_iters": float(np.mean(iters)),
            "p50_latency_s": st["p50_latency_s"], "p99_latency_s": st["p99_latency_s"],
            "batched": st["batched"],
            "status_counts": {int(x): statuses.count(x) for x in set(statuses)}}


KEYS_SAT = ("solves_per_s", "p50_latency_s", "p99_latency_s", "mean_wait_s", "peak_running",
            "batched", "mean_batch_slots", "engine_launch_s", "engine_sync_s", "engine_step_s",
            "cache_hits", "cache_misses", "evictions", "status_counts", "wall_s")
KEYS_POISSON = ("offered_qps", "solves_per_s", "p50_latency_s", "p99_latency_s", "mean_wait_s",
                "peak_running", "batched", "mean_batch_slots", "status_counts", "wall_s")


def main():
    from . import inputs
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=10000)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--batch-slots", type=int, default=16)
    ap.add_argument("--budget-gb", type=float, default=8.0)
    ap.add_argument("--out", default=None)
    ap.add_argument("--phase", choices=("all", "saturation", "poisson", "curves"), default="all",
                    help="saturation runs, Poisson runs (needs --qps), both, or the loading "
                         "curves of the requests with and without sessions")
    ap.add_argument("--continuous-k", action="store_true",
                    help="k off the 0.05 grid: every request builds its influence operator")
    ap.add_argument("--qps", type=float, default=None,
                    help="Poisson arrival rate (default: 0.8 x the FP64 saturation rate)")
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    reqs = inputs.serving_requests(a.requests, a.seed, continuous_k=a.continuous_k)
    print(f"[serving] {len(reqs)} requests built", file=sys.stderr, flush=True)
    budget = int(a.budget_gb * (1 << 30))
    out = {"requests": a.requests, "seed": a.seed, "continuous_k": a.continuous_k, "slots": a.slots,
           "batch_slots": a.batch_slots, "budget_bytes": budget}
    sat = {}
    if a.phase == "curves":
        for prec, name in ((bem.BEM_FP64, "fp64"), (bem.BEM_MIXED, "mixed")):
            for sessions in (True, False):
                key = f"{name}_curves_{'sessions' if sessions else 'independent'}"
                out[key] = run_curves(reqs, prec, sessions, n_slots=a.slots,
                                      budget_bytes=budget, batch_slots=a.batch_slots)
                print(f"[serving] {key} {out[key]['solves_per_s']:.1f} solves/s", file=sys.stderr,
                      flush=True)
    for prec, name in ((bem.BEM_FP64, "fp64"), (bem.BEM_MIXED, "mixed")):
        if a.phase in ("poisson", "curves"):
            break
        s = run_stream(reqs, prec, None, a.slots, budget, batch_slots=a.batch_slots,
                       progress=500)
        sat[name] = s["solves_per_s"]
        out[f"{name}_saturation"] = {k: s[k] for k in KEYS_SAT}
        print(f"[serving] {name} saturation {s['solves_per_s']:.1f} solves/s", file=sys.stderr,
              flush=True)
    qps = a.qps if a.qps else 0.8 * sat.get("fp64", 0.0)
    for prec, name in ((bem.BEM_FP64, "fp64"), (bem.BEM_MIXED, "mixed")):
        if a.phase in ("saturation", "curves") or qps <= 0:
            break
        s = run_stream(reqs, prec, qps, a.slots, budget, seed=7, batch_slots=a.batch_slots,
                       progress=500)
        out[f"{name}_poisson"] = {k: s[k] for k in KEYS_POISSON}
        print(f"[serving] {name} poisson p99 {s['p99_latency_s']:.3f} s", file=sys.stderr,
              flush=True)
    line = json.dumps(out)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(line + "\n")
    print(line, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
