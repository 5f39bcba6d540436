#!/usr/bin/env python3
"""FFT-CG contact solves/s at 2048^2 on one MI355X: mixed (FP32 transforms and
vectors, FP64 reductions) vs all-FP64.

Workload: non-adhesive contact of a self-affine rough surface with a
power-law graded half-space (Li & Popov, arXiv:1612.08395, Section 2.2,
rough-surface example), on a 2048 x 2048 grid (4096 x 4096 padded
transform): k = 0.3, nu = 0.3, side L = 1, Gaussian heights with
C(q) ~ q^-2(1+H), H = 0.7, roll-off q0 = 8 (2 pi / L), cut-off
q1 = 512 (2 pi / L), rms height 1e-3 L, seed 1612.  One bench step is an
indentation sweep of 20 depths d_s = s d10 / 20 (d10: depth of 10 % contact
area), each a full CG solve, with the gap profile resident in HBM, run by
bem_sweep_dev as --chains (default 2) concurrent warm-start chains (chain c
solves depths c, c + chains, ..., each warm-started from the chain's previous
depth).  value = solves per second of the mixed path; the same sweep as one
chain is reported beside it.

Prints one JSON line.  Also reports the FP64 path, the mixed-vs-FP64
pressure error per depth, the roofline of the dominant kernel and the FP64
CPU oracle timed on the host cores (bounded sample).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
METRIC = "FFT-CG contact solves/s & HBM GB/s at 2048² (FP32 vs FP64); serving p99 latency"
N, L, K_EXP, NU = 2048, 1.0, 0.3, 0.3
H_EXP, Q0, Q1, RMS, SEED = 0.7, 8.0, 512.0, 1e-3, 1612
N_DEPTHS, AREA_FRAC = 20, 0.10
# Depth of 10 % contact area, found by bisection on the FP64 GPU path
# (`python bench.py --find-d10`); None: find it before the timed region.
D10 = 0.004669638031382314
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(HERE, "profiles", "col_conv_f32_2048_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload():
    from paper_1612_08395_amd import inputs
    two_pi = 2.0 * math.pi / L
    return inputs.fractal_gap(N, L, H_EXP, Q0 * two_pi, Q1 * two_pi, RMS * L, SEED)


def find_d10(bem, K, h_dev, torch):
    """Bisection on the FP64 path for 10 % contact area (to 1 % of it)."""
    import numpy as np  # noqa
    hmax = float(h_dev.max().item())
    lo, hi = 0.0, hmax
    st = bem.bem_state_create(K)
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        _, res = bem.bem_solve_dev(K, h_dev, bem.bem_params_init(d=mid), state=st)
        frac = res.n_contact / float(N * N)
        log(f"[d10] d={mid:.6e} area={frac:.5f} iters={res.iters}")
        if abs(frac - AREA_FRAC) <= 0.01 * AREA_FRAC:
            st.free()
            return mid
        if frac < AREA_FRAC:
            lo = mid
        else:
            hi = mid
    st.free()
    return 0.5 * (lo + hi)


def run_sweep(bem, K, h_dev, depths, precision, keep_p=False, torch=None):
    st = bem.bem_state_create(K)
    out = []
    p_list = []
    for d in depths:
        prm = bem.bem_params_init(d=d, precision=precision)
        if keep_p:
            p = torch.empty((N, N), dtype=torch.float64, device="cuda")
            _, res = bem.bem_solve_dev(K, h_dev, prm, state=st, p_out=p)
            p_list.append(p)
        else:
            _, res = bem.bem_solve_dev(K, h_dev, prm, state=st)
        out.append(res.as_dict())
    st.free()
    return out, p_list


def sweep_dev(bem, K, h_dev, depths, precision, chains):
    """One sweep through bem_sweep_dev (h resident on the device) from a
    fresh state, its steps split over `chains` concurrent warm-start chains."""
    st = bem.bem_state_create(K)
    _, res = bem.bem_sweep_dev(K, h_dev, bem.bem_params_init(precision=precision), depths,
                               chains=chains, state=st)
    st.free()
    return [r.as_dict() for r in res]


def loop_bytes(f, w=4):
    """Algorithmic bytes per grid element of one CG iteration at contact
    fraction f, for w-byte reals (4 FP32, 8 FP64).  In FP32: update + R2C
    21 + 4 f (p, g, flags, spectrum; t on the contact set), column sweep 20,
    C2R + gap 17, direction + R2C 9 + 12 f (flags, spectrum; g and t read
    and t written on the contact set), column energy 12: 79 + 16 f.  The
    contact flags are 3 of those bytes and stay one byte per element in
    FP64."""
    return (76.0 + 16.0 * f) * w / 4 + 3.0


def timed(bem, K, h_dev, depths, precision, steps, warmup, torch, chains, clock=True):
    """Times `steps` sweeps, uninstrumented.  Then (clock=True) one more sweep
    of the same depths runs as a single chain with the library's solver clock
    (HIP events on the solver stream around every CG launch; the events cost
    about 10 % of a sweep, so they stay out of the timed steps) for the
    per-kernel durations."""
    for _ in range(warmup):
        sweep_dev(bem, K, h_dev, depths, precision, chains)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(steps):
        results.append(sweep_dev(bem, K, h_dev, depths, precision, chains))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    clk = None
    if clock:
        bem.bem_clock_start()
        sweep_dev(bem, K, h_dev, depths, precision, 1)
        torch.cuda.synchronize()
        clk = bem.bem_clock_stop()
    return (t1 - t0), results, clk


def roofline(bem, K, clock, torch):
    """Dominant kernel: the fused column sweep (FFT x spectrum x IFFT), FP32,
    launched once per CG iteration (the second convolution's column kernel,
    transform + spectral inner product, is reported beside it).  Algorithmic bytes per launch: read +
    write the ny x Lx complex row spectrum and read the (Lx+1) x (Ly+1) real
    kernel spectrum.  Duration: the solver clock's mean over every column
    launch that did work in one sweep of the timed workload (HIP events on
    the solver stream), less the cost of one event record on the stream: in
    displacement control the last two events of an iteration are recorded
    back to back, and their interval is that cost."""
    info = K.info
    Lx, Ly = info.Mx // 2, info.My // 2
    bytes_per_launch = 2 * info.ny * Lx * 8 + (Lx + 1) * (Ly + 1) * 4
    n_col = clock.launches[1]
    ev_ms = clock.ms[5] / max(1, clock.launches[5])
    ms_raw = clock.ms[1] / n_col
    ms = ms_raw - ev_ms
    achieved = bytes_per_launch / (ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        from paper_1612_08395_amd.profile_summary import kernel_source_sha
        if tr.get("source_sha") == kernel_source_sha():
            traffic = tr.get("bytes_per_launch")
    stream = torch.cuda.current_stream()
    iso = bem.bem_kernel_time(K, bem.BEM_MIXED, 1, reps=50, stream=stream)
    # practical ceilings beside the published peak: plain device copies
    # (torch), read + written bytes over their time, one moving as many bytes
    # as a column launch (its buffers stay in the last-level cache between
    # copies, as the CG loop's ~0.12 GB working set at 2048^2 can) and one of
    # 2 x 1 GiB (HBM)
    def copy_gbps(nbytes, reps):
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        t_a, t_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t_a.record()
        for _ in range(reps):
            dst.copy_(src)
        t_b.record()
        torch.cuda.synchronize()
        return 2 * src.numel() * 4 * reps / (t_a.elapsed_time(t_b) * 1e-3) / 1e9

    copy_same = copy_gbps(bytes_per_launch // 2, 50)
    copy_hbm = copy_gbps(1 << 30, 5)
    # the same launches against the usable fp32 vector peak: 4 FFTs of Ly
    # points per column (5 n log2 n flops each) and the spectrum multiply;
    # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz, non-packed fp32
    flop = Lx * (4 * 5 * Ly * math.log2(Ly) + 4 * Ly)
    tflops = flop / (ms * 1e-3) / 1e12
    loop = {name: round((clock.ms[k] / max(1, clock.launches[k]) - ev_ms) * 1e3, 2)
            for k, name in enumerate(("update_r2c", "column_conv", "gap_c2r", "direction_r2c",
                                      "column_energy"))}
    # second convolution's column kernel: reads S and the spectrum quarter
    e_bytes = info.ny * Lx * 8 + (Lx + 1) * (Ly + 1) * 4
    e_ms = clock.ms[4] / max(1, clock.launches[4]) - ev_ms
    return {"bound": "hbm", "kernel": "k_col_conv_w<2048,2> (column sweep, FP32)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "ms_per_launch": round(ms, 5), "launches_timed": n_col,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "timing": "HIP events on the solver stream around each column launch of one "
                      "sweep of the timed workload (run after the timed steps), launches past "
                      "convergence excluded, less the interval of two events recorded back to "
                      "back (the event's own cost on the stream)",
            "ms_per_launch_events": round(ms_raw, 5), "event_record_ms": round(ev_ms, 5),
            "isolated_ms_per_launch": round(iso, 5),
            "device_copy_GBps": {"same_bytes": round(copy_same, 1), "2x1GiB": round(copy_hbm, 1)},
            "frac_of_device_copy": round(achieved / copy_same, 4),
            "alu_view": {"flop_per_launch": round(flop), "achieved": round(tflops, 2),
                         "peak": 78.6, "unit": "TFLOP/s", "frac": round(tflops / 78.6, 4)},
            "loop_us_per_launch": loop,
            "column_energy": {"ms_per_launch": round(e_ms, 5), "algorithmic_bytes_per_launch":
                              e_bytes, "GBps": round(e_bytes / (e_ms * 1e-3) / 1e9, 1)},
            "loop_us_per_iteration_events": round(clock.loop_ms() / clock.iterations * 1e3, 2),
            "gap_shift_launches": clock.shifts,
            "gap_shift_us_per_launch": round(clock.shift_ms / max(1, clock.shifts) * 1e3, 2),
            "skipped_launches": clock.skipped,
            "skipped_us_total": round(clock.skipped_ms * 1e3, 1)}


def cpu_baseline(h, depths, iters_per_solve, sample_iters):
    """The FP64 oracle on the host cores: `sample_iters` CG iterations of the
    first depth, scaled to solves/s with the GPU FP64 mean iterations/solve."""
    from oracle import influence as inf
    from oracle import material as m
    from oracle import solver as so
    from oracle.convolution import FFTConvolver
    # worker threads: the CPUs this process may use, capped by OMP_NUM_THREADS
    cores = len(os.sched_getaffinity(0))
    cores = max(1, min(cores, int(os.environ.get("OMP_NUM_THREADS", cores))))
    dx = L / N
    t_setup = time.perf_counter()
    Kq = inf.influence_quarter(N, N, dx, dx, K_EXP)
    conv = FFTConvolver(Kq, m.compliance(K_EXP, NU), workers=cores)
    t_setup = time.perf_counter() - t_setup
    t0 = time.perf_counter()
    so.solve_nonadhesive(Kq, m.compliance(K_EXP, NU), h, depths[-1], tol=1e-12,
                         max_iter=sample_iters, conv=conv)
    t = time.perf_counter() - t0
    # sample_iters iterations plus one extra convolution at the final check
    per_iter = t / (sample_iters + 0.5)
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(1.0 / (per_iter * iters_per_solve), 5), "unit": "solves/s",
            "cores": cores, "cpu_model": cpu_model, "kind": "oracle",
            "sample": (f"{sample_iters} CG iterations of the FP64 oracle (numpy/scipy.fft, "
                       f"{cores} workers) at 2048^2, depth d10, {t:.1f} s; scaled by the GPU "
                       f"FP64 mean of {iters_per_solve:.1f} iterations/solve; influence "
                       f"setup {t_setup:.1f} s not counted"),
            "s_per_iter": round(per_iter, 4), "units": oracle_units(cores, Kq, h, depths)}


# Depth of 10 % contact area of the 4096^2 workload, by bisection on the
# MIXED GPU path (`python bench.py --find-d10-4096`); about 11 max(h): with
# k = -0.3 the long-range response keeps most of the surfaces apart.
D10_4096 = 0.0837569479935818


def big_grid_setup(bem, torch):
    from paper_1612_08395_amd import inputs
    n = 4096
    two_pi = 2.0 * math.pi / L
    h = inputs.fractal_gap(n, L, H_EXP, Q0 * two_pi, Q1 * two_pi, RMS * L, 8395)
    h_dev = torch.tensor(h, dtype=torch.float64, device="cuda")
    K = bem.bem_influence(n, n, L / n, -0.3, 0.25)
    return n, h_dev, K


def find_d10_4096(bem, torch):
    n, h_dev, K = big_grid_setup(bem, torch)
    st = bem.bem_state_create(K)

    def area(d):
        _, res = bem.bem_solve_dev(K, h_dev, bem.bem_params_init(d=d, precision=bem.BEM_MIXED),
                                   state=st)
        frac = res.n_contact / float(n * n)
        log(f"[d10-4096] d={d:.6e} area={frac:.5f} iters={res.iters}")
        return frac

    # with k < 0 the long-range response keeps most of the surface apart even
    # beyond d = max h: widen the bracket until it holds 10 % area
    lo, hi = 0.0, float(h_dev.max().item())
    for _ in range(12):
        if area(hi) >= AREA_FRAC:
            break
        lo, hi = hi, 2.0 * hi
    d = 0.5 * (lo + hi)
    for _ in range(40):
        d = 0.5 * (lo + hi)
        frac = area(d)
        if abs(frac - AREA_FRAC) <= 0.01 * AREA_FRAC:
            break
        if frac < AREA_FRAC:
            lo = d
        else:
            hi = d
    st.free()
    K.free()
    return d


def big_grid(bem, torch, depths_n=5):
    """4096^2 (8192^2 padded) rough surface, k = -0.3, nu = 0.25, seed 8395,
    same H / q0 / q1 as the 2048^2 workload: mixed-precision indentation
    sweep of 5 depths up to D10_4096 (10 % contact area).  Its ~0.75 GB
    working set exceeds the 256 MB last-level cache, so this is the
    HBM-resident figure."""
    n, h_dev, K = big_grid_setup(bem, torch)
    dq = D10_4096 if D10_4096 is not None else find_d10_4096(bem, torch)
    depths = [dq * s / depths_n for s in range(1, depths_n + 1)]

    def sweep():
        st = bem.bem_state_create(K)
        res = []
        for d in depths:
            _, r = bem.bem_solve_dev(K, h_dev, bem.bem_params_init(d=d, precision=bem.BEM_MIXED),
                                     state=st)
            res.append(r.as_dict())
        st.free()
        return res

    sweep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = sweep()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    bem.bem_clock_start()          # per-kernel durations from one more, instrumented sweep
    sweep()
    torch.cuda.synchronize()
    clk = bem.bem_clock_stop()
    # accuracy of the mixed path at the last depth against the FP64 path (cold
    # solves, untimed): this grid and k = -0.3 sit at the FP32 floor
    p32 = torch.empty_like(h_dev)
    p64 = torch.empty_like(h_dev)
    _, r32 = bem.bem_solve_dev(K, h_dev, bem.bem_params_init(d=dq, precision=bem.BEM_MIXED),
                               p_out=p32)
    _, r64 = bem.bem_solve_dev(K, h_dev, bem.bem_params_init(d=dq), p_out=p64)
    torch.cuda.synchronize()
    acc = {"rel_l2_pressure": float(f"{float(torch.linalg.norm(p32 - p64) / torch.linalg.norm(p64)):.3e}"),
           "contact_count_rel_diff": float(f"{abs(r32.n_contact - r64.n_contact) / r64.n_contact:.3e}"),
           "status_mixed": r32.status, "residual_mixed": float(f"{r32.residual:.3e}"),
           "iters_mixed": r32.iters, "iters_fp64": r64.iters}
    del p32, p64
    K.free()
    iters = sum(r["iters"] for r in res)
    # event intervals less the cost of one event record (the interval of the
    # two events recorded back to back at the end of each iteration)
    ev_ms = clk.ms[5] / max(1, clk.launches[5])
    col_ms = clk.ms[1] / clk.launches[1] - ev_ms
    col_bytes = 2 * n * n * 8 + (n + 1) * (n + 1) * 4
    return {"n": n, "padded": 2 * n, "k": -0.3, "nu": 0.25, "seed": 8395,
            "depths": depths_n, "d_max": dq, "solves_per_s": round(depths_n / t, 3),
            "iters_per_solve": round(iters / depths_n, 2),
            "loop_us_per_iteration": round(t / iters * 1e6, 2),
            "loop_GBps_algorithmic": round(sum(loop_bytes(r["n_contact"] / (n * n)) * n * n
                                               * r["iters"] for r in res) / t / 1e9, 1),
            "column_us_per_launch": round(col_ms * 1e3, 2),
            "column_GBps_algorithmic": round(col_bytes / (col_ms * 1e-3) / 1e9, 1),
            "contact_area_final": res[-1]["n_contact"] / float(n * n),
            "mixed_vs_fp64_last_depth": acc}


# Adhesive leg of the 4096^2 workload: work of adhesion 1e-4 E0 L (the third
# of the four values {1, 3, 10, 30} 1e-5 the crop tests sweep), 10 loading
# depths up to D10_4096, then 10 pull-off steps of D10_4096 / 20 down to half
# of it.  (Further down the detachment front needs hundreds of detach rounds
# per step: a full pull-off of this grid takes minutes in MIXED and far
# longer in FP64, beyond a bench leg.)
GAMMA_4096 = 1e-4


def adhesive_4096(bem, torch, n_load=10, n_unload=10):
    """Load-unload hysteresis of the 4096^2 rough surface with adhesion
    (Section 3.1): loading steps are non-adhesive solves, each pull-off step
    an adhesive solve with detach rounds, all warm-started on one state.  Run
    step by step in MIXED and in FP64; per step the force, contact count,
    iterations and detach rounds of both, and the MIXED-vs-FP64 pressure
    difference."""
    n, h_dev, K = big_grid_setup(bem, torch)
    dq = D10_4096
    depths = [dq * s / n_load for s in range(1, n_load + 1)]
    depths += [dq * (1.0 - 0.5 * s / n_unload) for s in range(1, n_unload + 1)]
    out = {"n": n, "padded": 2 * n, "k": -0.3, "nu": 0.25, "seed": 8395, "gamma": GAMMA_4096,
           "p_crit": bem.bem_p_crit(-0.3, 0.25, GAMMA_4096, L / n),
           "depths": [float(f"{d:.6e}") for d in depths]}
    runs = {}
    for prec, name in ((bem.BEM_MIXED, "mixed"), (bem.BEM_FP64, "fp64")):
        st = bem.bem_state_create(K)
        ps, rs = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, d in enumerate(depths):
            unload = i >= n_load
            prm = bem.bem_params_init(d=d, precision=prec, gamma=GAMMA_4096 if unload else 0.0)
            p = torch.empty_like(h_dev)
            _, r = bem.bem_solve_dev(K, h_dev, prm, state=st, p_out=p)
            ps.append(p)
            rs.append(r.as_dict())
            torch.cuda.synchronize()
            log(f"[adhesive-4096] {name} step {i} d={d:.4e} F={r.F:.4e} contact={r.n_contact} "
                f"iters={r.iters} rounds={r.detach_rounds} status={r.status} "
                f"t={time.perf_counter() - t0:.1f}s")
        torch.cuda.synchronize()
        runs[name] = (time.perf_counter() - t0, ps, rs)
        st.free()
    t32, p32, r32 = runs["mixed"]
    t64, p64, r64 = runs["fp64"]
    out["mixed_s"] = round(t32, 2)
    out["fp64_s"] = round(t64, 2)
    steps = []
    for i in range(len(depths)):
        a, b = p32[i], p64[i]
        nb = float(torch.linalg.norm(b))
        steps.append({
            "d": float(f"{depths[i]:.5e}"), "phase": "load" if i < n_load else "unload",
            "F_mixed": float(f"{r32[i]['F']:.6e}"), "F_fp64": float(f"{r64[i]['F']:.6e}"),
            "contact_mixed": r32[i]["n_contact"], "contact_fp64": r64[i]["n_contact"],
            "rel_l2_pressure": float(f"{float(torch.linalg.norm(a - b)) / nb:.3e}") if nb > 0
            else 0.0,
            "iters_mixed": r32[i]["iters"], "iters_fp64": r64[i]["iters"],
            "rounds_mixed": r32[i]["detach_rounds"], "rounds_fp64": r64[i]["detach_rounds"],
            "status_mixed": r32[i]["status"], "status_fp64": r64[i]["status"]})
    out["steps"] = steps
    del p32, p64
    K.free()
    return out


def oracle_units(cores, Kq, h=None, depths=None):
    """Further oracle timings (FP64 numpy / scipy.fft): one 2048^2
    convolution on `cores` workers and on one; the 128^2 Hertz-type solve
    (k = 0.5, nu = 0.3, R = 1, side 2, d = 0.01, tol 1e-12); one pull-off
    step of the 512^2 adhesive example (k = 0, gamma = 2.9995e-3, preload to
    (1.5 a_F)^2 / R untimed, then the step at half that depth); one 256^2
    window of the 4096^2 surface (k = -0.3, nu = 0.25, 10 % height quantile);
    and step 5 of the 20-step 2048^2 sweep, cold started (the deepest step
    is the sampled iterations scaled, see cpu_baseline)."""
    from oracle import influence as inf
    from oracle import material as m
    from oracle import solver as so
    from oracle.convolution import FFTConvolver
    from paper_1612_08395_amd import inputs
    out = {}
    p = inputs.random_pressure(N, N, 3)
    for w, key in ((cores, "convolution_2048_s"), (1, "convolution_2048_1thread_s")):
        conv = FFTConvolver(Kq, m.compliance(K_EXP, NU), workers=w)
        conv(p)
        t0 = time.perf_counter()
        conv(p)
        out[key] = round(time.perf_counter() - t0, 4)
    n1, L1 = 128, 2.0
    dx = L1 / n1
    Kq1 = inf.influence_quarter(n1, n1, dx, dx, 0.5)
    h1 = inputs.parabolic(n1, L1, 1.0)
    t0 = time.perf_counter()
    so.solve_nonadhesive(Kq1, m.compliance(0.5, 0.3), h1, 0.01, tol=1e-12)
    out["solve_128_hertz_s"] = round(time.perf_counter() - t0, 4)
    # 512^2 adhesive example: preload (untimed), then one pull-off step
    n2, L2, gam = 512, 2.0, 2.9995e-3
    dx2 = L2 / n2
    Kq2 = inf.influence_quarter(n2, n2, dx2, dx2, 0.0)
    C2 = m.compliance(0.0, 0.3)
    conv2 = FFTConvolver(Kq2, C2, workers=cores)
    h2 = inputs.parabolic(n2, L2, 1.0)
    d0 = (1.5 * 0.213) ** 2
    pre = so.solve_nonadhesive(Kq2, C2, h2, d0, tol=1e-12, conv=conv2)
    t0 = time.perf_counter()
    so.adhesive_step(Kq2, C2, h2, 0.5 * d0, pre.p > 0, pre.p,
                     m.p_crit(0.0, 0.3, gam, dx2), tol=1e-12, conv=conv2)
    out["adhesive_step_512_s"] = round(time.perf_counter() - t0, 4)
    # a 256^2 window of the 4096^2 surface
    n4, w = 4096, 256
    h4 = inputs.fractal_gap(n4, L, H_EXP, Q0 * 2 * math.pi / L, Q1 * 2 * math.pi / L, RMS * L,
                            8395)
    hw = h4[n4 // 4 - w // 2: n4 // 4 + w // 2, n4 // 4 - w // 2: n4 // 4 + w // 2].copy()
    del h4
    hw -= hw.min()
    Kq4 = inf.influence_quarter(w, w, L / n4, L / n4, -0.3)
    t0 = time.perf_counter()
    so.solve_nonadhesive(Kq4, m.compliance(-0.3, 0.25), hw, float(np.quantile(hw, 0.1)),
                         tol=1e-12, conv=FFTConvolver(Kq4, m.compliance(-0.3, 0.25),
                                                      workers=cores))
    out["crop_256_solve_s"] = round(time.perf_counter() - t0, 4)
    # a step of the 2048^2 sweep, solved from a cold start
    if h is not None and depths is not None:
        conv = FFTConvolver(Kq, m.compliance(K_EXP, NU), workers=cores)
        for s_i in (5,):
            t0 = time.perf_counter()
            r = so.solve_nonadhesive(Kq, m.compliance(K_EXP, NU), h, depths[s_i - 1], tol=1e-12,
                                     conv=conv)
            out[f"solve_2048_step{s_i}_s"] = round(time.perf_counter() - t0, 3)
            out[f"solve_2048_step{s_i}_iters"] = int(r.iters)
    return out


def serving(count, slots, bem):
    """Request stream of mixed grids (64^2..1024^2), k, indenters, 50 %
    adhesive (inputs.serving_requests): saturation throughput of each path
    with continuous batching (16 slots per geometry class), then Poisson
    arrivals at 0.8 x the FP64 saturation rate for both paths; the MIXED
    saturation run once more without batching (every request a solve of its
    own) and with continuous k (no influence operator reused) for
    comparison; and the requests the MIXED path stopped at its
    rounding floor (BEM_EFLOOR), solved alone in both precisions, with their
    pressure difference; then the loading curves of the requests with and
    without server sessions (serving.run_curves)."""
    from paper_1612_08395_amd import inputs
    from paper_1612_08395_amd.serving import KEYS_POISSON, KEYS_SAT, run_stream
    reqs = inputs.serving_requests(count, 2024)
    out = {"requests": count, "slots": slots, "batch_slots": 16, "budget_bytes": 8 << 30}
    sat = {}
    floor_idx = []
    for prec, name in ((bem.BEM_FP64, "fp64"), (bem.BEM_MIXED, "mixed")):
        s = run_stream(reqs, prec, None, slots)
        sat[name] = s["solves_per_s"]
        out[f"{name}_saturation"] = {k: s[k] for k in KEYS_SAT}
        if prec == bem.BEM_MIXED:
            floor_idx = [j for j, st in enumerate(s["statuses"]) if st == bem.BEM_EFLOOR]
    s = run_stream(reqs, bem.BEM_MIXED, None, slots, batch_slots=0)
    out["mixed_saturation_unbatched"] = {k: s[k] for k in KEYS_SAT}
    # the same stream with continuous k: every request builds its influence
    s = run_stream(inputs.serving_requests(count, 2024, continuous_k=True), bem.BEM_MIXED, None,
                   slots)
    out["mixed_saturation_continuous_k"] = {k: s[k] for k in KEYS_SAT}
    qps = 0.8 * sat["fp64"]
    for prec, name in ((bem.BEM_FP64, "fp64"), (bem.BEM_MIXED, "mixed")):
        s = run_stream(reqs, prec, qps, slots, seed=7)
        out[f"{name}_poisson"] = {k: s[k] for k in KEYS_POISSON}
    floors = []
    for j in floor_idx:
        r = reqs[j]
        n = r["n"]
        K = bem.bem_influence(n, n, 1.0 / n, r["k"], 0.3)
        ps = {}
        for prec in (bem.BEM_MIXED, bem.BEM_FP64):
            prm = bem.bem_params_init(d=r["d"], d_preload=r["d_preload"], gamma=r["gamma"],
                                      precision=prec)
            _, res, p, c, _ = bem.bem_solve(K, r["h"], prm)
            ps[prec] = (p, int(c.sum()), res)
        K.free()
        p32, c32, r32 = ps[bem.BEM_MIXED]
        p64, c64, _ = ps[bem.BEM_FP64]
        nrm = float(np.linalg.norm(p64))
        floors.append({"n": n, "k": r["k"], "shape": r["shape"], "adhesive": r["gamma"] > 0,
                       "residual_mixed": float(f"{r32.residual:.3e}"),
                       "rel_l2_pressure_vs_fp64": float(f"{np.linalg.norm(p32 - p64) / nrm:.3e}")
                       if nrm > 0 else 0.0,
                       "contact_mixed": c32, "contact_fp64": c64})
    out["mixed_floor_requests"] = floors
    # loading curves (8 steps each; adhesive requests 4 loading + 4 pull-off
    # steps) of the stream's requests, MIXED: one server session per curve
    # (state resident on the device, each step warm-started) against every
    # step an independent cold request
    from paper_1612_08395_amd.serving import run_curves
    cur = reqs
    out["curves_mixed"] = {"sessions": run_curves(cur, bem.BEM_MIXED, True, n_slots=slots),
                           "independent": run_curves(cur, bem.BEM_MIXED, False, n_slots=slots)}
    return out


def profile_kernels(bem, torch):
    """Few launches of each sweep kernel at 2048^2 and of the FP32 sweeps at
    4096^2 (for rocprofv3 --pmc), one
    mixed-precision solve of the bench workload at the deepest depth (the
    fused CG kernels), and a plain device copy of 2^28 floats (1 GiB read +
    1 GiB written) whose counter readings calibrate FETCH_SIZE / WRITE_SIZE."""
    K = bem.bem_influence(N, N, L / N, K_EXP, NU)
    out = {}
    for prec, name in ((bem.BEM_MIXED, "f32"), (bem.BEM_FP64, "f64")):
        for which, kname in ((0, "row_r2c"), (1, "col_conv"), (2, "row_c2r")):
            out[f"{kname}_{name}_ms"] = bem.bem_kernel_time(K, prec, which, reps=4)
    # the FP32 sweeps of the 4096^2 workload (k = -0.3, nu = 0.25)
    K4 = bem.bem_influence(4096, 4096, L / 4096, -0.3, 0.25)
    for which, kname in ((0, "row_r2c"), (1, "col_conv"), (2, "row_c2r"), (3, "col_energy")):
        out[f"{kname}_f32_4096_ms"] = bem.bem_kernel_time(K4, bem.BEM_MIXED, which, reps=2)
    K4.free()
    h_dev = torch.tensor(workload(), dtype=torch.float64, device="cuda")
    _, res = bem.bem_solve_dev(K, h_dev, bem.bem_params_init(d=D10, precision=bem.BEM_MIXED))
    out["solve_iters"] = res.iters
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    out["copy_bytes_each_way"] = 4 << 28
    print(json.dumps(out), flush=True)
    K.free()
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=8)
    ap.add_argument("--find-d10", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=300,
                    help="requests per serving run (0: skip the serving measurement)")
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--chains", type=int, default=2,
                    help="concurrent warm-start chains of the timed sweeps (1..8)")
    ap.add_argument("--find-d10-4096", action="store_true")
    ap.add_argument("--no-big-grid", action="store_true",
                    help="skip the 4096^2 (HBM-resident) mixed sweep")
    ap.add_argument("--no-adhesive-4096", action="store_true",
                    help="skip the 4096^2 adhesive load-unload leg (MIXED and FP64 per step)")
    ap.add_argument("--only-adhesive-4096", action="store_true",
                    help="run only the 4096^2 adhesive load-unload leg and print its JSON")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only launch each convolution sweep kernel a few times (FP32 and FP64) "
                         "and a 1 GiB device copy, for hardware-counter runs")
    args = ap.parse_args()
    if args.steps < 1 or args.fp64_steps < 1 or args.warmup < 0 or not 1 <= args.chains <= 8:
        ap.error("--steps and --fp64-steps must be >= 1, --warmup >= 0, 1 <= --chains <= 8")
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        return 2

    import torch
    from paper_1612_08395_amd import bem
    torch.cuda.set_device(0)
    if args.profile_kernels:
        return profile_kernels(bem, torch)
    if args.find_d10_4096:
        print(json.dumps({"d10_4096": find_d10_4096(bem, torch)}), flush=True)
        return 0
    if args.only_adhesive_4096:
        print(json.dumps({"adhesive_4096": adhesive_4096(bem, torch)}), flush=True)
        return 0
    log("[bench] building workload")
    h = workload()
    h_dev = torch.tensor(h, dtype=torch.float64, device="cuda")
    K = bem.bem_influence(N, N, L / N, K_EXP, NU)
    d10 = D10
    if d10 is None or args.find_d10:
        d10 = find_d10(bem, K, h_dev, torch)
        log(f"[bench] d10 = {d10!r}")
        if args.find_d10:
            print(json.dumps({"d10": d10}), flush=True)
            return 0
    depths = [d10 * s / N_DEPTHS for s in range(1, N_DEPTHS + 1)]

    # accuracy of the mixed path against the FP64 path, per depth (untimed)
    log("[bench] mixed vs FP64 pressures")
    r64, p64 = run_sweep(bem, K, h_dev, depths, bem.BEM_FP64, keep_p=True, torch=torch)
    r32, p32 = run_sweep(bem, K, h_dev, depths, bem.BEM_MIXED, keep_p=True, torch=torch)
    err = [float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) for a, b in zip(p32, p64)]
    cnt = [abs(x["n_contact"] - y["n_contact"]) / max(1, y["n_contact"]) for x, y in zip(r32, r64)]
    del p64, p32

    log("[bench] timed mixed sweeps")
    t32, res32, clk32 = timed(bem, K, h_dev, depths, bem.BEM_MIXED, args.steps, args.warmup,
                              torch, args.chains)
    t32s, res32s, _ = timed(bem, K, h_dev, depths, bem.BEM_MIXED, args.steps, 0, torch, 1,
                            clock=False)
    log("[bench] timed FP64 sweeps")
    # FP64: one chain (its kernels overlap less, and a second chain measured
    # slower than the sequential sweep)
    t64, res64, clk64 = timed(bem, K, h_dev, depths, bem.BEM_FP64, args.fp64_steps, 0, torch, 1)
    it32 = [x["iters"] for x in res32[-1]]
    it64 = [x["iters"] for x in res64[-1]]
    solves32 = N_DEPTHS * args.steps / t32
    solves64 = N_DEPTHS * args.fp64_steps / t64
    ms_step = t32 / args.steps * 1e3
    # whole-loop effective bandwidth: algorithmic bytes per element per CG
    # iteration (five launches) 79 + 16 f in FP32, with f the contact
    # fraction (the direction and update prologues read t and g, and the
    # direction prologue writes t, only in the contact set), 155 + 32 f in
    # FP64; f of each solve's final contact set
    loop32 = sum(loop_bytes(x["n_contact"] / (N * N)) * N * N * x["iters"]
                 for x in res32[-1]) / (t32 / args.steps) / 1e9
    loop64 = sum(loop_bytes(x["n_contact"] / (N * N), 8) * N * N * x["iters"]
                 for x in res64[-1]) / (t64 / args.fp64_steps) / 1e9

    log("[bench] roofline")
    roof = roofline(bem, K, clk32, torch)
    out = {
        "metric": METRIC, "value": round(solves32, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "rough-surface indentation sweep 2048^2 (4096^2 padded), "
                               "k=0.3 nu=0.3, 20 depths to 10% contact, mixed precision",
                   "n": N, "padded": 2 * N, "k": K_EXP, "nu": NU, "H": H_EXP,
                   "q0_over_2pi_L": Q0, "q1_over_2pi_L": Q1, "rms_over_L": RMS, "seed": SEED,
                   "depths_per_step": N_DEPTHS, "d10": d10, "chains": args.chains,
                   "sweep": f"bem_sweep_dev: {args.chains} concurrent warm-start chains "
                            f"(chain c solves depths c, c + {args.chains}, ...)"},
        "single_chain": {"value": round(N_DEPTHS * args.steps / t32s, 3), "unit": "solves/s",
                         "iters_per_solve": round(sum(x["iters"] for x in res32s[-1])
                                                  / N_DEPTHS, 2),
                         # whole sweep time (no events) per CG iteration
                         "loop_us_per_iteration": round(
                             t32s / args.steps / sum(x["iters"] for x in res32s[-1]) * 1e6, 2)},
        "roofline": roof,
        "fp64": {"value": round(solves64, 3), "unit": "solves/s", "steps": args.fp64_steps,
                 "chains": 1,
                 "ms_per_step": round(t64 / args.fp64_steps * 1e3, 3),
                 "iters_per_solve": round(sum(it64) / len(it64), 2),
                 "loop_GBps_algorithmic": round(loop64, 1),
                 "column_us_per_launch": round(clk64.ms[1] / clk64.launches[1] * 1e3, 2)},
        "iters_per_solve": round(sum(it32) / len(it32), 2),
        "loop_GBps_algorithmic": round(loop32, 1),
        "mixed_vs_fp64": {"rel_l2_pressure_per_depth": [float(f"{e:.3e}") for e in err],
                          "contact_count_rel_diff_per_depth": [float(f"{c:.2e}") for c in cnt],
                          "status_mixed": sorted({x["status"] for x in res32[-1]})},
        "contact_area_final": res32[-1][-1]["n_contact"] / float(N * N),
    }
    # compulsory traffic: the first convolution reads its input and the kernel
    # spectrum quarter and writes its output (12 B per element in FP32), the
    # second (an inner product) reads its input and the spectrum (8 B)
    comp = 20.0 * N * N * sum(it32) / (t32 / args.steps) / 1e9
    out["compulsory_GBps"] = round(comp, 1)
    out["compulsory_frac"] = round(comp / HBM_PEAK_GBS, 4)
    # the remaining legs report beside the headline; a failure in one of them
    # is recorded in its field (and the exit status) instead of losing the line
    failed = False

    def leg(key, fn):
        nonlocal failed
        try:
            out[key] = fn()
        except Exception as e:  # noqa: BLE001
            failed = True
            out[key] = {"error": f"{type(e).__name__}: {e}"}
            log(f"[bench] {key} failed: {e}")

    if not args.no_big_grid:
        log("[bench] 4096^2 sweep")
        leg("hbm_resident_4096", lambda: big_grid(bem, torch))
    if not args.no_adhesive_4096:
        log("[bench] 4096^2 adhesive load-unload")
        leg("adhesive_4096", lambda: adhesive_4096(bem, torch))
    if args.serving_requests > 0:
        log("[bench] serving")
        leg("serving", lambda: serving(args.serving_requests, args.serving_slots, bem))
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        leg("cpu_baseline",
            lambda: cpu_baseline(h, depths, sum(it64) / len(it64), args.cpu_iters))
    print(json.dumps(out), flush=True)
    if failed:
        K.free()
        return 1
    K.free()
    return 0


if __name__ == "__main__":
    sys.exit(main())
