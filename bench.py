"""Benchmark: directional-preconditioned CFIE solves on one MI355X.

Workload: the sound-hard kite x = cos t + 0.65 cos 2t - 0.65, y = 1.5 sin t,
n = 32768 arclength-equispaced nodes at 10 points per wavelength
(omega = 2208.1), eta = omega, 64 incident plane waves at angles 2 pi k/64,
all solved to FP64 relative residual 1e-8 with the directional
preconditioner.  Two solvers are timed on the same workload: mixed precision
(iterative refinement: FP64 residuals, corrections from right-preconditioned
GMRES(80) on the single-precision operator) and plain FP64 GMRES(80).

A step is the whole job: problem creation from the host geometry (upload,
Kress and diagonal tables, near-field list) -> preconditioner setup ->
plane-wave data -> the batched solve -> q copied to host memory; the problem
is destroyed after each step.  value = solved right-hand sides per second of
the mixed solver over the timed steps; the FP64 solver's figures, and both
solvers on a problem that stays resident (setup-excluded: preconditioner,
data and solve only), are reported beside it.

Prints one JSON line (metric, value, roofline of the dominant pair-sweep kernel
from HIP events recorded by the library around each of its launches, both
solvers' throughput and latency, GMRES iterations with and without the
preconditioner, the serving stream, and the CPU oracle's extrapolated rate on
a bounded sample).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CFIE solves/s at n=32768 to 1e-8 residual (mixed vs FP64); p50/p99 latency"
# FP64 peak, TFLOP/s: dense MFMA and vector FMA are both 256 CU x 4 SIMD x 32 flop/clk x 2.4 GHz
PEAK_FP64_VALU = 78.6
# FP32 vector peak (256 CU x 4 SIMD x 64 flop/clk x 2.4 GHz, packed FP32) and
# dense FP16 matrix-core peak, TFLOP/s: the single-precision sweep evaluates
# its kernel values on the vector ALUs and multiplies split-FP16 operands on
# the matrix cores; the two do not issue concurrently on one SIMD, so its
# time is bounded below by the sum of the two.
PEAK_FP32_VALU = 157.3
PEAK_FP16_MFMA = 2500.0
# Executed matrix-core flops per pair, density and column in that sweep: a
# complex product is 4 real products, each split into 3 FP16 products.
FLOPS_MFMA16_PER_COL = 24
# HBM bytes per launch of the two 64-column hard sweeps at n = 32768 with the
# default 2048-block grid (rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by the
# counts of a 512 MiB device copy in the same run; FETCH_SIZE counts half the
# bytes the copy moves).  They describe the current kernels in that
# configuration; another configuration or a changed kernel must be measured
# again before they are reported.
TRAFFIC_FP64_SWEEP = 1.1280e9 + 0.2705e9
TRAFFIC_FP32_SWEEP = 0.3025e9 + 0.2684e9

# Algorithmic FP64 flops of one ordered pair in the sound-hard sweep (far-field
# evaluation path; an FMA counts 2): geometry 5, 1/r 8, r and z 2, H0/H1 142,
# weights 2, nu_i.rhat 4, S / D' / G assembly 27; plus 2 complex MACs (8 flops
# each, the textbook count) per right-hand side.  The kernel executes each
# complex MAC as 3 real MFMA products (6 flops), so the achieved algorithmic
# rate may exceed the 8-flop accounting of the hardware.
FLOPS_PAIR_HARD = 190
FLOPS_PAIR_PER_RHS_HARD = 16


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(b, om, eta, nrhs, budget_s=25.0):
    """The oracle (dense Nystrom assembly + LU) timed on the host, on a sample.

    Sample: (a) oracle S and D' rows for 256 target rows at the full n (pair
    evaluations scale with n^2 -> x n/256); (b) the oracle's dense hard matrix
    at n0 = 1024 and 2048 on the same curve, its LU and 64 triangular solves;
    the cubic parts (Maue products, LU) are extrapolated from n0 = 2048 with
    (n/n0)^3, and the exponent measured between 1024 and 2048 is reported
    beside it.  The extrapolated time of one 64-RHS dense solve at n gives
    solves/s = nrhs / T.
    """
    import oracle.nystrom as ny
    from synth import sample_boundary, omega_for_ppw
    import scipy.linalg as sla

    n = b.n
    t0 = time.perf_counter()
    rows = np.arange(0, n, n // 256)[:256]
    ny.layer_rows(b, om, rows)
    t_rows = time.perf_counter() - t0
    t_pairs = t_rows * n / len(rows)
    cubic = {}
    for n0 in (1024, 2048):
        b0 = sample_boundary(b.name, n0)
        om0 = omega_for_ppw(n0, b0.L, 10.0)
        t1 = time.perf_counter()
        ny.layer_rows(b0, om0)
        t_pairs0 = time.perf_counter() - t1
        t1 = time.perf_counter()
        A0 = ny.hard_matrix(b0, om0, om0)                  # includes the pair work again
        t_asm0 = time.perf_counter() - t1
        F0 = ny.plane_wave_rhs(b0, om0, 2 * np.pi * np.arange(nrhs) / nrhs, 1)
        t1 = time.perf_counter()
        lu = sla.lu_factor(A0)
        sla.lu_solve(lu, F0)
        t_lu0 = time.perf_counter() - t1
        cubic[n0] = max(t_asm0 - t_pairs0, 0.0) + t_lu0  # Maue products + LU + solves
    n0 = 2048
    expo = float(np.log(cubic[2048] / cubic[1024]) / np.log(2.0)) if cubic[1024] > 0 else None
    T = t_pairs + cubic[n0] * (n / n0) ** 3
    used = time.perf_counter() - t0
    hi = host_info()
    threads = hi["blas_threads"] or int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": nrhs / T,
        "unit": "solves/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": hi["cpu_model"],
        "logical_cpus": hi["logical_cpus"],
        "blas": hi["blas"],
        "blas_threads": hi["blas_threads"],
        "cubic_exponent_measured_1024_2048": expo,
        "sample": (f"extrapolated: oracle pair work on {len(rows)} of {n} rows (x{n // len(rows)}), "
                   f"dense Maue assembly + LU + {nrhs} solves at n={n0} (x(n/{n0})^3; measured exponent "
                   f"between n=1024 and 2048: {expo:.2f}); {used:.1f} s of CPU wall time, projected "
                   f"{T:.0f} s per {nrhs}-RHS solve"),
    }


def _stream_request(k, seed):
    """Request k of the serving stream: n = 64 round(e^U(ln 2048, ln 65536) / 64),
    the seeded random star with seed k (geometry seed = request id), sound-soft
    or sound-hard with probability 1/2, 1-16 plane waves at U(0, 2 pi) angles,
    10 points per wavelength, eta = omega."""
    from synth import omega_for_ppw, sample_boundary
    rng = np.random.default_rng([seed, k])
    n = int(64 * round(np.exp(rng.uniform(np.log(2048), np.log(65536))) / 64))
    kind = int(rng.integers(0, 2))
    nrhs = int(rng.integers(1, 17))
    ang = rng.uniform(0, 2 * np.pi, nrhs)
    b = sample_boundary(f"randstar{k}", n)
    return b, omega_for_ppw(n, b.L, 10.0), kind, ang


def make_stream(nreq, seed=7, workers=None):
    """The requests of the serving stream, sampled on host worker processes
    (started before the GPU is touched)."""
    import multiprocessing as mp
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        return pool.starmap(_stream_request, [(k, seed) for k in range(nreq)])


def run_stream(dp, reqs, arrivals, precision, slots):
    """Serve reqs (arrival offsets in seconds) on a fresh server; per-request
    latency = completion - arrival (submission at the arrival time)."""
    import threading
    nreq = len(reqs)
    srv = dp.Server(slots=slots)
    # warm-up: one small request (kernel loading)
    b, om, kind, ang = min(reqs, key=lambda r: r[0].n)
    srv.wait(srv.submit(b, om, om, kind, angles=ang, precision=precision))
    ids = [None] * nreq
    failed = []
    start = time.perf_counter()

    def submitter():
        try:
            for k, (b, om, kind, ang) in enumerate(reqs):
                d = start + arrivals[k] - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                ids[k] = srv.submit(b, om, om, kind, angles=ang, precision=precision)
        except Exception as e:  # reported by the waiting loop below
            failed.append(e)

    th = threading.Thread(target=submitter)
    th.start()
    res = []
    for k in range(nreq):
        while ids[k] is None:
            if failed:
                th.join()
                srv.close()
                raise failed[0]
            time.sleep(0.001)
        res.append(srv.wait(ids[k]))
        if (k + 1) % 25 == 0:
            log(f"  served {k + 1}/{nreq}")
    th.join()
    st = srv.stats()
    srv.close()
    lat = np.array([t["t_done"] - t["t_submit"] for _, _, t, _ in res])
    qw = np.array([t["t_admit"] - t["t_submit"] for _, _, t, _ in res])
    t_first = min(t["t_submit"] for _, _, t, _ in res)
    t_last = max(t["t_done"] for _, _, t, _ in res)
    ev = sorted([(t["t_admit"], 1) for _, _, t, _ in res] + [(t["t_done"], -1) for _, _, t, _ in res])
    conc = peak = 0
    for _, d in ev:
        conc += d
        peak = max(peak, conc)
    solves = sum(r[3].size for r in reqs)
    return {
        "requests": nreq,
        "solves_per_s": solves / (t_last - t_first),
        "requests_per_s": nreq / (t_last - t_first),
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3),
                       "max": float(lat.max() * 1e3)},
        "queue_wait_ms": {"mean": float(qw.mean() * 1e3), "p99": float(np.percentile(qw, 99) * 1e3)},
        "makespan_s": t_last - t_first,
        "peak_concurrent": peak,
        "converged": all(r[3] == dp.DP_OK for r in res),
        "relres_max": float(max(r[1]["relres_max"] for r in res)),
        "mem_peak_gb": st["mem_peak"] / 1e9,
    }


def serve_stream(dp, reqs, slots, load=0.8, ncap=100, seed=11):
    """The serving stream of independent solve requests (see _stream_request),
    preconditioned, tolerance 1e-8 (FP64 residual), for each solver:
    capacity = completed requests per second when the first `ncap` requests
    all arrive at once (every slot kept busy); then all requests with Poisson
    arrivals at `load` x that capacity, with p50/p99 latency from arrival to
    completion."""
    out = {"requests": len(reqs), "slots": slots, "load": load,
           "rhs_total": int(sum(r[3].size for r in reqs)),
           "n_range": [int(min(r[0].n for r in reqs)), int(max(r[0].n for r in reqs))],
           "hard_fraction": float(np.mean([r[2] for r in reqs]))}
    for name, prec in (("mixed", dp.DP_PREC_MIXED), ("fp64", dp.DP_PREC_FP64)):
        cap = run_stream(dp, reqs[:ncap], np.zeros(ncap), prec, slots)
        log(f"serve [{name}] capacity: {json.dumps(cap)}")
        rate = load * cap["requests_per_s"]
        rng = np.random.default_rng(seed)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, len(reqs)))
        arrivals -= arrivals[0]
        loaded = run_stream(dp, reqs, arrivals, prec, slots)
        loaded["arrival_rate_per_s"] = rate
        log(f"serve [{name}] at {load:.0%} of capacity: {json.dumps(loaded)}")
        out[name] = {"capacity_requests_per_s": cap["requests_per_s"], "capacity_solves_per_s": cap["solves_per_s"],
                     "capacity_run": cap, "loaded": loaded}
    return out


def host_info():
    """CPU model, BLAS library and its thread count of the host running the oracle."""
    import platform
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas, blas_threads = "unknown", None
    try:
        import scipy.linalg  # noqa: F401  (loads LAPACK/BLAS)
        from threadpoolctl import threadpool_info
        pools = [p for p in threadpool_info() if p.get("user_api") == "blas"]
        if pools:
            blas = f"{pools[0].get('internal_api')} {pools[0].get('version')} ({os.path.basename(pools[0].get('filepath', ''))})"
            blas_threads = pools[0].get("num_threads")
    except Exception:  # threadpoolctl missing: report what is known
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "blas": blas, "blas_threads": blas_threads}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precond", action="store_true")
    ap.add_argument("--precision", choices=("both", "fp64", "mixed"), default="both",
                    help="fp64: GMRES on the FP64 operator; mixed: iterative refinement with "
                         "FP32-operator corrections and FP64 residuals (same 1e-8 FP64 residual); "
                         "both (default): mixed is the reported value, FP64 is reported beside it")
    ap.add_argument("--serve", type=int, default=200, metavar="N",
                    help="also serve a stream of N independent requests (0: skip)")
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="Poisson arrival rate as a fraction of the measured capacity")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving stream (e.g. under a kernel trace of the slots' streams)")
    ap.add_argument("--no-iteration-study", action="store_true",
                    help="skip the unpreconditioned solves that give n_n beside n_p")
    ap.add_argument("--resident-only", action="store_true",
                    help="time only steps on a resident problem (no problem creation per step)")
    ap.add_argument("--autotune", action="store_true",
                    help="also time the sweep tuner on a resident problem (informational; the "
                         "timed steps create their problem and use the default launch configuration)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of MIB MiB (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); "
              "a multi-GPU split of the sweep by target rows is not built", file=sys.stderr)
        sys.exit(2)

    stream = None
    if args.serve > 0:
        t0 = time.perf_counter()
        stream = make_stream(args.serve)     # host processes, before the GPU is touched
        log(f"serving stream: {args.serve} requests sampled in {time.perf_counter() - t0:.1f} s")

    import torch
    import paper_1408_1578_amd as dp
    from synth import config_boundary, plane_wave_angles

    if args.serve_only:
        if not stream:
            sys.exit("bench.py: --serve-only needs --serve N > 0")
        out = {"serving": serve_stream(dp, stream, args.serve_slots, load=args.serve_load,
                                       ncap=min(100, len(stream)))}
        print(json.dumps(out), flush=True)
        return

    b, om, eta, kind = config_boundary("kite", args.n)
    nrhs = args.nrhs
    ctx = dp.Context(0)
    angles = plane_wave_angles(nrhs)
    f = torch.empty((nrhs, b.n), dtype=torch.complex128, device="cuda:0")
    q = torch.empty_like(f)
    q_host = torch.empty(q.shape, dtype=q.dtype, pin_memory=True)
    use_pc = not args.no_precond
    if args.copy_calibration:
        a = torch.empty(args.copy_calibration * (1 << 20) // 8, dtype=torch.float64, device="cuda:0")
        a.fill_(1.0)
        bb = torch.empty_like(a)
        torch.cuda.synchronize()
        bb.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + written")
        del a, bb

    def run(precision, full):
        """W + K steps of the whole job.  full: a step is problem creation (host
        geometry in) -> preconditioner -> plane-wave data -> batched solve -> q in
        host memory, the problem destroyed after it; otherwise the problem stays
        resident and a step is preconditioner -> data -> solve (q on the device)."""
        prec = dp.DP_PREC_MIXED if precision == "mixed" else dp.DP_PREC_FP64
        resident = None if full else dp.Problem.from_boundary(ctx, b, om, eta, kind)
        tag = f"{precision}{'' if full else ', resident'}"

        def step():
            t0 = time.perf_counter()
            prob = dp.Problem.from_boundary(ctx, b, om, eta, kind) if full else resident
            t_create = time.perf_counter() - t0
            if use_pc:
                dp.dp_precond_build(prob)
            dp.dp_rhs_plane_wave(prob, angles, f)
            t1 = time.perf_counter()
            info = dp.dp_solve(prob, f, q, tol=1e-8, restart=80, use_precond=use_pc, precision=prec)
            t2 = time.perf_counter()
            if full:
                q_host.copy_(q)          # synchronous: q is in host memory when the step ends
            dt = time.perf_counter() - t0
            info["t_create"] = t_create
            info["t_build_rhs"] = t1 - t0 - t_create
            info["t_solve"] = t2 - t1
            info["t_readback"] = time.perf_counter() - t2
            if full:
                info["precond"] = dp.dp_precond_get_info(prob) if use_pc else {}
                prob.close()
            return info, dt

        for w in range(args.warmup):
            info, dt = step()
            log(f"[{tag}] warmup {w}: {dt:.3f} s iters={info['iters_max']} relres={info['relres_max']:.2e}")
        torch.cuda.synchronize()
        lat, infos = [], []
        t0 = time.perf_counter()
        for s_ in range(args.steps):
            info, dt = step()
            lat.append(dt)
            infos.append(info)
            log(f"[{tag}] step {s_}: {dt:.3f} s iters={info['iters_max']} relres={info['relres_max']:.2e} "
                f"sweep {info['t_sweep'] / max(info['sweep_launches'], 1) * 1e3:.2f} ms x {info['sweep_launches']}"
                f" fp32 {info['t_sweep_fp32'] / max(info['sweep_launches_fp32'], 1) * 1e3:.2f} ms x "
                f"{info['sweep_launches_fp32']} refinements={info['refinements']}")
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        if resident is not None:
            pinfo = dp.dp_precond_get_info(resident) if use_pc else {}
            for i in infos:
                i["precond"] = pinfo
            resident.close()
        return T, lat, infos

    nrp = 1
    while nrp < nrhs and nrp < 64:
        nrp *= 2
    pairs = b.n * (b.n - 1)
    flops = pairs * (FLOPS_PAIR_HARD + FLOPS_PAIR_PER_RHS_HARD * nrp)
    flops_valu = pairs * FLOPS_PAIR_HARD                       # kernel values (vector ALUs)
    flops_mac = pairs * FLOPS_PAIR_PER_RHS_HARD * nrp          # complex MACs (textbook 8 flops each)
    flops_mfma16_exec = pairs * 2 * nrp * FLOPS_MFMA16_PER_COL  # split-FP16 products executed

    # lower bound on one single-precision sweep: pair arithmetic on the vector
    # ALUs plus the executed split-FP16 products on the matrix cores
    t_bound32 = flops_valu / (PEAK_FP32_VALU * 1e12) + flops_mfma16_exec / (PEAK_FP16_MFMA * 1e12)

    def sweep_rate(infos, key_l, key_t):
        launches = sum(i[key_l] for i in infos)
        t = sum(i[key_t] for i in infos)
        avg = t / max(launches, 1)
        return launches, avg, (flops / avg / 1e12 if avg > 0 else 0.0)

    def summary(precision, T, lat, infos):
        lat_ms = np.array(lat) * 1e3
        launches, avg, achieved = sweep_rate(infos, "sweep_launches", "t_sweep")
        out = {
            "value": nrhs * args.steps / T,
            "systems_per_s": args.steps / T,
            "ms_per_step": T / args.steps * 1e3,
            "converged": all(i["converged"] and i["relres_max"] <= 1e-8 for i in infos),
            "iterations": int(max(i["iters_max"] for i in infos)),
            "relres_max": float(max(i["relres_max"] for i in infos)),
            "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
            "phase_s_per_step": {
                "matvec": float(np.mean([i["t_matvec"] for i in infos])),
                "precond_apply": float(np.mean([i["t_apply"] for i in infos])),
                "krylov": float(np.mean([i["t_krylov"] for i in infos])),
                "precond_setup": float(np.mean([i["precond"].get("t_setup", 0.0) for i in infos])),
                "problem_create": float(np.mean([i["t_create"] for i in infos])),
                "precond_build_and_rhs_wall": float(np.mean([i["t_build_rhs"] for i in infos])),
                "solve_wall": float(np.mean([i["t_solve"] for i in infos])),
                "q_to_host": float(np.mean([i["t_readback"] for i in infos])),
            },
            "sweep_fp64": {"launch_ms": avg * 1e3, "launches": launches, "tflops": achieved,
                           "frac_fp64_peak": achieved / PEAK_FP64_VALU},
        }
        if precision == "mixed":
            l32, a32, ach32 = sweep_rate(infos, "sweep_launches_fp32", "t_sweep_fp32")
            out["refinements"] = int(max(i["refinements"] for i in infos))
            out["matvecs_fp32"] = int(max(i["matvecs_fp32"] for i in infos))
            out["sweep_fp32"] = {"launch_ms": a32 * 1e3, "launches": l32, "tflops": ach32,
                                 "frac_of_bound": t_bound32 / a32 if a32 > 0 else 0.0}
        return out

    tuned = None
    if args.autotune:
        tp = dp.Problem.from_boundary(ctx, b, om, eta, kind)
        tuned = {pr: dp.dp_autotune(tp, nrhs, dp.DP_PREC_MIXED if pr == "mixed" else dp.DP_PREC_FP64)
                 for pr in ("mixed", "fp64")}
        tp.close()
        log(f"autotune (informational): {tuned}")

    precisions = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    runs, resident_runs = {}, {}
    for precision in precisions:
        if not args.resident_only:
            runs[precision] = summary(precision, *run(precision, True))
        resident_runs[precision] = summary(precision, *run(precision, False))
    if args.resident_only:
        runs = resident_runs
    head = "mixed" if "mixed" in runs else "fp64"
    main_run = runs[head]

    if head == "mixed":
        sw = main_run["sweep_fp32"]
        t_launch = sw["launch_ms"] * 1e-3
        frac = (flops / t_launch / 1e12) / PEAK_FP16_MFMA if t_launch > 0 else 0.0
        roof = {"kernel": "sweep_mfma16<hard, 64 columns> (FP32 kernel values, FP64 phase reduction; "
                          "split-FP16 operands on v_mfma_f32_16x16x32_f16 with FP32 accumulation; 8 waves x "
                          "16 targets, LDS density tiles)",
                "bound": "mfma", "achieved": sw["tflops"], "peak": PEAK_FP16_MFMA, "unit": "TFLOP/s",
                "frac": frac, "traffic": TRAFFIC_FP32_SWEEP if b.n == 32768 and nrhs == 64 else None,
                "launch_ms": sw["launch_ms"], "launches": sw["launches"], "flops_per_launch": flops,
                "components": {
                    "mfma_fp16_algorithmic": {
                        "flops": flops_mac, "achieved": flops_mac / t_launch / 1e12, "peak": PEAK_FP16_MFMA,
                        "frac": flops_mac / t_launch / 1e12 / PEAK_FP16_MFMA},
                    "mfma_fp16_executed": {
                        "flops": flops_mfma16_exec, "achieved": flops_mfma16_exec / t_launch / 1e12,
                        "peak": PEAK_FP16_MFMA, "frac": flops_mfma16_exec / t_launch / 1e12 / PEAK_FP16_MFMA},
                    "valu_fp32": {
                        "flops": flops_valu, "achieved": flops_valu / t_launch / 1e12, "peak": PEAK_FP32_VALU,
                        "frac": flops_valu / t_launch / 1e12 / PEAK_FP32_VALU},
                    "composite_valu_plus_mfma": {
                        "t_bound_ms": t_bound32 * 1e3, "frac": sw["frac_of_bound"],
                        "note": "vector ALUs and matrix cores do not issue concurrently on a SIMD: the "
                                "launch takes at least the VALU time plus the executed FP16 product time"},
                }}
    else:
        sw = main_run["sweep_fp64"]
        roof = {"kernel": "sweep_mfma<hard, 64 columns, FP64> (v_mfma_f64_16x16x4 products; 8 waves, "
                          "shared kernel values, LDS density tiles)",
                "bound": "mfma", "achieved": sw["tflops"], "peak": PEAK_FP64_VALU, "unit": "TFLOP/s",
                "frac": sw["tflops"] / PEAK_FP64_VALU,
                "traffic": TRAFFIC_FP64_SWEEP if b.n == 32768 and nrhs == 64 else None,
                "launch_ms": sw["launch_ms"], "launches": sw["launches"], "flops_per_launch": flops}
    out = {
        "metric": METRIC,
        "value": main_run["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"sound-hard kite, n={b.n}, 10 points/wavelength (omega={om:.1f}), eta=omega, "
                        f"{nrhs} plane waves at 2*pi*k/{nrhs}, directional preconditioner + GMRES(80) "
                        f"to 1e-8 FP64 residual; " + ("mixed: iterative refinement with FP32-operator "
                                                      "corrections" if head == "mixed" else "FP64")
                        + ("; step = resident problem" if args.resident_only else
                           "; step = problem creation from host geometry to q in host memory"),
            "n": b.n, "nrhs": nrhs, "omega": om, "tol": 1e-8, "restart": 80,
            "precision": head, "precond": use_pc, "setup_included": not args.resident_only,
        },
        "converged": main_run["converged"],
        "iterations": main_run["iterations"],
        "relres_max": main_run["relres_max"],
        "latency_ms": main_run["latency_ms"],
        "roofline": roof,
        "precision_runs": runs,
        "setup_excluded_runs": resident_runs,
    }
    if tuned is not None:
        out["autotune"] = tuned
    # preconditioner structure of this workload
    if use_pc:
        tp = dp.Problem.from_boundary(ctx, b, om, eta, kind)
        dp.dp_precond_build(tp)
        pinfo = dp.dp_precond_get_info(tp)
        out["precond"] = {k: pinfo[k] for k in ("m", "NW", "nnzW", "nnzLU", "levels", "t_setup")}
        if not args.no_iteration_study:
            out["iteration_study"] = iteration_study(dp, ctx, tp, b, om, eta, kind, f, q, nrhs)
        tp.close()
    if stream:
        log(f"serving stream: {args.serve} requests ...")
        out["serving"] = serve_stream(dp, stream, args.serve_slots, load=args.serve_load,
                                      ncap=min(100, len(stream)))
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, bounded sample) ...")
        out["cpu_baseline"] = cpu_baseline(b, om, eta, nrhs)
    print(json.dumps(out), flush=True)


def iteration_study(dp, ctx, prob, b, om, eta, kind, f, q, nrhs):
    """GMRES iterations with (n_p) and without (n_n) the preconditioner, FP64
    (Sec. 3's table columns): at the bench workload (all columns), and for one
    plane wave along +x on the kite at n = 8192, 16384, 32768 (omega grows
    with n at 10 points per wavelength)."""
    import torch
    from synth import config_boundary
    out = {}
    dp.dp_rhs_plane_wave(prob, plane_wave_angles_all(nrhs), f)
    ip = dp.dp_solve(prob, f, q, tol=1e-8, restart=80, use_precond=True)
    i_n = dp.dp_solve(prob, f, q, tol=1e-8, restart=80, use_precond=False, max_iters=2000)
    out["bench_workload"] = {"n": b.n, "omega": om, "nrhs": nrhs, "n_p": int(ip["iters_max"]),
                             "n_n": int(i_n["iters_max"]), "n_n_converged": bool(i_n["converged"])}
    log(f"iterations at the bench workload: {out['bench_workload']}")
    rows = []
    for n in (8192, 16384, 32768):
        bb, omb, etab, kb = config_boundary("kite", n)
        pr = dp.Problem.from_boundary(ctx, bb, omb, etab, kb)
        dp.dp_precond_build(pr)
        f1 = torch.empty((1, n), dtype=torch.complex128, device="cuda:0")
        q1 = torch.empty_like(f1)
        dp.dp_rhs_plane_wave(pr, np.array([0.0]), f1)
        a = dp.dp_solve(pr, f1, q1, tol=1e-8, restart=80, use_precond=True)
        c = dp.dp_solve(pr, f1, q1, tol=1e-8, restart=80, use_precond=False, max_iters=2000)
        rows.append({"n": n, "omega": omb, "n_p": int(a["iters_max"]), "n_n": int(c["iters_max"]),
                     "n_n_converged": bool(c["converged"])})
        log(f"iterations vs omega: {rows[-1]}")
        pr.close()
    out["kite_hard_vs_omega"] = rows
    return out


def plane_wave_angles_all(nrhs):
    from synth import plane_wave_angles
    return plane_wave_angles(nrhs)


if __name__ == "__main__":
    main()
