"""Benchmark: directional-preconditioned CFIE solves on one MI355X.

Workload (one step): the sound-hard kite x = cos t + 0.65 cos 2t - 0.65,
y = 1.5 sin t, n = 32768 arclength-equispaced nodes at 10 points per
wavelength (omega = 2208.1), eta = omega, 64 incident plane waves at angles
2 pi k/64, all solved to FP64 relative residual 1e-8 with the directional
preconditioner.  Two solvers are timed on the same workload: mixed precision
(iterative refinement: FP64 residuals, corrections from right-preconditioned
GMRES(80) on the single-precision operator) and plain FP64 GMRES(80).  A step
= preconditioner setup + plane-wave data + the batched solve (the problem's
geometry, Kress table and near-field list are resident on the device before
the timed region).  value = solved right-hand sides per second of the mixed
solver; the FP64 solver's figures are reported beside it.

Prints one JSON line (metric, value, roofline of the dominant pair-sweep kernel
from HIP events recorded by the library around each of its launches, both
solvers' throughput and latency, and the CPU oracle's extrapolated rate on a
bounded sample).
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
# counts of a 512 MiB device copy in the same run).  They describe the current
# kernels in that configuration; another configuration or a changed kernel
# must be measured again before they are reported.
TRAFFIC_FP64_SWEEP = 1.4011e9
TRAFFIC_FP32_SWEEP = 0.5774e9

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
    evaluations scale with n^2 -> x n/256); (b) the oracle's dense hard matrix at
    n0 = 2048 on the same curve and its LU + 64 triangular solves (cubic parts
    scale with (n/n0)^3).  The extrapolated time of one 64-RHS dense solve at n
    gives solves/s = nrhs / T.
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
    n0 = 2048
    b0 = sample_boundary(b.name, n0)
    om0 = omega_for_ppw(n0, b0.L, 10.0)
    t1 = time.perf_counter()
    lay = ny.layer_rows(b0, om0)
    t_pairs0 = time.perf_counter() - t1
    t1 = time.perf_counter()
    A0 = ny.hard_matrix(b0, om0, om0)                  # includes the pair work again
    t_asm0 = time.perf_counter() - t1
    t_cubic_asm0 = max(t_asm0 - t_pairs0, 0.0)         # dense products of Maue's identity
    F0 = ny.plane_wave_rhs(b0, om0, 2 * np.pi * np.arange(nrhs) / nrhs, 1)
    t1 = time.perf_counter()
    lu = sla.lu_factor(A0)
    sla.lu_solve(lu, F0)
    t_lu0 = time.perf_counter() - t1
    scale3 = (n / n0) ** 3
    T = t_pairs + (t_cubic_asm0 + t_lu0) * scale3
    used = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": nrhs / T,
        "unit": "solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"extrapolated: oracle pair work on {len(rows)} of {n} rows (x{n // len(rows)}), "
                   f"dense Maue assembly + LU + {nrhs} solves at n={n0} (x(n/{n0})^3); "
                   f"{used:.1f} s of CPU wall time, projected {T:.0f} s per {nrhs}-RHS solve"),
    }


def serve_stream(dp, nreq, rate, slots, seed=7):
    """Serving stream: Poisson arrivals of independent solve requests on the
    seeded random-star family, n = 2^k log-uniform in [2048, 65536], soft and
    hard 50/50, 1-16 plane waves each, 10 points per wavelength, eta = omega,
    preconditioned, tolerance 1e-8 (FP64 residual).  The same stream (same
    arrival times) is served by the mixed-precision and by the FP64 solver."""
    import threading
    from synth import omega_for_ppw, sample_boundary

    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, nreq))
    arrivals -= arrivals[0]
    geo = {}
    reqs = []
    t0 = time.perf_counter()
    for k in range(nreq):
        n = int(2 ** int(np.rint(rng.uniform(11, 16))))
        gs = int(rng.integers(0, 4))
        kind = int(rng.integers(0, 2))
        nrhs = int(rng.integers(1, 17))
        ang = rng.uniform(0, 2 * np.pi, nrhs)
        if (gs, n) not in geo:
            geo[(gs, n)] = sample_boundary(f"randstar{gs}", n)
        b = geo[(gs, n)]
        om = omega_for_ppw(n, b.L, 10.0)
        reqs.append((b, om, kind, ang))
    t_geo = time.perf_counter() - t0

    def run(precision):
        srv = dp.Server(slots=slots)
        # warm-up: one small request (kernel loading)
        b, om, kind, ang = reqs[0]
        srv.wait(srv.submit(b, om, om, kind, angles=ang, precision=precision))
        ids = [None] * nreq
        start = time.perf_counter()

        def submitter():
            for k, (b, om, kind, ang) in enumerate(reqs):
                d = start + arrivals[k] - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                ids[k] = srv.submit(b, om, om, kind, angles=ang, precision=precision)

        th = threading.Thread(target=submitter)
        th.start()
        res = []
        for k in range(nreq):
            while ids[k] is None:
                time.sleep(0.001)
            res.append(srv.wait(ids[k]))
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
            "solves_per_s": solves / (t_last - t_first),
            "requests_per_s": nreq / (t_last - t_first),
            "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3),
                           "max": float(lat.max() * 1e3)},
            "queue_wait_ms_mean": float(qw.mean() * 1e3),
            "makespan_s": t_last - t_first,
            "peak_concurrent": peak,
            "converged": all(r[3] == dp.DP_OK for r in res),
            "relres_max": float(max(r[1]["relres_max"] for r in res)),
            "mem_peak_gb": st["mem_peak"] / 1e9,
        }

    out = {"requests": nreq, "arrival_rate_per_s": rate, "slots": slots, "rhs_total": int(sum(r[3].size for r in reqs)),
           "n_range": [int(min(r[0].n for r in reqs)), int(max(r[0].n for r in reqs))],
           "hard_fraction": float(np.mean([r[2] for r in reqs])), "geometry_prep_s": t_geo}
    for name, prec in (("mixed", dp.DP_PREC_MIXED), ("fp64", dp.DP_PREC_FP64)):
        out[name] = run(prec)
        log(f"serve [{name}]: {json.dumps(out[name])}")
    return out


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
    ap.add_argument("--serve", type=int, default=32, metavar="N",
                    help="also serve a stream of N independent requests (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=2.5, help="mean arrivals per second")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default sweep launch configuration (2048-block grid)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of MIB MiB (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); "
              "a multi-GPU split of the sweep by target rows is not built", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1408_1578_amd as dp
    from synth import config_boundary, plane_wave_angles

    b, om, eta, kind = config_boundary("kite", args.n)
    nrhs = args.nrhs
    ctx = dp.Context(0)
    prob = dp.Problem.from_boundary(ctx, b, om, eta, kind)
    angles = plane_wave_angles(nrhs)
    f = torch.empty((nrhs, b.n), dtype=torch.complex128, device="cuda:0")
    q = torch.empty_like(f)
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

    def run(precision):
        prec = dp.DP_PREC_MIXED if precision == "mixed" else dp.DP_PREC_FP64

        def step():
            t0 = time.perf_counter()
            if use_pc:
                dp.dp_precond_build(prob)
            dp.dp_rhs_plane_wave(prob, angles, f)
            info = dp.dp_solve(prob, f, q, tol=1e-8, restart=80, use_precond=use_pc, precision=prec)
            return info, time.perf_counter() - t0

        for w in range(args.warmup):
            info, dt = step()
            log(f"[{precision}] warmup {w}: {dt:.3f} s iters={info['iters_max']} relres={info['relres_max']:.2e}")
        torch.cuda.synchronize()
        lat, infos = [], []
        t0 = time.perf_counter()
        for s in range(args.steps):
            info, dt = step()
            lat.append(dt)
            infos.append(info)
            log(f"[{precision}] step {s}: {dt:.3f} s iters={info['iters_max']} relres={info['relres_max']:.2e} "
                f"sweep {info['t_sweep'] / max(info['sweep_launches'], 1) * 1e3:.2f} ms x {info['sweep_launches']}"
                f" fp32 {info['t_sweep_fp32'] / max(info['sweep_launches_fp32'], 1) * 1e3:.2f} ms x "
                f"{info['sweep_launches_fp32']} refinements={info['refinements']}")
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        return T, lat, infos

    nrp = 1
    while nrp < nrhs and nrp < 64:
        nrp *= 2
    pairs = b.n * (b.n - 1)
    flops = pairs * (FLOPS_PAIR_HARD + FLOPS_PAIR_PER_RHS_HARD * nrp)

    # lower bound on one single-precision sweep: pair arithmetic on the vector
    # ALUs plus the executed split-FP16 products on the matrix cores
    t_bound32 = pairs * (FLOPS_PAIR_HARD / (PEAK_FP32_VALU * 1e12)
                         + 2 * nrp * FLOPS_MFMA16_PER_COL / (PEAK_FP16_MFMA * 1e12))

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
            "ms_per_step": T / args.steps * 1e3,
            "converged": all(i["converged"] and i["relres_max"] <= 1e-8 for i in infos),
            "iterations": int(max(i["iters_max"] for i in infos)),
            "relres_max": float(max(i["relres_max"] for i in infos)),
            "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
            "phase_s_per_step": {
                "matvec": float(np.mean([i["t_matvec"] for i in infos])),
                "precond_apply": float(np.mean([i["t_apply"] for i in infos])),
                "krylov": float(np.mean([i["t_krylov"] for i in infos])),
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

    # launch configuration of the sweep for this shape, chosen before the timed region
    # (--no-autotune keeps the default 2048-block grid, e.g. for counter runs
    # that must all see one configuration)
    tuned = {}
    for precision in (["mixed", "fp64"] if args.precision == "both" else [args.precision]):
        if args.no_autotune:
            tuned[precision] = {"target_blocks": 2048, "default": True}
            continue
        tuned[precision] = dp.dp_autotune(prob, nrhs, dp.DP_PREC_MIXED if precision == "mixed" else dp.DP_PREC_FP64)
        log(f"autotune [{precision}]: {tuned[precision]}")
    runs = {}
    for precision in (["mixed", "fp64"] if args.precision == "both" else [args.precision]):
        runs[precision] = summary(precision, *run(precision))
    head = "mixed" if "mixed" in runs else "fp64"
    main_run = runs[head]
    pinfo = dp.dp_precond_get_info(prob) if use_pc else {}

    def measured_cfg(precision):
        # the counters were taken at this shape with a 2048-block grid
        return b.n == 32768 and nrhs == 64 and tuned.get(precision, {}).get("target_blocks") == 2048

    if head == "mixed":
        sw = main_run["sweep_fp32"]
        roof = {"kernel": "sweep_mfma16<hard, 64 columns> (FP32 kernel values, FP64 phase reduction; "
                          "split-FP16 operands on v_mfma_f32_16x16x32_f16 with FP32 accumulation; 8 waves x "
                          "16 targets, LDS density tiles)",
                "bound": "alu+mfma", "achieved": sw["tflops"], "peak": flops / t_bound32 / 1e12,
                "unit": "TFLOP/s", "frac": sw["frac_of_bound"],
                "traffic": TRAFFIC_FP32_SWEEP if measured_cfg("mixed") else None, "launch_ms": sw["launch_ms"],
                "launches": sw["launches"], "flops_per_launch": flops, "t_bound_ms": t_bound32 * 1e3,
                "valu_peak_tflops": PEAK_FP32_VALU, "mfma_peak_tflops": PEAK_FP16_MFMA}
    else:
        sw = main_run["sweep_fp64"]
        roof = {"kernel": "sweep_mfma<hard, 64 columns, FP64> (v_mfma_f64_16x16x4 products; 8 waves, "
                          "shared kernel values, LDS density tiles)",
                "bound": "mfma", "achieved": sw["tflops"], "peak": PEAK_FP64_VALU, "unit": "TFLOP/s",
                "frac": sw["tflops"] / PEAK_FP64_VALU,
                "traffic": TRAFFIC_FP64_SWEEP if measured_cfg("fp64") else None, "launch_ms": sw["launch_ms"],
                "launches": sw["launches"], "flops_per_launch": flops}
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
                                                      "corrections" if head == "mixed" else "FP64"),
            "n": b.n, "nrhs": nrhs, "omega": om, "tol": 1e-8, "restart": 80,
            "precision": head, "precond": use_pc,
        },
        "converged": main_run["converged"],
        "iterations": main_run["iterations"],
        "relres_max": main_run["relres_max"],
        "latency_ms": main_run["latency_ms"],
        "roofline": roof,
        "precision_runs": runs,
        "autotune": tuned,
    }
    out["precond_setup_s"] = float(pinfo.get("t_setup", 0.0))
    if pinfo:
        out["precond"] = {k: pinfo[k] for k in ("m", "NW", "nnzW", "nnzLU", "levels")}
    if args.serve > 0:
        log(f"serving stream: {args.serve} requests ...")
        out["serving"] = serve_stream(dp, args.serve, args.serve_rate, args.serve_slots)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, bounded sample) ...")
        out["cpu_baseline"] = cpu_baseline(b, om, eta, nrhs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
