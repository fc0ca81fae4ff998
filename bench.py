"""ADASAP hot-path benchmark on one MI355X (gfx950).

Workload: the 2M-point, 11-dimensional RBF problem with 64 right-hand sides
(standardised y plus 63 pathwise right-hand sides f_s(X) + eps_s), lambda = 1e-2,
b = 16384, r = 128, matrix-core float16 kernel-block products with float32
accumulation (MIXED precision), synthetic seeded data.

A step is one ADASAP iteration (Alg. 2: block sampling, the kernel-block
gradient, the Nystrom sketch and factorisation, powering, the Woodbury direction
and the Nesterov update).  `value` is the step-I kernel-block throughput over the
whole step, pairs * (2d + 2k) flops / step time.  The line also reports the
time to relative residual 1e-3 (iterations timed on the device, residual checks
once per data pass off the clock), the roofline of the dominant kernel, and the
CPU float64 oracle timed on a bounded sample on the host.

With --workload batched it instead times the 256-problem batch (n_p log-uniform in
[2000, 65536], d_p in {4..16}, ell_p ~ U(0.2, 2), lambda = 1e-2, b = 1024, r = 64, FP32):
a step is one round, one ADASAP iteration of every problem with one persistent Step-I
launch; `value` is the batch's aggregate kernel-block GFLOP/s.

With --workload warm it times the learned warm start: 32 windows of one GP field (d = 9,
RBF ell = 0.1, point density of 1e8 points in the unit cube) are solved by the batched
solver, the network is trained on them, and a larger problem of the same field is solved
to relative residual 1e-3 from zero and from the learned start (kept only if its residual
after a one-pass probe beats the cold start's); `value` is the guarded time to residual.

With --workload step1 it times the solver's Step-I launch alone (adasap_block_gradient on the
2M-point, 64-column problem, K calls) and then copies a 1 GiB buffer once: the known-size
transfer against which rocprofv3's FETCH_SIZE / WRITE_SIZE counters are calibrated.

With --workload matern32_n1m (Matern-3/2, n = 1M, d = 11 with 5% clustered near-duplicates,
lambda = 1e-3, b = 8192, r = 100, FP32) or --workload rbf_n100m (RBF, n = 1e8, d = 9,
lambda = 1e-2, b = 32768, r = 128, FP32) it times K iterations of that single problem; the
first also runs to relative residual 1e-3 (checked once per pass), the second reports the
row-subsampled residual estimate (2^17 rows) after its K iterations.

With --workload batched_ttr it counts how many of the 256 batched problems one batched solve
brings to relative residual 1e-3 within 128 .. 2048 rounds, against a loop of single-problem
solves over every 8th problem; --workload c1 times the small float64 problem (n = 4096,
200 iterations) beside the oracle's full run and a direct solve; --workload tailavg runs the
tail-averaging study, --workload matern32_precision the FP32/FP64 convergence comparison of
the Matern problem and --workload bo the Thompson-sampling optimisation.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-ttr] [--no-cpu]
                       [--workload c3|batched|batched_ttr|warm|step1|matern32_n1m|rbf_n100m|
                                   matern32_precision|tailavg|bo|c1]
                       [--ws-lam L] [--ws-n N]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time to rel. residual 1e-3 (s) & kernel-block GFLOP/s, n=2M d=11, 1 GPU"
# published MI355X peaks used for the roofline fraction
PEAK_F16_MFMA_TFLOPS = 2500.0
# transcendental (v_exp_f32) issue rate: 256 CUs x 4 SIMDs x 8 lanes per clock x 2.4 GHz
PEAK_EXP_TPS = 256 * 4 * 8 * 2.4e9 / 1e12
# HBM bytes of one Step-I launch at the 2M-point, 64-column shape: rocprofv3 FETCH_SIZE and
# WRITE_SIZE of the launch (1.020e6 and 2.867e4 KiB), each scaled by the ratio of true to
# counted KiB of a 1 GiB copy in the same run (2.0 for FETCH_SIZE, which prices the 128-byte
# reads of gfx950 at 64 bytes, and 1.0 for WRITE_SIZE); profiles/mkw_kernel_rbf_n2m_d11_k64.md
STEP1_TRAFFIC_BYTES_N2M = 2.118e9
# the same for the Matern-3/2 Step-I launch at n = 1M, d = 11, b = 8192 (FETCH_SIZE 1.268e5 KiB
# on average over three launches, WRITE_SIZE 672 KiB); profiles/mkv_kernel_matern32_n1m_d11.md
MATERN_STEP1_TRAFFIC_BYTES_N1M = 2.603e8
# and for the persistent batched Step-I launch over the 256 uneven problems (FETCH_SIZE 5.000e5
# KiB over two rounds, WRITE_SIZE 1.138e4 KiB with 32-tile work items; 64-tile items write half
# that); profiles/mkq_kernel_batched_256_uneven.md
BATCHED_STEP1_TRAFFIC_BYTES = 1.036e9
# and for the 1e8-point RBF Step-I launch, d = 9, b = 32768 (FETCH_SIZE 2.894e7 KiB on average
# over two launches, WRITE_SIZE 2048 KiB); profiles/mkv_kernel_rbf_n1e8_d9.md
RBF_N100M_STEP1_TRAFFIC_BYTES = 5.926e10


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=2_000_000)
    ap.add_argument("--no-ttr", action="store_true", help="skip the time-to-residual run")
    ap.add_argument("--ttr-passes", type=int, default=40, help="data passes allowed for time-to-residual")
    ap.add_argument("--ttr-rows", default="mixed,fp32,mixed_refine",
                    help="time-to-residual runs: mixed (the headline), fp32, mixed_refine")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--calib-copy", action="store_true",
                    help="end the batched and single-column workloads with a 1 GiB device copy, the "
                         "copy of known size that scales the HBM byte counters")
    ap.add_argument("--cpu-rows", type=int, default=384, help="oracle block rows per host core")
    ap.add_argument("--workload", choices=["c3", "batched", "warm", "step1", "matern32_n1m", "rbf_n100m",
                                           "bo", "matern32_precision", "tailavg", "batched_ttr", "c1"],
                    default="c3")
    ap.add_argument("--bo-n0", type=int, default=250_000, help="initial points of the BO workload")
    ap.add_argument("--bo-steps", type=int, default=10)
    ap.add_argument("--bo-acq", type=int, default=1000, help="acquisitions per BO step")
    ap.add_argument("--bo-seeds", type=int, default=1, help="objective functions per lengthscale")
    ap.add_argument("--bo-passes", type=int, default=10, help="ADASAP data passes per solve")
    ap.add_argument("--bo-ells", default="2,3", help="lengthscales of the BO objectives")
    ap.add_argument("--precision", choices=["fp32", "fp64", "mixed"], default=None,
                    help="precision of the single-problem workloads (default: the workload's)")
    ap.add_argument("--check-rows", type=int, default=0,
                    help="residual checks of the single-problem workloads on this many sampled rows "
                         "(0: all rows)")
    ap.add_argument("--shape", choices=["rbf_n2m_k64", "rbf_n100m"], default="rbf_n2m_k64",
                    help="problem of the step1 workload")
    ap.add_argument("--ws-lam", type=float, default=1.0, help="noise variance of the warm workload")
    ap.add_argument("--ws-n", type=int, default=1 << 20, help="points of the warm-start target")
    ap.add_argument("--ws-budget", type=int, default=20,
                    help="iterations of the fixed warm-start budget above 2^22 points")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2505_13723_amd import binding, inputs

    if args.workload == "batched":
        return bench_batched(args, torch, binding, inputs)
    if args.workload == "warm":
        return bench_warm(args, torch, binding, inputs)
    if args.workload == "step1":
        return bench_step1(args, torch, binding, inputs)
    if args.workload in ("matern32_n1m", "rbf_n100m"):
        return bench_single_k1(args, torch, binding, inputs)
    if args.workload == "bo":
        return bench_bo(args, torch, binding)
    if args.workload == "matern32_precision":
        return bench_matern_precision(args, torch, binding, inputs)
    if args.workload == "tailavg":
        return bench_tailavg(args, torch, binding, inputs)
    if args.workload == "batched_ttr":
        return bench_batched_ttr(args, torch, binding, inputs)
    if args.workload == "c1":
        return bench_c1(args, torch, binding, inputs)
    cfgw = dict(inputs.WORKLOADS["c3_rbf_n2m_k64"])
    n, d, k = args.n, cfgw["d"], cfgw["k"]
    b, r, lam, ell = cfgw["b"], cfgw["r"], cfgw["lam"], cfgw["ell"]
    if n != 2_000_000:
        b = max(256, n // 122)
    lib = binding.load()
    log("generating inputs n=%d d=%d k=%d on the GPU" % (n, d, k))
    X, Y, Xt, yt, Pt = inputs.make_c3(seed=cfgw["seed"], n=n, d=d, k=k, ell=ell, lam=lam,
                                      device="cuda", n_test=N_TEST)
    test = (Xt, yt, Pt)
    torch.cuda.synchronize()

    def make(max_iters, tol=0.0, check_every=0, refine=0):
        c = lib.config(kernel="rbf", lengthscale=ell, lam=lam, block_size=b, rank=r,
                       max_iters=max_iters, tol=tol, check_every=check_every,
                       refine_sweeps=refine, seed=cfgw["seed"], precision="mixed")
        return lib.create(c, X, Y)

    # ---- throughput: warmup, then exactly `steps` timed iterations -------------------------
    h = make(args.warmup)
    W = torch.zeros_like(Y)
    if args.warmup > 0:
        h.solve(W)
    h.close()
    h = make(args.steps)
    W.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = h.solve(W)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    h.close()
    ms_per_step = rep["solve_ms"] / max(1, rep["iters"])
    pairs = float(b) * n
    flops_step1 = pairs * (2 * d + 2 * k)
    value = flops_step1 / (ms_per_step * 1e-3) / 1e9
    kern_ms = rep["step1_kernel_ms"] / max(1, rep["step1_launches"])
    achieved = flops_step1 / (kern_ms * 1e-3) / 1e12
    log("steps=%d solve_ms=%.1f (%.3f ms/step), wall %.3f s, step-I kernel %.3f ms, "
        "Jacobi sweeps <= %d" % (rep["iters"], rep["solve_ms"], ms_per_step, wall, kern_ms,
                                 rep["jacobi_sweeps_max"]))

    # ---- time to relative residual 1e-3 -------------------------------------------------------
    ttr, ttr_rows = None, {}
    if not args.no_ttr:
        per_pass = int(math.ceil(n / b))
        for row in args.ttr_rows.split(","):
            prec, refine = {"mixed": ("mixed", 0), "fp32": ("fp32", 0),
                            "mixed_refine": ("mixed", 1)}[row]
            ttr_rows[row] = time_to_residual(torch, lib, X, Y, W, cfgw, b, n, per_pass,
                                             args.ttr_passes, prec, refine, test)
            log("time-to-residual %s: %s" % (row, json.dumps(ttr_rows[row])))
        ttr = ttr_rows.get("mixed")

    # ---- CPU float64 oracle on a bounded sample ------------------------------------------------
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(X, Y, args.cpu_rows, ell, d, k, b, n)
        log("cpu baseline: %s" % json.dumps(cpu))

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": rep["iters"], "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16 matrix-core products, f32 accumulation, f64 Nystrom core",
        "data": "synthetic (seeded Gaussian X, RFF prior-draw right-hand sides)",
        "config": {"workload": "rbf_n%d_d%d_k%d" % (n, d, k), "n": n, "d": d, "k": k, "b": b,
                   "r": r, "lambda": lam, "lengthscale": ell, "kernel": "rbf",
                   "precision": "mixed"},
        "time_to_relres_1e-3": ttr,
        "time_to_relres_1e-3_rows": ttr_rows,
        "warm_start_row": "not run at this workload: its 64 columns are independent prior draws "
                          "at lambda = 1e-2, where the residual guard keeps the cold start "
                          "(bench.py --workload warm measures both regimes)",
        "roofline": {"bound": "mfma", "achieved": round(achieved, 1),
                     "peak": PEAK_F16_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_F16_MFMA_TFLOPS, 4),
                     "traffic": STEP1_TRAFFIC_BYTES_N2M if n == 2_000_000 else None,
                     "kernel": "mkw_kernel (Step-I kernel-block product, float16 32x32x16 MFMA)",
                     "kernel_ms": round(kern_ms, 4),
                     "algorithmic_flops_per_launch": flops_step1},
        # the same launch against the instruction rates of this part, measured in the same
        # run (adasap_probe_rates): the 32x32x16 float16 MFMA on the flops per pair the kernel
        # executes (48 distance slots for the 3d + 6 = 39 of the hi/lo split, and K Z), one
        # v_exp_f32 and half a conversion per pair on the vector ALUs
        "roofline_probe": probe_bound(lib.probe_rates(), b, n, d, k, kern_ms),
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def probe_bound(rates, b, n, d, k, kern_ms, simds=1024):
    """T_bound = max(MFMA time, vector time) of the MIXED Step-I launch at the measured rates."""
    pairs = float(b) * n
    slots = 16 * math.ceil((3 * d + 6) / 16)
    mfma_ms = pairs * 2 * (slots + k) / (rates["mfma32_f16_tflops"] * 1e12) * 1e3
    valu_ms = pairs / 64 * (rates["exp_ns"] + 0.5 * rates["valu_ns"]) / simds * 1e-6
    bound = max(mfma_ms, valu_ms)
    return {"t_bound_ms": round(bound, 4), "mfma_ms": round(mfma_ms, 4), "valu_ms": round(valu_ms, 4),
            "measured_ms": round(kern_ms, 4), "frac": round(bound / kern_ms, 4) if kern_ms > 0 else None,
            "rates": {key: round(v, 4) for key, v in rates.items()},
            "basis": "rates of this part from adasap_probe_rates in the same run; under the Step-I "
                     "load the part runs power-limited at 1.8-1.9 GHz (GRBM_GUI_ACTIVE)"}


CERT_ROWS = 1 << 17
N_TEST = 16384


def time_to_residual(torch, lib, X, Y, W, cfgw, b, n, per_pass, passes, precision, refine, test=None):
    """Solve from zero until the relative residual is certified <= 1e-3 in float64.

    The solve checks once per data pass with the row-subsampled estimate (2^17 rows, the
    handle's own products) and stops at the first estimate <= 1e-3 (with one refinement sweep:
    each sweep stops at 10^-1.5, so the two together reach 1e-3).  The stop point is then
    certified with float64 kernel values on 2^17 rows (adasap_residual_rows_f64, with its
    standard error) and by the full hi/lo residual over all n rows; while the float64 estimate
    is above 1e-3 the same run is continued one pass at a time (adasap_solve_more).  `seconds`
    is the device time of the iterations; `wall_seconds` adds every check and certificate."""
    tol = 1e-3 if refine == 0 else 10 ** -1.5
    c = lib.config(kernel="rbf", lengthscale=cfgw["ell"], lam=cfgw["lam"], block_size=b,
                   rank=cfgw["r"], max_iters=per_pass * passes, tol=tol, check_every=per_pass,
                   check_rows=CERT_ROWS, refine_sweeps=refine, seed=cfgw["seed"],
                   precision=precision)
    h = lib.create(c, X, Y)
    W.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = h.solve(W)
    solve_s, iters = rep["solve_ms"] / 1e3, rep["iters"]
    est, worst, se = h.residual_rows_f64(W, CERT_ROWS, 12)
    extra = 0
    while est > 1e-3 and refine == 0 and extra < 10 and rep["iters"] > 0:
        rep = h.solve_more(W, per_pass)
        solve_s += rep["solve_ms"] / 1e3
        iters += rep["iters"]
        extra += 1
        est, worst, se = h.residual_rows_f64(W, CERT_ROWS, 12)
    full, full_max = h.residual(W)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pred = None
    if test is not None:
        # pathwise posterior samples at the held-out points (column 0 of W solves for y, the
        # others for prior functions plus noise) and the test RMSE / mean NLL (Sec. 5.1)
        Xt, yt, Pt = test
        t1 = time.perf_counter()
        smp = h.posterior_samples(W, Xt, Pt)
        rmse, nll = lib.predictive_metrics(smp, yt, cfgw["lam"])
        pred = {"test_points": int(Xt.shape[0]), "samples": int(Y.shape[1] - 1),
                "test_rmse": rmse, "test_mean_nll": nll,
                "seconds": round(time.perf_counter() - t1, 4)}
    h.close()
    ok = est <= 1e-3
    return {"seconds": round(solve_s, 3) if ok else None, "reached": bool(ok),
            "wall_seconds": round(wall, 3), "iterations": iters, "passes": round(iters / per_pass, 3),
            "precision": precision, "refine_sweeps": refine,
            "relres_f64_rows": est, "relres_f64_rows_rel_se": se, "relres_f64_rows_maxcol": worst,
            "certificate_rows": CERT_ROWS, "relres_hilo_full": full, "relres_hilo_full_maxcol": full_max,
            "passes_added_after_certificate": extra, "check_every_iters": per_pass,
            "check": "row estimate on %d rows once per pass" % CERT_ROWS, "predictive": pred}


def bench_batched(args, torch, binding, inputs):
    """256 independent uneven problems, one round = one iteration of each."""
    import numpy as np

    w = inputs.WORKLOADS["c4_batched_256"]
    ns, ds, ells = inputs.c4_problem_sizes(seed=w["seed"], count=w["count"], nmin=w["nmin"],
                                           nmax=w["nmax"], dmin=w["dmin"], dmax=w["dmax"],
                                           ellmin=w["ellmin"], ellmax=w["ellmax"])
    b, r, lam = w["b"], w["r"], w["lam"]
    lib = binding.load()
    log("generating %d problems, %d rows in total" % (len(ns), int(ns.sum())))
    Xs, Ys, Ws, host = [], [], [], []
    for p in range(len(ns)):
        X, y = inputs.make_c4_problem(p, int(ns[p]), int(ds[p]), seed=w["seed"])
        if p < 32:
            host.append((X, y))
        Xs.append(torch.as_tensor(X, dtype=torch.float32).cuda())
        Ys.append(torch.as_tensor(y[:, None], dtype=torch.float32).cuda())
        Ws.append(torch.zeros((int(ns[p]), 1), dtype=torch.float32, device="cuda"))

    def run(iters):
        cfg = lib.config(kernel="rbf", lam=lam, block_size=b, rank=r, max_iters=iters,
                         seed=w["seed"], precision="fp32")
        for W in Ws:
            W.zero_()
        torch.cuda.synchronize()
        return lib.solve_batch(cfg, Xs, Ys, Ws, ells)

    if args.warmup > 0:
        run(args.warmup)
    t0 = time.perf_counter()
    reps = run(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rep = reps[0]
    ms_per_step = rep["solve_ms"] / max(1, rep["iters"])
    pairs = float(b) * float(ns.sum())
    flops = float(b) * float(np.sum(ns * (2 * ds + 2)))
    value = flops / (ms_per_step * 1e-3) / 1e9
    kern_ms = rep["step1_kernel_ms"] / max(1, rep["step1_launches"])
    achieved = pairs / (kern_ms * 1e-3) / 1e12
    tuned = {"rows_per_workgroup": rep["tuned_rows_per_wg"], "workgroups_per_cu": rep["tuned_wg_per_cu"],
             "column_tiles_per_item": rep["reserved"], "from_cache": bool(rep["tuned_from_cache"])}
    log("rounds=%d solve_ms=%.2f (%.3f ms/round), wall %.3f s, step-I kernel %.3f ms, autotuner %s"
        % (rep["iters"], rep["solve_ms"], ms_per_step, wall, kern_ms, tuned))
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline_batched(host, ds, ells, b)
        log("cpu baseline: %s" % json.dumps(cpu))
    line = {
        "metric": "batched kernel-block GFLOP/s, 256 uneven problems, 1 GPU", "value": round(value, 1),
        "unit": "GFLOP/s", "n_gpus": 1, "steps": rep["iters"], "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (f16 hi/lo matrix-core distances), f64 Nystrom cores",
        "data": "synthetic (seeded Gaussian X, sum-of-sines targets)",
        "config": {"workload": "batched_256_rbf_uneven", "problems": len(ns), "rows": int(ns.sum()),
                   "b": b, "r": r, "lambda": lam, "kernel": "rbf", "precision": "fp32"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_EXP_TPS,
                     "unit": "Texp/s", "frac": round(achieved / PEAK_EXP_TPS, 4),
                     "traffic": BATCHED_STEP1_TRAFFIC_BYTES,
                     "kernel": "mkq_kernel (persistent batched Step-I product)",
                     "kernel_ms": round(kern_ms, 4), "algorithmic_exp_per_launch": pairs},
        "autotuner": tuned,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    if args.calib_copy:
        calibration_copy(torch)


def bench_matern_precision(args, torch, binding, inputs):
    """The ill-conditioned Matern-3/2 problem (n = 1M with near-duplicates, lambda = 1e-3) solved
    with the same seed at FP32 (float16 hi/lo distances on the matrix cores) and at FP64 (float64
    distances and products), in chunks of 10 data passes continued on the same run; after each
    chunk the float64 row certificate (2^14 rows).  If FP64 goes below the FP32 run's level,
    the float16 distances set the floor; if both track each other, convergence is slow."""
    w = inputs.WORKLOADS["c2_matern32_n1m"]
    lib = binding.load()
    n, d, b, r, lam, ell = w["n"], w["d"], w["b"], w["r"], w["lam"], w["ell"]
    X, y = inputs.make_c2(seed=w["seed"], n=n, d=d, ell=ell, lam=lam, device="cuda")
    Y = y[:, None].contiguous()
    per_pass = int(math.ceil(n / b))
    chunk = 10 * per_pass
    out = {}
    for prec in ("fp32", "fp64"):
        Xp, Yp = (X.double(), Y.double()) if prec == "fp64" else (X, Y)
        h = lib.create(lib.config(kernel="matern32", lengthscale=ell, lam=lam, block_size=b, rank=r,
                                  max_iters=chunk, seed=w["seed"], precision=prec), Xp, Yp)
        W = torch.zeros_like(Yp)
        curve, secs = [], 0.0
        for c in range(args.ttr_passes // 10):
            rep = h.solve(W) if c == 0 else h.solve_more(W, chunk)
            secs += rep["solve_ms"] / 1e3
            est, _, se = h.residual_rows_f64(W, 1 << 14, 12)
            curve.append({"passes": 10 * (c + 1), "relres_f64_rows": est, "rel_se": se,
                          "solve_seconds": round(secs, 2)})
            log("%s after %d passes: relres %.4e (s.e. %.1f%%), %.1f s" % (prec, 10 * (c + 1), est,
                                                                          100 * se, secs))
        h.close()
        out[prec] = curve
    line = {"metric": "relative residual vs data passes, FP32 and FP64, Matern-3/2 n=1M, 1 GPU",
            "value": out["fp64"][-1]["relres_f64_rows"], "unit": "relres", "n_gpus": 1,
            "steps": args.ttr_passes * per_pass, "warmup": 0, "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32 (f16 hi/lo distances) and f64",
            "data": "synthetic (uniform points with 5% near-duplicates, Matern-3/2 prior target)",
            "config": {"workload": "matern32_n1m_d11_precision", "n": n, "d": d, "b": b, "r": r,
                       "lambda": lam, "lengthscale": ell},
            "curves": out, "roofline": None, "cpu_baseline": None}
    print(json.dumps(line), flush=True)


def bench_tailavg(args, torch, binding, inputs):
    """Tail averaging with and without (appendix, impact of tail averaging): n = 1000 RBF, the
    relative error of the posterior mean on the top-l spectral subspace, l in {10, 100, 1000},
    ||P_l(m_hat) - P_l(m_n)||_H^2 / ||P_l(m_n)||_H^2, after 1 .. 50 data passes, for three
    block sizes; FP64 solves through the library (tail_average flag), the subspace errors from
    the eigendecomposition of K on the host."""
    lib = binding.load()
    n, d, ell, lam, seed = 1000, 3, 1.0, 1e-2, 21
    X, Y = inputs.make_small(seed, n, d, 1)
    Xd = torch.as_tensor(X, dtype=torch.float64).cuda()
    Yd = torch.as_tensor(Y, dtype=torch.float64).cuda()
    # the exact solution and the spectral basis of K (float64 kernel values on the device, as
    # products with blocks of the identity)
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    Kh = torch.cat([lib.kblock_matmul("rbf", ell, "fp64", Xd, Xd, eye[:, j:j + 100].contiguous())
                    for j in range(0, n, 100)], dim=1).cpu().numpy()
    Kh = 0.5 * (Kh + Kh.T)
    ev, U = np.linalg.eigh(Kh)
    ev, U = ev[::-1], U[:, ::-1]
    Wstar = np.linalg.solve(Kh + lam * np.eye(n), Y)

    def sub_err(W, l):
        a = U[:, :l].T @ (W - Wstar)[:, 0]
        c = U[:, :l].T @ Wstar[:, 0]
        return float(np.sum(ev[:l] * a * a) / np.sum(ev[:l] * c * c))

    passes = [1, 2, 5, 10, 20, 50]
    res = {}
    for b in (25, 100, 400):
        per_pass = n // b
        for tail in (0, 1):
            curve = []
            for P in passes:
                h = lib.create(lib.config(kernel="rbf", lengthscale=ell, lam=lam, block_size=b,
                                          rank=min(b, 50), max_iters=P * per_pass, seed=seed,
                                          precision="fp64", tail_average=tail), Xd, Yd)
                W = torch.zeros_like(Yd)
                h.solve(W)
                h.close()
                Wh = W.cpu().numpy()
                curve.append({"passes": P, **{"err_top%d" % l: sub_err(Wh, l) for l in (10, 100, 1000)}})
            res["b%d_%s" % (b, "tail" if tail else "last")] = curve
            log("b=%d tail=%d: %s" % (b, tail, curve[-1]))
    summary = {}
    for b in (25, 100, 400):
        for l in (10, 100, 1000):
            last = res["b%d_last" % b][-1]["err_top%d" % l]
            tail = res["b%d_tail" % b][-1]["err_top%d" % l]
            summary["b%d_top%d" % (b, l)] = {"last_iterate": last, "tail_average": tail,
                                             "tail_over_last": tail / last if last > 0 else None}
    line = {"metric": "top-l subspace error after 50 passes, tail averaging vs last iterate, 1 GPU",
            "value": None, "unit": "relative error", "n_gpus": 1, "steps": 50, "warmup": 0,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic (n = 1000, d = 3, sum-of-sines target)",
            "config": {"workload": "tail_average_rbf_n1000", "n": n, "d": d, "lengthscale": ell,
                       "lambda": lam, "blocks": [25, 100, 400]},
            "summary": summary, "curves": res, "roofline": None, "cpu_baseline": None}
    print(json.dumps(line), flush=True)


def bench_c1(args, torch, binding, inputs):
    """The small float64 workload (n = 4096, d = 8, RBF ell = 1, lambda = rho = 1e-2, b = 256,
    r = 64, 200 iterations, one right-hand side): the library's FP64 solve timed on the device,
    beside the oracle's full 200-iteration run and a direct Cholesky solve on the host cores,
    with the relative residual of each and the GPU-oracle difference
    ||(K + lambda I)(W_gpu - W_oracle)|| / ||y||."""
    lib = binding.load()
    cfg = inputs.WORKLOADS["c1_fp64_n4096"]
    X, y = inputs.make_c1(seed=cfg["seed"])
    T = cfg["iters"]
    Xd = torch.as_tensor(X).cuda()
    Yd = torch.as_tensor(y[:, None]).contiguous().cuda()
    c = lib.config(kernel="rbf", lengthscale=cfg["ell"], lam=cfg["lam"], block_size=cfg["b"],
                   rank=cfg["r"], rho_rule=1, rho=cfg["rho"], max_iters=T, seed=cfg["seed"],
                   precision="fp64")
    times = []
    for rep in range(1 + max(1, args.steps // 10)):
        h = lib.create(c, Xd, Yd)
        W = torch.zeros_like(Yd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.solve(W)
        torch.cuda.synchronize()
        if rep > 0:
            times.append(time.perf_counter() - t0)
        relres_gpu = h.residual(W)[0]
        h.close()
    t_gpu = min(times)
    log("GPU FP64: %d iterations in %.4f s, relres %.4e" % (T, t_gpu, relres_gpu))
    base = None
    if not args.no_cpu:
        base = cpu_baseline_c1(X, y, cfg, W.cpu().numpy()[:, 0])
        log("oracle: %s" % base)
    line = {"metric": "FP64 solve time, %d iterations, n=4096 d=8, 1 GPU" % T, "value": t_gpu,
            "unit": "s", "n_gpus": 1, "steps": T, "warmup": 1, "ms_per_step": 1e3 * t_gpu / T,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic (X ~ N(0, I_8), y = sum_j sin(x_j) + N(0, 0.1^2))",
            "config": {"workload": "c1_fp64_rbf_n4096_d8", "n": cfg["n"], "d": cfg["d"], "b": cfg["b"],
                       "r": cfg["r"], "lambda": cfg["lam"], "rho": cfg["rho"], "iters": T},
            "relres_gpu": relres_gpu, "roofline": None, "cpu_baseline": base}
    print(json.dumps(line), flush=True)


def cpu_baseline_c1(X, y, cfg, Wg):
    """The oracle's full run and the direct solve of the small float64 workload, on the host
    cores (BLAS threads), with the relative residuals and the GPU-oracle difference."""
    from threadpoolctl import threadpool_limits

    from oracle import adasap as OA
    from oracle import kernels as OK
    from oracle import linsys as OL

    cores, nproc, ncpu, model = host_cores()
    with threadpool_limits(limits=cores):
        t0 = time.perf_counter()
        Wo, _ = OA.adasap(X, y, OK.RBF, cfg["ell"], cfg["lam"], cfg["b"], cfg["r"], cfg["iters"],
                          cfg["seed"], rho_rule=1, rho=cfg["rho"])
        t_or = time.perf_counter() - t0
        t0 = time.perf_counter()
        Wd = OL.direct_solve(X, y[:, None], OK.RBF, cfg["ell"], cfg["lam"])
        t_dir = time.perf_counter() - t0
        Y = y[:, None]
        Wo = Wo.reshape(-1, 1)
        delta = float(np.linalg.norm(OL.residual(X, np.zeros_like(Y), Wg[:, None] - Wo, OK.RBF,
                                                 cfg["ell"], cfg["lam"])) / np.linalg.norm(Y))
        rr_or = float(OL.relres(X, Y, Wo, OK.RBF, cfg["ell"], cfg["lam"])[0])
        rr_dir = float(OL.relres(X, Y, Wd, OK.RBF, cfg["ell"], cfg["lam"])[0])
    return {"value": t_or, "unit": "s", "cores": cores, "nproc": nproc, "logical_cpus": ncpu,
            "cpu_model": model, "kind": "oracle",
            "sample": "the whole workload: %d iterations" % cfg["iters"],
            "relres_oracle": rr_or, "direct_solve_s": t_dir, "relres_direct": rr_dir,
            "delta_gpu_vs_oracle": delta}


def bench_batched_ttr(args, torch, binding, inputs):
    """The 256 uneven problems against relative residual 1e-3: how many problems one batched
    solve brings to 1e-3 within T rounds (T = 128 .. 2048, each from zero), against a loop of
    single-problem solves (every 8th problem in size order, 32 problems) that each stop at
    their first per-pass check <= 1e-3 or after the same round cap.  The slowest problems
    (low dimension, long lengthscales) converge slowly at any precision, so the comparison is
    the number reached per second of device time, not the time until the last one."""
    w = inputs.WORKLOADS["c4_batched_256"]
    ns, ds, ells = inputs.c4_problem_sizes(seed=w["seed"], count=w["count"], nmin=w["nmin"],
                                           nmax=w["nmax"], dmin=w["dmin"], dmax=w["dmax"],
                                           ellmin=w["ellmin"], ellmax=w["ellmax"])
    b, r, lam = w["b"], w["r"], w["lam"]
    P = len(ns)
    lib = binding.load()
    Xs, Ys, Ws = [], [], []
    for p in range(P):
        X, y = inputs.make_c4_problem(p, int(ns[p]), int(ds[p]), seed=w["seed"])
        Xs.append(torch.as_tensor(X, dtype=torch.float32).cuda())
        Ys.append(torch.as_tensor(y[:, None], dtype=torch.float32).cuda())
        Ws.append(torch.zeros((int(ns[p]), 1), dtype=torch.float32, device="cuda"))
    checkpoints = [128, 256, 512, 1024, 2048]
    batched = []
    for T in checkpoints:
        cfg = lib.config(kernel="rbf", lam=lam, block_size=b, rank=r, max_iters=T, seed=w["seed"],
                         precision="fp32", tol=1e-3)
        for Wt in Ws:
            Wt.zero_()
        torch.cuda.synchronize()
        reps = lib.solve_batch(cfg, Xs, Ys, Ws, ells)
        rr = np.array([rp["relres"] for rp in reps])
        row = {"rounds": T, "seconds": round(reps[0]["solve_ms"] / 1e3, 3),
               "reached": int(np.sum(rr <= 1e-3)),
               "relres_quantiles_50_90_max": [float(x) for x in np.quantile(rr, [0.5, 0.9, 1.0])]}
        batched.append(row)
        log("batched T=%d: %s" % (T, row))
    cap = 1024
    sample = [int(p) for p in np.argsort(ns)[::8]]
    loop_s, loop_it, loop_reached = 0.0, 0, 0
    for i, p in enumerate(sample):
        per_pass = int(math.ceil(ns[p] / b))
        h = lib.create(lib.config(kernel="rbf", lengthscale=float(ells[p]), lam=lam, block_size=b,
                                  rank=r, max_iters=cap, tol=1e-3, check_every=per_pass,
                                  seed=w["seed"] + p, precision="fp32"), Xs[p], Ys[p])
        Wt = torch.zeros_like(Ys[p])
        rp = h.solve(Wt)
        h.close()
        loop_s += rp["solve_ms"] / 1e3
        loop_it += rp["iters"]
        loop_reached += int(0 <= rp["relres"] <= 1e-3)
        if i % 8 == 7:
            log("loop: %d of %d problems, %.2f s, %d reached" % (i + 1, len(sample), loop_s, loop_reached))
    at_cap = next(row for row in batched if row["rounds"] == cap)
    line = {"metric": "uneven problems reaching relres 1e-3 per second, batched vs loop, 1 GPU",
            "value": round(at_cap["reached"] / at_cap["seconds"], 2), "unit": "problems/s",
            "n_gpus": 1, "steps": cap, "warmup": 0, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32 (f16 hi/lo matrix-core distances), f64 Nystrom cores",
            "data": "synthetic (seeded Gaussian X, sum-of-sines targets)",
            "config": {"workload": "batched_256_rbf_uneven_ttr", "problems": P, "b": b, "r": r,
                       "lambda": lam, "round_cap": cap},
            "batched": batched,
            "single_loop": {"problems": len(sample), "sample": "every 8th problem in size order",
                            "seconds": round(loop_s, 3), "iterations": loop_it,
                            "reached": loop_reached, "round_cap": cap,
                            "checked_every": "one data pass (off the clock)",
                            "problems_per_second": round(loop_reached / loop_s, 2) if loop_s > 0 else None,
                            "seconds_for_all_256_extrapolated": round(loop_s * P / len(sample), 1)},
            "roofline": None, "cpu_baseline": None}
    print(json.dumps(line), flush=True)


def bench_bo(args, torch, binding):
    """Parallel Thompson sampling on Matern-3/2 objectives over [0, 1]^8 (lengthscales 2 and 3,
    noise 1e-6, b = n/5), against random search with as many evaluations."""
    from paper_2505_13723_amd import bo

    lib = binding.load()
    res = {}
    t0 = time.perf_counter()
    for ell in [float(v) for v in args.bo_ells.split(",")]:
        runs = []
        for sd in range(args.bo_seeds):
            out = bo.thompson_bo(lib, d=8, ell=ell, noise=1e-6, n0=args.bo_n0, steps=args.bo_steps,
                                 acq=args.bo_acq, passes=args.bo_passes, seed=100 * sd + int(ell),
                                 log=log)
            log("BO ell=%.1f seed %d: improvement %.3f%%" % (ell, sd, out["improvement_percent"]))
            runs.append(out)
        res["ell_%.1f" % ell] = {
            "improvement_percent_mean": float(np.mean([r["improvement_percent"] for r in runs])),
            "runs": [{k: v for k, v in r.items()} for r in runs]}
    wall = time.perf_counter() - t0
    line = {"metric": "BO improvement over random search (%), Matern-3/2 on [0,1]^8, 1 GPU",
            "value": round(float(np.mean([v["improvement_percent_mean"] for v in res.values()])), 4),
            "unit": "%", "n_gpus": 1, "steps": args.bo_steps, "warmup": 0, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f16 matrix-core products (MIXED)",
            "data": "synthetic (random-feature Matern-3/2 objectives)",
            "config": {"workload": "bo_matern32_d8_n%d" % args.bo_n0, "n0": args.bo_n0,
                       "acquisitions_per_step": args.bo_acq, "steps": args.bo_steps,
                       "objectives_per_lengthscale": args.bo_seeds, "passes_per_solve": args.bo_passes,
                       "b": "n/5", "noise": 1e-6},
            "results": res, "wall_seconds": round(wall, 2), "roofline": None, "cpu_baseline": None}
    print(json.dumps(line), flush=True)


def bench_single_k1(args, torch, binding, inputs):
    """One right-hand side, FP32: the ill-conditioned Matern-3/2 problem or the 1e8-point one."""
    big = args.workload == "rbf_n100m"
    w = inputs.WORKLOADS["c5_rbf_n100m" if big else "c2_matern32_n1m"]
    lib = binding.load()
    n, d, b, r, lam, ell = w["n"], w["d"], w["b"], w["r"], w["lam"], w["ell"]
    log("generating inputs n=%d d=%d on the GPU" % (n, d))
    if big:
        X, y = inputs.make_c5(seed=w["seed"], n=n, d=d, ell=ell, lam=lam, device="cuda", chunk=1 << 18)
    else:
        X, y = inputs.make_c2(seed=w["seed"], n=n, d=d, ell=ell, lam=lam, device="cuda")
    Y = y[:, None].contiguous()
    del y
    torch.cuda.synchronize()

    prec = args.precision or w["precision"]
    if prec == "fp64":
        X, Y = X.double(), Y.double()

    def make(iters, tol=0.0, check_every=0):
        c = lib.config(kernel=w["kernel"], lengthscale=ell, lam=lam, block_size=b, rank=r,
                       max_iters=iters, tol=tol, check_every=check_every, seed=w["seed"],
                       precision=prec, check_rows=args.check_rows)
        return lib.create(c, X, Y)

    W = torch.zeros_like(Y)
    if args.warmup > 0:
        h = make(args.warmup)
        h.solve(W)
        h.close()
    h = make(args.steps)
    W.zero_()
    torch.cuda.synchronize()
    rep = h.solve(W)
    ms_per_step = rep["solve_ms"] / max(1, rep["iters"])
    kern_ms = rep["step1_kernel_ms"] / max(1, rep["step1_launches"])
    pairs = float(b) * n
    trans = 1 if w["kernel"] == "rbf" else 2  # exp2, or sqrt and exp2 (Matern)
    # the float64 path has no matrix-core Step-I launch to time (kern_ms = 0)
    achieved = pairs * trans / (kern_ms * 1e-3) / 1e12 if kern_ms > 0 else 0.0
    value = pairs * (2 * d + 2) / (ms_per_step * 1e-3) / 1e9
    extra = {}
    if big:
        m = 1 << 17
        t0 = time.perf_counter()
        est, worst = h.residual_rows(W, m, 12)
        extra["relres_subsampled"] = {"rows": m, "estimate": est, "after_iterations": rep["iters"],
                                      "seconds": round(time.perf_counter() - t0, 3)}
    h.close()
    log("steps=%d solve_ms=%.1f (%.3f ms/step), step-I kernel %.3f ms" % (rep["iters"], rep["solve_ms"],
                                                                       ms_per_step, kern_ms))
    if not big and not args.no_ttr:
        per_pass = int(math.ceil(n / b))
        h = make(per_pass * args.ttr_passes, tol=1e-3, check_every=per_pass)
        W.zero_()
        rep2 = h.solve(W)
        h.close()
        reached = 0 <= rep2["relres"] <= 1e-3
        extra["time_to_relres_1e-3"] = {"seconds": rep2["solve_ms"] / 1e3 if reached else None,
                                        "reached": bool(reached), "iterations": rep2["iters"],
                                        "passes": rep2["iters"] / per_pass, "relres": rep2["relres"],
                                        "check_seconds_off_clock": rep2["check_ms"] / 1e3,
                                        "check_rows": args.check_rows or n}
        log("time-to-residual: %s" % json.dumps(extra["time_to_relres_1e-3"]))
    line = {
        "metric": "kernel-block GFLOP/s (Step-I flops per whole iteration), %s, 1 GPU" % args.workload,
        "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1, "steps": rep["iters"],
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (f16 hi/lo matrix-core distances, f32 vector K.Z), f64 Nystrom core",
        "data": "synthetic (seeded, GP prior-draw targets)",
        "config": {"workload": "%s_n%d_d%d" % (w["kernel"], n, d), "n": n, "d": d, "b": b, "r": r,
                   "lambda": lam, "lengthscale": ell, "kernel": w["kernel"], "precision": prec},
        "roofline": None if kern_ms <= 0 else {
            "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_EXP_TPS,
            "unit": "Ttranscendental/s", "frac": round(achieved / PEAK_EXP_TPS, 4),
            "traffic": None if prec != "fp32" else (RBF_N100M_STEP1_TRAFFIC_BYTES if big
                                                     else MATERN_STEP1_TRAFFIC_BYTES_N1M),
            "kernel": "mkv_kernel (Step-I product, float32 vector mode, 32x32x16 distances)",
            "kernel_ms": round(kern_ms, 4)},
        "cpu_baseline": None,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)
    if args.calib_copy:
        calibration_copy(torch)


def calibration_copy(torch):
    """A 1 GiB float32 device copy (torch.clone), the dispatch of known size that the
    FETCH_SIZE and WRITE_SIZE counters of the same run are scaled by."""
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    a.clone()
    torch.cuda.synchronize()
    del a


def bench_step1(args, torch, binding, inputs):
    """The Step-I product alone (the solver's launch), then a 1 GiB copy for calibration."""
    lib = binding.load()
    if args.shape == "rbf_n100m":
        w = dict(inputs.WORKLOADS["c5_rbf_n100m"], k=1)
        X, y = inputs.make_c5(seed=w["seed"], n=w["n"], d=w["d"], ell=w["ell"], lam=w["lam"],
                              device="cuda", chunk=1 << 18)
        Y = y[:, None].contiguous()
        prec = "fp32"
    else:
        w = inputs.WORKLOADS["c3_rbf_n2m_k64"]
        X, Y = inputs.make_c3(seed=w["seed"], n=w["n"], d=w["d"], k=w["k"], ell=w["ell"],
                              lam=w["lam"], device="cuda")
        prec = "mixed"
    h = lib.create(lib.config(kernel="rbf", lengthscale=w["ell"], lam=w["lam"], block_size=w["b"],
                              rank=w["r"], seed=w["seed"], precision=prec, max_iters=1), X, Y)
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    Z = torch.randn(Y.shape, generator=g, device="cuda", dtype=torch.float32)
    for t in range(args.warmup):
        h.block_gradient(t, Z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(args.steps):
        h.block_gradient(t, Z)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / max(1, args.steps) * 1e3
    h.close()
    calibration_copy(torch)
    flops = float(w["b"]) * w["n"] * (2 * w["d"] + 2 * w["k"])
    print(json.dumps({"metric": "Step-I launch (block gradient) wall time",
                      "value": round(ms, 4), "unit": "ms", "steps": args.steps, "warmup": args.warmup,
                      "higher_is_better": False, "gflops_per_s": round(flops / ms / 1e6, 1),
                      "config": {"workload": "rbf_n%d_d%d_k%d_step1" % (w["n"], w["d"], w["k"]),
                                 "b": w["b"]},
                      "calibration_copy_bytes": 1 << 30}), flush=True)


def bench_warm(args, torch, binding, inputs):
    """Cold vs learned warm start on a problem drawn from the training windows' field.

    Three starts of the target problem: W_0 = 0 (cold), the random-feature ridge mean alone,
    W_0 = (y - m_rff) / lambda (the network's last input; computed up to 2^24 points), and the
    network's m^, W_0 = (y - m^) / lambda.  Each is reported by its relative residual at W_0
    and after the same fixed budget of iterations (two passes up to 2^22 points, otherwise
    --ws-budget iterations, with the residual estimated on 2^17 rows).  Up to 2^22 points the
    line also times the solve to relres 1e-3 from the cold start and from the guarded warm
    start (kept only if its residual after a one-pass probe beats the cold start's)."""
    import numpy as np

    w = inputs.WORKLOADS["ws_rbf_d9"]
    d, ell, lam, D, H = w["d"], w["ell"], args.ws_lam, w["D"], w["H"]
    n = args.ws_n
    large = n > (1 << 22)
    b = 32768 if large else max(1024, n // 64)
    lib = binding.load()
    field = inputs.ws_field(w["seed"], d, ell, w["field_features"])
    outer = inputs.box_side(n, w["density"], d)
    side = inputs.box_side(w["n_window"], w["density"], d)
    corners = inputs.ws_window_corners(w["seed"] + 1, w["windows"], d, outer, side)
    Xs, ys, Ws = [], [], []
    for p in range(w["windows"]):
        X, y = inputs.ws_points(field, w["n_window"], corners[p], side, lam, 100 + p, device="cuda")
        Xs.append(X.float().contiguous())
        ys.append(y.float().contiguous())
        Ws.append(torch.zeros(w["n_window"], dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cfgb = lib.config(kernel="rbf", lam=lam, block_size=1024, rank=128, max_iters=480, seed=7,
                      precision="fp32", tol=1e-12)
    reps = lib.solve_batch(cfgb, Xs, [y.view(-1, 1) for y in ys], [W.view(-1, 1) for W in Ws],
                           [ell] * w["windows"])
    t_label = time.perf_counter() - t0
    cfg = lib.ws_config(d=d, D=D, hidden=H, lam=lam)
    Wf, c = inputs.ws_rff(w["seed"] + 2, d, ell, D)
    ws = lib.warm_start(cfg, Wf, c, inputs.ws_init_params(w["seed"] + 3, [D + 2, H, H, H, 1]))
    t0 = time.perf_counter()
    for p in range(w["windows"]):
        ws.add_problem(Xs[p], ys[p], Ws[p])
    losses = ws.train(epochs=12, batch=512, lr=1e-3, seed=11)
    t_train = time.perf_counter() - t0
    log("labels: worst relres %.2e in %.2f s; training %.2f s, losses %s"
        % (max(r["relres"] for r in reps), t_label, t_train, np.round(losses, 4).tolist()))
    del Xs, ys, Ws
    log("generating the target problem, n = %d" % n)
    X, y = inputs.ws_points(field, n, np.zeros(d), outer, lam, 999, device="cuda", chunk=1 << 16)
    X, y = X.float().contiguous(), y.float().contiguous()
    Y = y.view(-1, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W0 = ws.initial_iterate(X, y).view(-1, 1)
    torch.cuda.synchronize()
    t_infer = time.perf_counter() - t0
    starts = {"cold": None, "ridge": None, "network": W0}
    if n <= (1 << 24):
        feats, _ = ws.features(X, y)
        starts["ridge"] = ((y - feats[:, D + 1]) / lam).view(-1, 1).contiguous()
        del feats
    per_pass = int(math.ceil(n / b))
    rows = 1 << 17

    def cfg_of(iters, tol=0.0, check_every=0):
        return lib.config(kernel="rbf", lengthscale=ell, lam=lam, block_size=b, rank=128,
                          max_iters=iters, seed=13, precision="fp32", tol=tol,
                          check_every=check_every, check_rows=rows if large else 0)

    def relres(h, W):
        return h.residual_rows(W, rows, 21)[0] if large else h.residual(W)[0]

    budget = 2 * per_pass if not large else args.ws_budget
    arms = {}
    for name, W0a in starts.items():
        if name != "cold" and W0a is None:
            arms[name] = None
            continue
        W = torch.zeros_like(Y) if W0a is None else W0a.clone()
        h = lib.create(cfg_of(budget), X, Y)
        r0 = relres(h, W)
        rep = h.solve(W)
        r1 = relres(h, W)
        h.close()
        arms[name] = {"relres_at_W0": r0, "relres_after_budget": r1, "budget_iterations": budget,
                      "solve_seconds": round(rep["solve_ms"] / 1e3, 3)}
        log("%s start: relres %.4e at W0, %.4e after %d iterations" % (name, r0, r1, budget))
    ttr = None
    if not large:
        def solve(start, iters, tol):
            h = lib.create(cfg_of(iters, tol, per_pass), X, Y)
            rep = h.solve(start)
            h.close()
            return rep

        # guard: one probe pass from each start, judged by the residual
        probe = {}
        for name, start in (("cold", torch.zeros_like(Y)), ("warm", W0.clone())):
            # a positive tolerance no solve reaches makes the solver check once, after the pass
            probe[name] = solve(start, per_pass, 1e-300)["relres"]
        use_warm = probe["warm"] < probe["cold"]
        out = {}
        for name, start in (("cold", torch.zeros_like(Y)), ("warm", W0.clone())):
            rep = solve(start, per_pass * args.ttr_passes, 1e-3)
            ok = 0 <= rep["relres"] <= 1e-3
            out[name] = {"seconds": rep["solve_ms"] / 1e3 if ok else None, "reached": bool(ok),
                         "passes": rep["iters"] / per_pass, "relres": rep["relres"],
                         "ms_per_iteration": rep["solve_ms"] / max(1, rep["iters"]),
                         "step1_kernel_ms": rep["step1_kernel_ms"] / max(1, rep["step1_launches"])}
            log("%s: %s" % (name, json.dumps(out[name])))
        ttr = {"probe_relres": probe, "used": bool(use_warm), "cold": out["cold"], "warm": out["warm"]}
    h = lib.create(cfg_of(3), X, Y)
    Wt = torch.zeros_like(Y)
    rep = h.solve(Wt)
    h.close()
    kern_ms = rep["step1_kernel_ms"] / max(1, rep["step1_launches"])
    ms_iter = rep["solve_ms"] / max(1, rep["iters"])
    achieved = float(b) * n / (kern_ms * 1e-3) / 1e12
    if ttr is not None:
        chosen = ttr["warm"] if ttr["used"] else ttr["cold"]
        value = chosen["seconds"]
        if value is not None and ttr["used"]:
            value += t_infer
        metric = "time to rel. residual 1e-3 (s), learned warm start (guarded) vs cold, 1 GPU"
        unit = "s"
    else:
        value = arms["network"]["relres_after_budget"]
        metric = "relative residual after %d iterations from the learned warm start, 1 GPU" % budget
        unit = "relres"
    line = {
        "metric": metric, "value": None if value is None else round(value, 6), "unit": unit,
        "n_gpus": 1, "steps": budget, "warmup": 0, "ms_per_step": round(ms_iter, 4),
        "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (f16 hi/lo matrix-core distances), f64 Nystrom cores",
        "data": "synthetic (one RBF prior field, 32 training windows, fresh target points)",
        "config": {"workload": "warm_start_rbf_d9_n%d" % n, "n": n, "d": d, "lambda": lam,
                   "lengthscale": ell, "b": b, "r": 128, "windows": w["windows"],
                   "n_window": w["n_window"], "D": D, "hidden": H, "epochs": 12},
        "warm_start": {"arms": arms, "time_to_relres_1e-3": ttr,
                       "inference_seconds": round(t_infer, 4), "training_seconds": round(t_train, 3),
                       "label_seconds": round(t_label, 3),
                       "residual": "2^17-row estimate" if large else "all rows"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_EXP_TPS,
                     "unit": "Texp/s", "frac": round(achieved / PEAK_EXP_TPS, 4), "traffic": None,
                     "kernel": "mkv_kernel (Step-I product, float32 vector mode, 32x32x16 distances)",
                     "kernel_ms": round(kern_ms, 4)},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    ws.close()


def cpu_baseline_batched(host, ds, ells, b):
    """The float64 oracle's Step-I product for the first problems of the batch, one problem per
    host core (one BLAS thread each)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits

    from oracle import kernels as OK
    from oracle import rng as OR

    cores, nproc, ncpu, model = host_cores()

    def one(p):
        X, y = host[p]
        B = OR.sample_block(4 + p, 0, X.shape[0], b)
        OK.kernel_matmul(X[B], X, y[:, None], OK.RBF, float(ells[p]))
        return float(b) * X.shape[0] * (2 * int(ds[p]) + 2)

    with threadpool_limits(limits=1):
        with ThreadPoolExecutor(cores) as ex:
            t0 = time.perf_counter()
            flops = sum(ex.map(one, range(len(host))))
            sec = time.perf_counter() - t0
    return {"value": round(flops / sec / 1e9, 3), "unit": "GFLOP/s", "cores": cores, "nproc": nproc,
            "logical_cpus": ncpu, "cpu_model": model, "kind": "oracle",
            "sample": "Step-I products of the first %d problems (b=%d rows against all n_p "
                      "columns, float64 numpy, %d threads): %.2f s" % (len(host), b, cores, sec)}


def host_cores():
    """(threads to use, nproc, logical CPUs, CPU model) of this host: the CPUs this process may
    run on (its affinity), at most 16 (the host share of one GPU)."""
    nproc = len(os.sched_getaffinity(0))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return min(nproc, 16), nproc, os.cpu_count(), model


def cpu_baseline(X, Y, rows_per_core, ell, d, k, b, n):
    """The float64 oracle's kernel-block product on block rows against all n points, the rows
    split over the host cores (one thread each, numpy releases the interpreter lock)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits

    from oracle import kernels as OK
    from oracle import rng as OR

    cores, nproc, ncpu, model = host_cores()
    Xh = X.double().cpu().numpy()
    Yh = Y.double().cpu().numpy()
    rows = min(b, rows_per_core * cores)
    B = OR.sample_block(3, 0, n, b)[:rows]
    parts = np.array_split(B, cores)
    with threadpool_limits(limits=1):
        with ThreadPoolExecutor(cores) as ex:
            t0 = time.perf_counter()
            list(ex.map(lambda idx: OK.kernel_matmul(Xh[idx], Xh, Yh, OK.RBF, ell), parts))
            sec = time.perf_counter() - t0
    flops = float(rows) * n * (2 * d + 2 * k)
    return {"value": round(flops / sec / 1e9, 3), "unit": "GFLOP/s", "cores": cores, "nproc": nproc,
            "logical_cpus": ncpu, "cpu_model": model, "kind": "oracle",
            "sample": "%d block rows x %d columns x %d right-hand sides of the step-I product "
                      "(float64 numpy, %d threads of one BLAS thread each): %.2f s"
                      % (rows, n, k, cores, sec),
            "seconds_per_step_extrapolated": round(sec * b / rows, 2)}


if __name__ == "__main__":
    main()
