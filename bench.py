#!/usr/bin/env python3
"""Benchmark: guaranteed bounds on A_H for a 3D random-field voxel composite.

One step = the whole hot path on one microstructure: material setup
(A_M, B_M on the doubled grid), the d primal and d dual CG solves, and the
FP64 energy quadrature giving the upper and lower bounds ("time to bounds").
Workload: d = 3, N = 113 per axis (doubled grid M = 225, 11,390,625 points),
a two-phase voxel image of 225^3 voxels from a seeded Gaussian random field
(correlation length 0.05) thresholded at volume fraction 0.4, phases 1 and
100, CG to relative residual 1e-8.  The image is resident in HBM before the
timed region starts.

The metric is Mpoint-CG-iter/s: (2N-1)^3 grid points times the CG iterations
of all six solves, divided by the step time, for the plain FP64 path.  The
same steps are then timed in the FP32-iteration form (tolerance calibrated so
that the bounds stay within 1e-6 of the FP64 path), and the 2D serving mix
(512 requests of random circles, contrast 10..1e4, N in {41, 63, 123, 365})
is run sequentially through the plain FP64 path and through the
continuous-batching loop in the FP32-iteration form: all at once (capacity),
then with Poisson arrivals at 0.5, 0.8, 1.0 and 1.2x that capacity (p50/p99
latency, throughput).  A sample of 3D
random-field requests (N in {41, 63, 113}) is served the same way under an
HBM budget that admits about two N = 113 plans at once.  Further sections:
the FP32-iteration form on the anisotropic cube (N = 63), the 2D disc at
N = 41, 365, 1013 (bounds vs N), warm start, GaNi, reduced Ga and envelope
bounds; --main-only times the main workload alone.

    python bench.py [--gpus 1] [--steps 2] [--warmup 1] [--serve 32]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("fftgal_kernels.hip", "fftgal_internal.h"):
        with open(os.path.join(ROOT, "paper_1412_2033_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(cls, precision):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE medians scaled by the copy calibration), or None
    when no summary exists for this class or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    r = rec.get("%s/%s" % (cls, precision))
    if r is None or r.get("source_sha256_16") != kernel_source_hash():
        return None
    return int(1024 * (r["fetch_kib_median"] * r["fetch_scale"] + r["write_kib_median"] * r["write_scale"]))


def algorithmic_bytes(cls, d, N, M, es, gs, nc):
    """HBM bytes one launch of a kernel class must move (inputs read once, outputs written once)."""
    Nh = (N[-1] + 1) // 2
    Ns = (N[0] * N[1] if d == 3 else N[0]) * Nh
    if d == 3:
        t1 = d * M[0] * N[1] * Nh
        t2 = d * M[0] * M[1] * Nh
    else:
        t1 = t2 = d * M[0] * Nh
    Mt = 1
    for m in M:
        Mt *= m
    if cls == "expand":
        return es * (3 * nc * Ns + t1)
    if cls == "pencil_inv" or cls == "pencil_fwd":
        return es * (t1 + t2)
    if cls == "row":
        return es * 2 * t2 + gs * Mt
    if cls == "project":
        return es * (t1 + 2 * nc * Ns)
    if cls == "cg_update":
        return es * 6 * nc * Ns
    return 0


def iteration_model_bytes(d, N, M, w):
    """Bytes of one CG iteration in the pass-minimal model of the hot path (the
    operator in one round trip of the N x ... x (N+1)/2 half-spectrum per
    transform axis plus the material field, and the CG state): 4 d M N (N+1)/2
    2w + M^3 w + 7 N^2 (N+1)/2 2w in 3D, 4 d M (N+1)/2 2w + M^2 w + 7 (N+1)/2 2w
    in 2D (w = bytes of a real)."""
    Nh = (N[-1] + 1) // 2
    Mt = 1
    for m in M:
        Mt *= m
    if d == 3:
        return 4 * d * M[0] * N[1] * Nh * 2 * w + Mt * w + 7 * N[0] * N[1] * Nh * 2 * w
    return 4 * d * M[0] * Nh * 2 * w + Mt * w + 7 * N[0] * Nh * 2 * w


def host_workers():
    """Host threads the oracle's FFTs may use: the cores this process may run
    on, capped by OMP_NUM_THREADS when set (the host's share per GPU)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(micro, N, d, gpu_iters, gpu_small):
    """The oracle, as it stands (scipy.fft with every host thread it may use),
    on a bounded sample: full time to bounds of the two 2D N = 41 workloads
    (square of side 0.6 at contrast 10; disc of volume fraction 0.3 at
    contrast 100; FP64, rtol 1e-10), and one CG iteration of the 3D benchmark
    workload at full size, whose time times the GPU's CG iteration count
    estimates the oracle's time to bounds there (labelled as an estimate)."""
    import numpy as np
    import synth
    from oracle import ga, grids, material
    workers = host_workers()
    grids.set_workers(workers)
    full = {}
    for key, m in (("c1_square_N41", synth.square_inclusion(2, 0.6, 1.0, 10.0)),
                   ("c2_disc_N41", synth.circle_inclusion_vf(0.3, 1.0, 100.0))):
        t0 = time.perf_counter()
        res = ga.ga_bounds(material.make_material(m), (41, 41), tol=1e-10)
        dt = time.perf_counter() - t0
        its = sum(res["iters_primal"]) + sum(res["iters_dual"])
        full[key] = {"time_to_bounds_s": round(dt, 3), "cg_iterations": its,
                     "Mpoint_iter_per_s": round(81 * 81 * its / dt / 1e6, 3),
                     "gpu_time_to_bounds_s": gpu_small.get(key)}
    t0 = time.perf_counter()
    mat = material.make_material(micro)
    AM = material.double_grid_matrix(mat, N, tuple(2 * n - 1 for n in N), "A")
    setup_s = time.perf_counter() - t0
    M = next(a for a in AM.values() if a is not None).shape
    rng = np.random.default_rng(0)
    p = ga.project(rng.standard_normal((d,) + M), N, "E")
    x = np.zeros_like(p)
    r = p.copy()
    rr = ga.inner(r, r)
    t0 = time.perf_counter()
    q = ga.matvec(AM, p, N, "E")
    alpha = rr / ga.inner(p, q)
    x = x + alpha * p
    r = r - alpha * q
    rr_new = ga.inner(r, r)
    p = r + (rr_new / rr) * p
    it_s = time.perf_counter() - t0
    pts = 1
    for m in M:
        pts *= m
    grids.set_workers(1)
    est = 2 * setup_s + it_s * gpu_iters
    return {"value": round(pts / it_s / 1e6, 3), "unit": "Mpoint*CG-iter/s", "cores": workers, "kind": "oracle",
            "sample": "1 oracle CG iteration of the benchmark workload (Algorithm 2 matvec, FP64, d=3, M=225, "
                      "scipy.fft with %d threads) after building A_M (%.1f s): %.3f s per iteration; plus the full "
                      "oracle runs of the two 2D N=41 workloads" % (workers, setup_s, it_s),
            "host": {"os_cpu_count": os.cpu_count(), "threads_used": workers, "cpu_model": cpu_model()},
            "full_runs": full,
            "benchmark_time_to_bounds_estimate_s": round(est, 1),
            "estimate_note": "ESTIMATE, not a run: the measured oracle iteration time x the %d CG iterations the "
                             "GPU takes on this workload, plus twice the A_M setup (A and its inverse)" % gpu_iters}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"],
                    help="form whose rate is the headline value (default: the plain FP64 path)")
    ap.add_argument("--rtol", type=float, default=None)
    ap.add_argument("--rtol32", type=float, default=5e-6, help="CG tolerance of the FP32-iteration form")
    ap.add_argument("--serve", type=int, default=512, help="serving-mix requests (0: skip)")
    ap.add_argument("--aniso", type=int, default=63,
                    help="N of the anisotropic-cube comparison of the FP32-iteration form with FP64 (0: skip)")
    ap.add_argument("--main-only", action="store_true",
                    help="time the main workload only (every other section off; used for profiling)")
    ap.add_argument("--sweep2d", type=int, default=1,
                    help="2D disc (vf 0.3, contrast 100) bounds at N = 41, 365, 1013, FP64 rtol 1e-10 (0: skip)")
    ap.add_argument("--serve3d", type=int, default=8,
                    help="3D random-field requests (N in {41, 63, 113}) served under an HBM budget (0: skip)")
    ap.add_argument("--serve3d-budget-gib", type=float, default=2.5,
                    help="HBM budget of the 3D serving sample (GiB of plan workspaces)")
    ap.add_argument("--N", type=int, default=113)
    ap.add_argument("--equal-accuracy", type=int, default=1,
                    help="compare both forms at the same bound accuracy (1e-6) over a tolerance sweep (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--gani", type=int, default=225,
                    help="grid of the GaNi section (the paper compares GaNi of order 2N-1; 0: skip)")
    ap.add_argument("--warm-coarse", type=int, default=41,
                    help="coarse N of the warm-start / bound-monitoring section (0: skip)")
    ap.add_argument("--reduced", type=int, default=81,
                    help="N of the reduced-Ga section (3D, on the benchmark image; 0: skip)")
    ap.add_argument("--reduced-prime", type=int, default=113,
                    help="N of the reduced-Ga section at an order that is not 3,5,7-smooth (Bluestein "
                         "transforms; default the benchmark order 113; 0: skip)")
    ap.add_argument("--fast-grid", type=int, default=1,
                    help="FFTGAL_FAST_GRID against the default grid at 3D N = 81 and 2D N = 201 (0: skip)")
    ap.add_argument("--generic", type=int, default=1,
                    help="plans on lengths without specialised kernels (3D 45^3, GaNi 41^3 and 201^2; 0: skip)")
    ap.add_argument("--envelope", type=int, default=1,
                    help="upper-upper / lower-lower bounds section on an anisotropic cube inclusion (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes 5 times (profiler counter scale)")
    args = ap.parse_args()
    if args.main_only:
        args.serve = args.serve3d = args.gani = args.warm_coarse = args.reduced = args.reduced_prime = 0
        args.fast_grid = args.generic = 0
        args.equal_accuracy = 0
        args.envelope = args.aniso = args.sweep2d = 0
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU (independent solves and requests shard across GPUs "
              "by problem); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        # a plain device copy: the profiler's counter scale, and the streaming
        # rate this GPU reaches (read + write bytes over event time)
        src = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        dst.copy_(src)
        e0.record()
        for _ in range(4):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 4
        print(json.dumps({"copy_calibration_bytes": src.numel() * 4, "launches": 5,
                          "copy_GBs": round(2 * src.numel() * 4 / (ms * 1e-3) / 1e9, 1)}))
        return

    import synth
    from paper_1412_2033_amd import fftgal

    d = 3
    N = (args.N,) * d
    M = tuple(2 * n - 1 for n in N)
    rtol64 = args.rtol if args.rtol is not None else 1e-8
    print("bench: building workload d=3 N=%d M=%d" % (N[0], M[0]), file=sys.stderr, flush=True)
    micro = synth.grf_voxels(5, M, d=3, corr_len=0.05, vf=0.4, a_matrix=1.0, a_incl=100.0)
    dev = torch.device("cuda:0")
    micro_dev = dict(micro)
    micro_dev["image"] = torch.from_numpy(np.ascontiguousarray(micro["image"])).to(dev)
    pts = M[0] * M[1] * M[2]

    def time_form(precision, rtol):
        plan = fftgal.Plan(d, N, precision, device=dev, P=M)
        es = 16 if precision == "fp64" else 8
        gs = 8 if precision == "fp64" else 4
        for w in range(args.warmup):
            res = plan.run(micro_dev, rtol=rtol)
            print("bench: %s warmup %d done, iters %s / %s" % (
                precision, w, [i["iters"] for i in res["info_primal"]], [i["iters"] for i in res["info_dual"]]),
                file=sys.stderr, flush=True)
        # one fully traced step (outside the timed region): per-class breakdown
        plan.set_timing(True)
        plan.read_timing()
        traced = plan.run(micro_dev, rtol=rtol)
        breakdown = plan.read_timing()
        it_p = sum(i["iters"] for i in traced["info_primal"])
        it_d = sum(i["iters"] for i in traced["info_dual"])
        per_cls = {}
        design_bytes = 0
        for cls, (ms, cnt) in breakdown.items():
            if cnt == 0:
                continue
            by = algorithmic_bytes(cls, d, N, M, es, gs, 1) * it_p + algorithmic_bytes(cls, d, N, M, es, gs, d - 1) * it_d
            design_bytes += by
            per_cls[cls] = {"ms": round(ms, 3), "launches": cnt, "avg_us": round(1e3 * ms / cnt, 2),
                            "GBs": round(by / (ms * 1e-3) / 1e9, 1) if by > 0 else None}
        design_bytes /= max(1, it_p + it_d)
        dom = max((c for c in per_cls if per_cls[c]["GBs"]), key=lambda c: per_cls[c]["ms"])
        # timed steps: only the dominant class is bracketed by HIP events
        plan.set_timing(True, classes=(dom,))
        plan.read_timing()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        results = []
        for k in range(args.steps):
            results.append(plan.run(micro_dev, rtol=rtol))
            print("bench: %s step %d done" % (precision, k), file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        timing = plan.read_timing()
        plan.set_timing(False)
        plan.close()
        iters_p = sum(sum(i["iters"] for i in r["info_primal"]) for r in results)
        iters_d = sum(sum(i["iters"] for i in r["info_dual"]) for r in results)
        total_iters = iters_p + iters_d
        # algorithmic bytes of all operator launches of the class over the timed
        # steps, divided by their total event-timed duration (launches of
        # solves that already stopped return at once; their time is included)
        dom_bytes_total = (algorithmic_bytes(dom, d, N, M, es, gs, 1) * iters_p +
                           algorithmic_bytes(dom, d, N, M, es, gs, d - 1) * iters_d)
        dom_bytes = dom_bytes_total / total_iters
        dom_avg_s = timing[dom][0] * 1e-3 / total_iters
        achieved = dom_bytes_total / (timing[dom][0] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom, precision),
                "kernel": dom, "bytes_per_launch": int(dom_bytes), "avg_launch_us": round(dom_avg_s * 1e6, 2),
                "launches_timed": timing[dom][1], "iterations_timed": total_iters}
        # the whole CG iteration: the pass-minimal model's bytes and this
        # design's algorithmic bytes per iteration, over the time per iteration
        # of the whole timed run (material setup, right-hand sides and bounds
        # included, so conservative)
        it_s = elapsed / total_iters
        model = iteration_model_bytes(d, N, M, es // 2)
        roof["iteration"] = {"model_bytes": int(model), "design_bytes": int(design_bytes),
                             "us_per_iteration": round(it_s * 1e6, 2),
                             "frac_model": round(model / it_s / 1e9 / HBM_PEAK_GBS, 4),
                             "frac_design": round(design_bytes / it_s / 1e9 / HBM_PEAK_GBS, 4)}
        last = results[-1]
        return {"elapsed": elapsed, "value": pts * total_iters / elapsed / 1e6, "ms_per_step": 1e3 * elapsed / args.steps,
                "kernels": per_cls, "roofline": roof, "last": last,
                "iters": {"primal": [i["iters"] for i in last["info_primal"]],
                          "dual": [i["iters"] for i in last["info_dual"]]}}

    main_prec = args.precision
    main_rtol = rtol64 if main_prec == "fp64" else args.rtol32
    prim = time_form(main_prec, main_rtol)
    other_prec = "fp32" if main_prec == "fp64" else "fp64"
    other = time_form(other_prec, args.rtol32 if other_prec == "fp32" else rtol64)
    f64 = prim if main_prec == "fp64" else other
    f32 = other if main_prec == "fp64" else prim

    def rel(a, b):
        return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))

    last = prim["last"]
    out = {
        "metric": "Mpoint*CG-iter/s (time-to-bounds at d=3,N=113)",
        "value": round(prim["value"], 2),
        "unit": "Mpoint*CG-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(prim["ms_per_step"], 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "3D two-phase GRF voxel composite (225^3 voxels, corr. length 0.05, vf 0.4, "
                               "contrast 1:100), Ga primal+dual CG to rel. residual %g, bounds in FP64" % main_rtol,
                   "d": d, "N": N[0], "M": M[0], "P": M[0], "precision": main_prec},
        "time_to_bounds_s": round(prim["ms_per_step"] / 1e3, 4),
        "cg_iterations": prim["iters"],
        "upper_diag": [round(float(v), 10) for v in np.diag(last["upper"])],
        "lower_diag": [round(float(v), 10) for v in np.diag(last["lower"])],
        "gap": last["gap"],
        "kernels": prim["kernels"],
        "roofline": prim["roofline"],
        "fp32_iteration_form": {
            "rtol": args.rtol32, "time_to_bounds_s": round(f32["ms_per_step"] / 1e3, 4),
            "Mpoint_iter_per_s": round(f32["value"], 1), "cg_iterations": f32["iters"],
            "bound_rel_err_vs_fp64": max(rel(f32["last"][k], f64["last"][k]) for k in ("upper", "lower")),
            "speedup_vs_fp64": round(f64["ms_per_step"] / f32["ms_per_step"], 3),
            "kernels": f32["kernels"], "roofline": f32["roofline"]},
    }
    if args.equal_accuracy:
        out["equal_accuracy"] = equal_accuracy_bench(fftgal, micro_dev, d, N, M, f64["last"], dev)
    if args.warm_coarse > 0:
        out["warm_start"] = warm_start_bench(fftgal, micro_dev, d, N, M, args.warm_coarse, rtol64, dev)
    if args.gani > 0:
        out["gani"] = gani_bench(fftgal, micro_dev, d, M, args.gani, rtol64, last, dev)
    if args.reduced > 0:
        out["reduced"] = reduced_bench(fftgal, micro_dev, d, M, args.reduced, rtol64, dev)
    if args.reduced_prime > 0:
        out["reduced_bluestein"] = reduced_bench(fftgal, micro_dev, d, M, args.reduced_prime, rtol64, dev,
                                                 variants=("reduced", "reduced_lean"))
    if args.fast_grid:
        out["fast_grid"] = fast_grid_bench(fftgal, micro_dev, d, M, dev)
    if args.generic:
        out["generic"] = generic_bench(fftgal, dev)
    if args.envelope:
        out["envelope"] = envelope_bench(fftgal, d, N, M, rtol64, dev)
    if args.aniso:
        out["aniso_fp32"] = aniso_bench(fftgal, args.aniso, rtol64, args.rtol32, dev)
    if args.sweep2d:
        out["sweep_2d"] = sweep2d_bench(fftgal, dev)
    if args.serve > 0:
        out["serving"] = serving_bench(args.serve, args.rtol32)
    if args.serve3d > 0:
        out["serving_3d"] = serving3d_bench(args.serve3d, args.rtol32, args.serve3d_budget_gib)
    if not args.no_cpu_baseline:
        gpu_small = small_2d_times(fftgal, dev)
        print("bench: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        gpu_iters = sum(f64["iters"]["primal"]) + sum(f64["iters"]["dual"])
        out["cpu_baseline"] = cpu_baseline(micro, N, d, gpu_iters, gpu_small)
    print(json.dumps(out), flush=True)


def small_2d_times(fftgal, dev):
    """GPU time to bounds of the two 2D N = 41 workloads the CPU baseline runs
    in full (FP64, rtol 1e-10; best of three after one warm-up)."""
    import synth
    import torch
    out = {}
    for key, m in (("c1_square_N41", synth.square_inclusion(2, 0.6, 1.0, 10.0)),
                   ("c2_disc_N41", synth.circle_inclusion_vf(0.3, 1.0, 100.0))):
        plan = fftgal.Plan(2, (41, 41), "fp64", device=dev)
        plan.run(m, rtol=1e-10)
        best = None
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.run(m, rtol=1e-10)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        plan.close()
        out[key] = round(best, 5)
    return out


BOUND_TOL = 1e-6  # bound tolerance of the monitoring section (the FP32-iteration form's stated accuracy)


def warm_start_bench(fftgal, micro_dev, d, N, M, Nc, rtol, dev):
    """Bound monitoring and coarse-to-fine warm start on the benchmark workload
    (FP64): time to bounds and CG iterations from e_0 = 0, from the prolonged
    solution of an N = Nc plan, and with the bound test at BOUND_TOL; the first
    bound of each start, and the iterations after which the monitored bound
    entries are within 1e-4 / 1e-6 / 1e-8 of their final values."""
    import numpy as np
    import torch
    print("bench: warm start from N=%d" % Nc, file=sys.stderr, flush=True)

    def within(h, tol):
        fin = h[-1]
        return [int(np.argmax(np.abs(h - fin) <= t * abs(fin))) for t in tol]

    out = {"coarse_N": Nc, "rtol": rtol, "btol": BOUND_TOL}
    tols = (1e-4, 1e-6, 1e-8)
    for mode in ("cold", "warm", "bound_tol"):
        fine = fftgal.Plan(d, N, "fp64", device=dev, P=M)
        coarse = fftgal.Plan(d, (Nc,) * d, "fp64", device=dev, P=M) if mode == "warm" else None
        if mode == "bound_tol":
            fine.set_bound_tol(BOUND_TOL)
        try:
            for rep in range(2):  # the second repetition is timed
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                t_coarse = 0.0
                if coarse is not None:
                    coarse.run(micro_dev, rtol=rtol)
                    torch.cuda.synchronize()
                    t_coarse = time.perf_counter() - t0
                res = fine.run(micro_dev, rtol=rtol, warm_from=coarse)
                torch.cuda.synchronize()
                elapsed = time.perf_counter() - t0
            hist = {(k, a): fine.history(k, a) for k in (0, 1) for a in range(d)}
        finally:
            fine.close()
            if coarse is not None:
                coarse.close()
        out[mode] = {
            "time_to_bounds_s": round(elapsed, 4), "coarse_s": round(t_coarse, 4),
            "cg_iterations": {"primal": [i["iters"] for i in res["info_primal"]],
                              "dual": [i["iters"] for i in res["info_dual"]]},
            "first_upper_diag": [round(float(hist[(0, a)][0]), 6) for a in range(d)],
            "first_lower_diag": [round(float(1.0 / hist[(1, a)][0]), 6) for a in range(d)],
            "iters_to_bound_rel_1e-4_1e-6_1e-8": {"primal": [within(hist[(0, a)], tols) for a in range(d)],
                                                   "dual": [within(hist[(1, a)], tols) for a in range(d)]},
            "upper_diag": [round(float(v), 10) for v in np.diag(res["upper"])],
        }
        if mode == "bound_tol":
            ref = out["cold"]["_bounds"]
            out[mode]["bound_rel_diff_vs_cold"] = max(
                float(np.linalg.norm(res[k] - ref[k]) / np.linalg.norm(ref[k])) for k in ("upper", "lower"))
            out[mode]["speedup_vs_cold"] = round(out["cold"]["time_to_bounds_s"] / elapsed, 3)
        out[mode]["_bounds"] = {"upper": res["upper"], "lower": res["lower"]}
    for mode in ("cold", "warm", "bound_tol"):
        del out[mode]["_bounds"]
    return out


def gani_bench(fftgal, micro_dev, d, P, Ng, rtol, ga_last, dev):
    """GaNi of order Ng on the benchmark image (material sampled at the grid
    points; the paper compares GaNi of order 2N-1 with Ga of order N) and its
    a-posteriori guaranteed bounds (exact energies of the GaNi minimisers on a
    Ga plan of order Ng), against the Ga bounds of the main run."""
    import numpy as np
    import torch
    print("bench: GaNi N=%d" % Ng, file=sys.stderr, flush=True)
    Nt = (Ng,) * d
    gp = fftgal.Plan(d, Nt, "fp64", device=dev, P=P, scheme="gani")
    ap = fftgal.Plan(d, Nt, "fp64", device=dev, P=P)
    try:
        gp.run(micro_dev, rtol=rtol)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = gp.run(micro_dev, rtol=rtol)
        torch.cuda.synchronize()
        t_gani = time.perf_counter() - t0
        ap.set_material(micro_dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        up, lo, gap = ap.bounds_of(gp)
        torch.cuda.synchronize()
        t_apost = time.perf_counter() - t0
    finally:
        gp.close()
        ap.close()

    def diag(m):
        return [round(float(v), 6) for v in np.diag(m)]

    return {"N": Ng, "rtol": rtol, "time_gani_s": round(t_gani, 4), "time_apost_s": round(t_apost, 4),
            "cg_iterations": {"primal": [i["iters"] for i in res["info_primal"]],
                              "dual": [i["iters"] for i in res["info_dual"]]},
            "A_gani_diag": diag(res["upper"]), "duality_rel_diff": float(
                np.linalg.norm(res["upper"] - res["lower"]) / np.linalg.norm(res["upper"])),
            "apost_upper_diag": diag(up), "apost_lower_diag": diag(lo), "apost_gap": round(gap, 6),
            "ga_N113_upper_diag": diag(ga_last["upper"]), "ga_N113_lower_diag": diag(ga_last["lower"]),
            "ga_N113_gap": round(float(ga_last["gap"]), 6)}


def reduced_bench(fftgal, micro_dev, d, P, Nr, rtol, dev, variants=("reduced", "reduced_lean")):
    """Reduced Ga (Lemma reduce_grid, Algorithm 3) against the double-grid Ga
    of the same order Nr on the benchmark image: time to bounds, CG
    iterations, workspace bytes and the difference of the bounds (FP64)."""
    import numpy as np
    import torch
    print("bench: reduced Ga N=%d" % Nr, file=sys.stderr, flush=True)
    Nt = (Nr,) * d
    out = {"N": Nr, "rtol": rtol}
    res = {}
    # "reduced": the shifts of each pass in one launch; "reduced_lean": one set
    # of intermediates, shifts in turn (smallest workspace); "ga": double grid
    for name in tuple(variants) + ("ga",):
        scheme = "ga" if name == "ga" else "reduced"
        plan = fftgal.Plan(d, Nt, "fp64", device=dev, P=P, scheme=scheme, lean=name == "reduced_lean")
        try:
            plan.run(micro_dev, rtol=rtol)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = plan.run(micro_dev, rtol=rtol)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            grid = list(plan.M)
        finally:
            plan.close()
        res[name] = r
        out[name] = {"time_to_bounds_s": round(el, 4), "workspace_bytes": plan.nbytes, "transform_grid": grid,
                       "cg_iterations": {"primal": [i["iters"] for i in r["info_primal"]],
                                         "dual": [i["iters"] for i in r["info_dual"]]},
                       "upper_diag": [round(float(v), 8) for v in np.diag(r["upper"])]}
    out["bound_rel_diff"] = max(
        float(np.linalg.norm(res[v][k] - res["ga"][k]) / np.linalg.norm(res["ga"][k]))
        for v in variants for k in ("upper", "lower"))
    return out


def fast_grid_bench(fftgal, micro_dev, d, P, dev, N3=81, N2=201):
    """FFTGAL_FAST_GRID against the default grid: the benchmark image at 3D
    order N3 (default double grid 175^3, generic kernels; fast 225^3) and the
    2D disc at order N2 (405^2 against 729^2), FP64."""
    import numpy as np
    import synth
    import torch
    print("bench: fast grid 3D N=%d, 2D N=%d" % (N3, N2), file=sys.stderr, flush=True)
    cases = (("3d", (N3,) * d, micro_dev, P, 1e-8),
             ("2d", (N2, N2), synth.circle_inclusion_vf(0.3, 1.0, 100.0), None, 1e-10))
    out = {}
    for tag, Nt, micro, Pm, rtol in cases:
        res = {}
        sec = {"N": Nt[0], "rtol": rtol}
        for fast in (False, True):
            plan = fftgal.Plan(len(Nt), Nt, "fp64", device=dev, P=Pm, fast_grid=fast)
            try:
                plan.run(micro, rtol=rtol)  # warm-up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = plan.run(micro, rtol=rtol)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                grid = list(plan.M)
            finally:
                plan.close()
            res[fast] = r
            sec["fast_grid" if fast else "default"] = {
                "time_to_bounds_s": round(el, 4), "grid": grid, "workspace_bytes": plan.nbytes,
                "cg_iterations": sum(i["iters"] for i in r["info_primal"] + r["info_dual"])}
        sec["speedup"] = round(sec["default"]["time_to_bounds_s"] / sec["fast_grid"]["time_to_bounds_s"], 2)
        sec["bound_rel_diff"] = max(float(np.linalg.norm(res[True][k] - res[False][k]) / np.linalg.norm(res[False][k]))
                                    for k in ("upper", "lower"))
        out[tag] = sec
    return out


def generic_bench(fftgal, dev):
    """Plans on lengths without specialised kernels (the generic transform
    kernels): the 3D double grid 45^3 (order 21, radices 9 5), 3D GaNi of order
    41 (Bluestein, L = 81) and 2D GaNi of order 201 (Bluestein, L = 405 = 9 9 5),
    FP64 and FP32 iterations; time to bounds (set_material, 2d solves, bounds;
    best of two runs after a warm-up) and that time per CG iteration."""
    import synth
    import torch
    print("bench: generic lengths", file=sys.stderr, flush=True)
    cases = (("ga3d_N21", 3, 21, "ga", 1e-8),
             ("gani3d_N41", 3, 41, "gani", 1e-8),
             ("gani2d_N201", 2, 201, "gani", 1e-10))
    out = {}
    for tag, d, n, scheme, rtol in cases:
        P = 2 * n - 1
        if d == 3:
            micro = synth.grf_voxels(5, (P,) * 3, d=3, corr_len=0.05, vf=0.4, a_matrix=1.0, a_incl=100.0)
        else:
            micro = synth.circle_inclusion_vf(0.3, 1.0, 100.0)
        sec = {}
        for prec in ("fp64", "fp32"):
            rt = rtol if prec == "fp64" else 5e-6
            plan = fftgal.Plan(d, (n,) * d, prec, device=dev, P=micro.get("P"), scheme=scheme)
            try:
                plan.run(micro, rtol=rt)  # warm-up
                best = None
                for _ in range(2):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    r = plan.run(micro, rtol=rt)
                    torch.cuda.synchronize()
                    el = time.perf_counter() - t0
                    best = el if best is None else min(best, el)
                grid = list(plan.M)
            finally:
                plan.close()
            its = sum(i["iters"] for i in r["info_primal"] + r["info_dual"])
            sec[prec] = {"rtol": rt, "grid": grid, "time_to_bounds_s": round(best, 4), "cg_iterations": its,
                         "us_per_cg_iteration": round(best / max(its, 1) * 1e6, 1)}
        out[tag] = sec
    return out


def envelope_bench(fftgal, d, N, M, rtol, dev):
    """Upper-upper / lower-lower bounds (Lemma bounds_bounds) on an anisotropic
    cube inclusion whose faces cut the voxels: the voxel envelope images on the
    P = M grid, the Ga bounds of the envelope material (primal with the upper
    image, dual with the lower), against the Ga bounds of the exact inclusion
    material on the same plan size."""
    import numpy as np
    import torch
    import synth
    print("bench: envelope bounds", file=sys.stderr, flush=True)
    micro = synth.cube_inclusion_aniso(0.45, 5)
    plan = fftgal.Plan(d, N, "fp64", device=dev, P=M)
    try:
        times = {}
        for rep in range(2):  # the second repetition is timed
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            up, lo = plan.envelope_images(micro, M)
            torch.cuda.synchronize()
            times["images_s"] = time.perf_counter() - t0
            env = plan.run({"d": d, "kind": "voxels", "P": M, "image": up, "image_dual": lo}, rtol=rtol)
            torch.cuda.synchronize()
            times["envelope_to_bounds_s"] = time.perf_counter() - t0
            t0 = time.perf_counter()
            exact = plan.run(micro, rtol=rtol)
            torch.cuda.synchronize()
            times["exact_to_bounds_s"] = time.perf_counter() - t0
        cut = int(torch.count_nonzero(up != lo).item())
    finally:
        plan.close()

    def diag(m):
        return [round(float(v), 6) for v in np.diag(m)]

    scale = np.abs(exact["upper"]).max()
    return {"microstructure": "cube inclusion, side 0.45, anisotropic SPD phases (seed 5)", "P": M[0], "N": N[0],
            "rtol": rtol, **{k: round(v, 4) for k, v in times.items()}, "cut_voxels": cut,
            "envelope_upper_diag": diag(env["upper"]), "envelope_lower_diag": diag(env["lower"]),
            "exact_upper_diag": diag(exact["upper"]), "exact_lower_diag": diag(exact["lower"]),
            "envelope_gap": round(float(env["gap"]), 6), "exact_gap": round(float(exact["gap"]), 6),
            "brackets_exact": bool(np.min(np.linalg.eigvalsh(env["upper"] - exact["upper"])) >= -1e-10 * scale and
                                   np.min(np.linalg.eigvalsh(exact["lower"] - env["lower"])) >= -1e-10 * scale)}


def serving_bench(n, rtol, seed=4):
    """Serving-mix sample: sequential plain FP64 vs continuous-batched FP32 iterations, same tolerance."""
    import numpy as np
    import synth
    from paper_1412_2033_amd import serve
    base = synth.serving_requests(seed, n, rate_per_s=1.0)
    print("bench: serving sample of %d requests: sequential FP64" % n, file=sys.stderr, flush=True)
    seq, t_seq = serve.sequential(base, precision="fp64", rtol=rtol)
    by = {r["id"]: r for r in seq}
    at_once = [dict(r, arrival_s=0.0) for r in base]
    print("bench: serving: batched FP32, one solve slot per plan, all requests at t=0", file=sys.stderr, flush=True)
    srv1 = serve.Server(precision="fp32", rtol=rtol, concurrent=False)
    rec1, st1 = srv1.run(at_once)
    lat1 = [r["latency_s"] for r in rec1]
    srv1.close()
    srv = serve.Server(precision="fp32", rtol=rtol)
    print("bench: serving: batched FP32, all requests at t=0", file=sys.stderr, flush=True)
    rec0, st0 = srv.run(at_once)
    lat0 = [r["latency_s"] for r in rec0]
    capacity = n / st0["wall_s"]
    # Poisson arrivals at 0.8x the batched capacity, and a sweep of the load
    sweep = []
    rec = st = None
    for factor in (0.5, 0.8, 1.0, 1.2):
        r_f = factor * capacity
        reqs = synth.serving_requests(seed, n, rate_per_s=r_f)
        print("bench: serving: Poisson arrivals at %.1f req/s (%.1fx capacity)" % (r_f, factor), file=sys.stderr,
              flush=True)
        rec_f, st_f = srv.run(reqs)
        lat_f = [r["latency_s"] for r in rec_f]
        sweep.append({"load": factor, "rate_req_per_s": round(r_f, 2), "wall_s": round(st_f["wall_s"], 3),
                      "p50_s": round(serve.percentile(lat_f, 50), 4), "p99_s": round(serve.percentile(lat_f, 99), 4)})
        if factor == 0.8:
            rec, st, rate = rec_f, st_f, r_f
    srv.close()
    lat = [r["latency_s"] for r in rec]
    seq_t = [r["seconds"] for r in seq]
    err = max(float(np.linalg.norm(r[k] - by[r["id"]][k]) / np.linalg.norm(by[r["id"]][k]))
              for r in rec for k in ("upper", "lower"))
    bad = sum(1 for r in rec for s in r["status"] if s != 0)
    return {"requests": n, "mix": "2D random circles k~U{5..50}, r~U[0.02,0.08], contrast logU[10,1e4], "
                                  "N in {41,63,123,365}",
            "rtol": rtol,
            "sequential_fp64": {"wall_s": round(t_seq, 3), "req_per_s": round(n / t_seq, 2),
                                "p50_s": round(serve.percentile(seq_t, 50), 4),
                                "p99_s": round(serve.percentile(seq_t, 99), 4)},
            "batched_fp32_capacity": {"wall_s": round(st0["wall_s"], 3), "req_per_s": round(capacity, 2),
                                      "Mpoint_iter_per_s": round(st0["Mpoint_iter_per_s"], 1),
                                      "solves_per_request_at_once": "all 2d (concurrent plans)",
                                      "p50_s_all_at_t0": round(serve.percentile(lat0, 50), 4),
                                      "p99_s_all_at_t0": round(serve.percentile(lat0, 99), 4)},
            "batched_fp32_capacity_one_solve_at_a_time": {
                "wall_s": round(st1["wall_s"], 3), "req_per_s": round(n / st1["wall_s"], 2),
                "p50_s_all_at_t0": round(serve.percentile(lat1, 50), 4),
                "p99_s_all_at_t0": round(serve.percentile(lat1, 99), 4)},
            "batched_fp32_poisson": {"rate_req_per_s": round(rate, 2), "wall_s": round(st["wall_s"], 3),
                                     "p50_s": round(serve.percentile(lat, 50), 4),
                                     "p99_s": round(serve.percentile(lat, 99), 4),
                                     "Mpoint_iter_per_s": round(st["Mpoint_iter_per_s"], 1)},
            "load_sweep": sweep,
            "throughput_speedup_vs_sequential_fp64": round(capacity / (n / t_seq), 2),
            "max_bound_rel_diff_vs_fp64": err, "solves_not_converged": bad}


def aniso_bench(fftgal, n, rtol64, rtol32, dev):
    """Centred cube of side 0.5 with an anisotropic SPD inclusion (eigenvalues
    log-uniform in [10, 1000], random rotation, seed 3) in an isotropic matrix
    of 1, d = 3, order n: time to bounds of the plain FP64 path and of the
    FP32-iteration form (the anisotropic row pass), and the bound error of the
    latter against the former."""
    import numpy as np
    import synth
    import torch
    micro = synth.cube_inclusion_aniso(0.5, 3)
    N = (n,) * 3
    out = {"microstructure": "cube side 0.5, anisotropic SPD inclusion (seed 3), matrix 1", "N": n}
    res = {}
    for prec, rtol in (("fp64", rtol64), ("fp32", rtol32)):
        plan = fftgal.Plan(3, N, prec, device=dev)
        plan.run(micro, rtol=rtol)  # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = plan.run(micro, rtol=rtol)
        torch.cuda.synchronize()
        res[prec] = r
        out[prec] = {"rtol": rtol, "time_to_bounds_s": round(time.perf_counter() - t, 4),
                     "cg_iterations": {"primal": [i["iters"] for i in r["info_primal"]],
                                       "dual": [i["iters"] for i in r["info_dual"]]},
                     "upper_diag": [round(float(v), 8) for v in np.diag(r["upper"])],
                     "lower_diag": [round(float(v), 8) for v in np.diag(r["lower"])]}
        plan.close()
    out["fp32_bound_rel_err_vs_fp64"] = max(
        float(np.linalg.norm(res["fp32"][k] - res["fp64"][k]) / np.linalg.norm(res["fp64"][k]))
        for k in ("upper", "lower"))
    out["speedup_fp32_vs_fp64"] = round(out["fp64"]["time_to_bounds_s"] / out["fp32"]["time_to_bounds_s"], 3)
    return out


def equal_accuracy_bench(fftgal, micro_dev, d, N, M, ref, dev, target=1e-6):
    """Time to bounds of both forms at the same stated bound accuracy: for each
    form the loosest CG tolerance of a sweep whose bounds stay within `target`
    (relative, Frobenius) of the FP64 bounds at rtol 1e-8 (`ref`)."""
    import numpy as np
    import torch
    out = {"target_bound_rel_err": target, "reference": "FP64 path at rtol 1e-8", "forms": {}}
    for prec in ("fp64", "fp32"):
        plan = fftgal.Plan(d, N, prec, device=dev, P=M)
        plan.run(micro_dev, rtol=1e-4)  # warm-up
        rows = []
        for rtol in (1e-3, 3e-4, 1e-4, 3e-5, 1e-5, 5e-6):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = plan.run(micro_dev, rtol=rtol)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            err = max(float(np.linalg.norm(r[k] - ref[k]) / np.linalg.norm(ref[k])) for k in ("upper", "lower"))
            rows.append({"rtol": rtol, "time_to_bounds_s": round(el, 4), "bound_rel_err": err,
                         "cg_iterations": sum(i["iters"] for i in r["info_primal"] + r["info_dual"])})
            print("bench: equal accuracy %s rtol %g: %.4f s, err %.2e" % (prec, rtol, el, err), file=sys.stderr,
                  flush=True)
        plan.close()
        ok = [row for row in rows if row["bound_rel_err"] <= target]
        out["forms"][prec] = {"sweep": rows, "chosen": ok[0] if ok else None}
    a, b = out["forms"]["fp64"]["chosen"], out["forms"]["fp32"]["chosen"]
    out["fp32_speedup_at_equal_accuracy"] = round(a["time_to_bounds_s"] / b["time_to_bounds_s"], 3) if a and b else None
    return out


def sweep2d_bench(fftgal, dev, Ns=(41, 365, 1013)):
    """Centred disc of volume fraction 0.3, phases 1 and 100, d = 2: plain FP64
    bounds to relative residual 1e-10 at each order N (doubled grids 81^2,
    729^2, 2025^2), with time to bounds (best of three runs after a warm-up)
    and the trace gap."""
    import numpy as np
    import synth
    import torch
    micro = synth.circle_inclusion_vf(0.3, 1.0, 100.0)
    out = {"microstructure": "centred disc, vf 0.3, contrast 100", "rtol": 1e-10, "orders": []}
    for n in Ns:
        times = {}
        for conc in (False, True):
            # one solve after another, or all four in shared launches (fftgal_solve_all)
            plan = fftgal.Plan(2, (n, n), "fp64", device=dev, concurrent=conc)
            plan.run(micro, rtol=1e-10)  # warm-up
            best = float("inf")
            for _ in range(3):  # runs of a few ms: the best of three
                torch.cuda.synchronize()
                t = time.perf_counter()
                r = plan.run(micro, rtol=1e-10)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t)
            times[conc] = best
            plan.close()
        dt = times[False]
        out["orders"].append({"N": n, "M": 2 * n - 1, "time_to_bounds_s": round(dt, 4),
                              "time_to_bounds_concurrent_s": round(times[True], 4),
                              "cg_iterations": {"primal": [i["iters"] for i in r["info_primal"]],
                                                "dual": [i["iters"] for i in r["info_dual"]]},
                              "upper_diag": [round(float(v), 10) for v in np.diag(r["upper"])],
                              "lower_diag": [round(float(v), 10) for v in np.diag(r["lower"])],
                              "gap": round(float(r["gap"]), 10)})
    return out


def serving3d_bench(n, rtol, budget_gib, seed=9):
    """3D random-field requests (N in {41, 63, 113}, the benchmark's material
    recipe) served under an HBM budget that admits about two N = 113 plans at
    once: sequential plain FP64 vs continuous-batched FP32 iterations, same
    tolerance."""
    import numpy as np
    import synth
    from paper_1412_2033_amd import serve
    print("bench: 3D serving sample of %d requests: building images" % n, file=sys.stderr, flush=True)
    base = synth.serving_requests_3d(seed, n, rate_per_s=1.0)
    print("bench: 3D serving: sequential FP64", file=sys.stderr, flush=True)
    seq, t_seq = serve.sequential(base, precision="fp64", rtol=rtol)
    by = {r["id"]: r for r in seq}
    budget = int(budget_gib * (1 << 30))
    srv = serve.Server(precision="fp32", rtol=rtol, hbm_budget=budget, capacity=16)
    print("bench: 3D serving: batched FP32, all requests at t=0", file=sys.stderr, flush=True)
    rec0, st0 = srv.run(synth.with_arrivals(base, seed, 1e9))
    capacity = n / st0["wall_s"]
    rate = 0.8 * capacity
    print("bench: 3D serving: Poisson arrivals at %.1f req/s" % rate, file=sys.stderr, flush=True)
    rec, st = srv.run(synth.with_arrivals(base, seed + 1, rate))
    srv.close()
    lat = [r["latency_s"] for r in rec]
    seq_t = [r["seconds"] for r in seq]
    err = max(float(np.linalg.norm(r[k] - by[r["id"]][k]) / np.linalg.norm(by[r["id"]][k]))
              for r in rec for k in ("upper", "lower"))
    bad = sum(1 for r in rec for s in r["status"] if s != 0)
    return {"requests": n, "N": [r["N"] for r in base],
            "mix": "3D Gaussian random-field voxels on (2N-1)^3, correlation length 0.05, vf 0.4, contrast 100, "
                   "N in {41,63,113}",
            "rtol": rtol, "hbm_budget_bytes": budget,
            "sequential_fp64": {"wall_s": round(t_seq, 3), "req_per_s": round(n / t_seq, 2),
                                "p50_s": round(serve.percentile(seq_t, 50), 4),
                                "p99_s": round(serve.percentile(seq_t, 99), 4)},
            "batched_fp32_capacity": {"wall_s": round(st0["wall_s"], 3), "req_per_s": round(capacity, 2),
                                      "Mpoint_iter_per_s": round(st0["Mpoint_iter_per_s"], 1),
                                      "peak_hbm_bytes": st0["peak_hbm_bytes"],
                                      "deferred_requests": st0["deferred_requests"]},
            "batched_fp32_poisson": {"rate_req_per_s": round(rate, 2), "wall_s": round(st["wall_s"], 3),
                                     "p50_s": round(serve.percentile(lat, 50), 4),
                                     "p99_s": round(serve.percentile(lat, 99), 4),
                                     "peak_hbm_bytes": st["peak_hbm_bytes"],
                                     "deferred_requests": st["deferred_requests"]},
            "throughput_speedup_vs_sequential_fp64": round(capacity / (n / t_seq), 2),
            "max_bound_rel_diff_vs_fp64": err, "solves_not_converged": bad}


if __name__ == "__main__":
    main()
