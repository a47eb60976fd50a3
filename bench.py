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
of all six solves, divided by the step time.

    python bench.py [--gpus 1] [--steps 2] [--warmup 1] [--precision fp64|fp32]
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
KERNEL_SYMBOL = {"row": "row_kernel", "expand": "pencil_kernel", "pencil_inv": "pencil_kernel",
                 "pencil_fwd": "pencil_kernel", "project": "pencil_kernel", "cg_update": "cg_update_kernel"}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("fftgal_kernels.hip", "fftgal_internal.h"):
        with open(os.path.join(ROOT, "paper_1412_2033_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(cls, precision):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when no summary exists for this kernel or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    sym = "%s<%s>" % (KERNEL_SYMBOL.get(cls, cls), "double" if precision == "fp64" else "float")
    r = rec.get(sym)
    if r is None or r.get("class") != cls or r.get("precision") != precision:
        return None
    if r.get("source_sha256_16") != kernel_source_hash():
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


def cpu_baseline(micro, N, d):
    """The oracle, as it stands, on a bounded sample: one CG iteration at full size."""
    import numpy as np
    from oracle import ga, material
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
    return {"value": pts / it_s / 1e6, "unit": "Mpoint*CG-iter/s", "cores": 1, "kind": "oracle",
            "sample": "1 oracle CG iteration (Algorithm 2 matvec, FP64, numpy.fft single-threaded, "
                      "primal, d=3, M=225) after building A_M (%.1f s); %.2f s per iteration" % (setup_s, it_s)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--rtol", type=float, default=None)
    ap.add_argument("--N", type=int, default=113)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes 5 times (profiler counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the path shards by independent solves/requests; "
              "see the design notes); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        src = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": src.numel() * 4, "launches": 5}))
        return

    import synth
    from paper_1412_2033_amd import fftgal

    d = 3
    N = (args.N,) * d
    M = tuple(2 * n - 1 for n in N)
    rtol = args.rtol if args.rtol is not None else 1e-8
    print("bench: building workload d=3 N=%d M=%d (%s)" % (N[0], M[0], args.precision), file=sys.stderr, flush=True)
    micro = synth.grf_voxels(5, M, d=3, corr_len=0.05, vf=0.4, a_matrix=1.0, a_incl=100.0)
    dev = torch.device("cuda:0")
    micro_dev = dict(micro)
    micro_dev["image"] = torch.from_numpy(np.ascontiguousarray(micro["image"])).to(dev)
    plan = fftgal.Plan(d, N, args.precision, device=dev, P=M)
    es = 16 if args.precision == "fp64" else 8
    gs = 8 if args.precision == "fp64" else 4

    for w in range(args.warmup):
        res = plan.run(micro_dev, rtol=rtol)
        print("bench: warmup %d done, iters %s / %s" % (w, [i["iters"] for i in res["info_primal"]],
                                                        [i["iters"] for i in res["info_dual"]]),
              file=sys.stderr, flush=True)
    plan.set_timing(True)
    plan.read_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for k in range(args.steps):
        res = plan.run(micro_dev, rtol=rtol)
        results.append(res)
        print("bench: step %d done" % k, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timing = plan.read_timing()
    plan.set_timing(False)

    ms_per_step = 1e3 * elapsed / args.steps
    pts = M[0] * M[1] * M[2]
    iters_p = [sum(i["iters"] for i in r["info_primal"]) for r in results]
    iters_d = [sum(i["iters"] for i in r["info_dual"]) for r in results]
    total_iters = sum(iters_p) + sum(iters_d)
    value = pts * total_iters / elapsed / 1e6

    # dominant kernel and its roofline (algorithmic bytes / measured duration)
    nc_p, nc_d = 1, d - 1
    per_cls = {}
    for cls, (ms, cnt) in timing.items():
        if cnt == 0:
            continue
        by = algorithmic_bytes(cls, d, N, M, es, gs, nc_p) * sum(iters_p) + \
            algorithmic_bytes(cls, d, N, M, es, gs, nc_d) * sum(iters_d)
        per_cls[cls] = {"ms": round(ms, 3), "launches": cnt, "avg_us": round(1e3 * ms / cnt, 2),
                        "GBs": round(by / (ms * 1e-3) / 1e9, 1) if by > 0 else None}
    dom = max((c for c in per_cls if per_cls[c]["GBs"]), key=lambda c: per_cls[c]["ms"])
    work_launches = total_iters
    dom_bytes = (algorithmic_bytes(dom, d, N, M, es, gs, nc_p) * sum(iters_p) +
                 algorithmic_bytes(dom, d, N, M, es, gs, nc_d) * sum(iters_d)) / work_launches
    dom_avg_s = timing[dom][0] * 1e-3 / timing[dom][1]
    achieved = dom_bytes / dom_avg_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom, args.precision), "kernel": dom,
                "bytes_per_launch": int(dom_bytes), "avg_launch_us": round(dom_avg_s * 1e6, 2)}

    last = results[-1]
    out = {
        "metric": "Mpoint*CG-iter/s (time-to-bounds at d=3,N=113)",
        "value": round(value, 2),
        "unit": "Mpoint*CG-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "3D two-phase GRF voxel composite (corr. length 0.05, vf 0.4, contrast 1:100), "
                               "Ga primal+dual CG to rel. residual %g, bounds in FP64" % rtol,
                   "d": d, "N": N[0], "M": M[0], "P": M[0], "precision": args.precision},
        "time_to_bounds_s": round(ms_per_step / 1e3, 4),
        "cg_iterations": {"primal": [i["iters"] for i in last["info_primal"]],
                          "dual": [i["iters"] for i in last["info_dual"]]},
        "upper_diag": [round(float(v), 10) for v in np.diag(last["upper"])],
        "lower_diag": [round(float(v), 10) for v in np.diag(last["lower"])],
        "gap": last["gap"],
        "kernels": per_cls,
        "roofline": roofline,
    }
    plan.close()
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(micro, N, d)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
