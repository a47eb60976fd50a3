"""Write the oracle's FP64 Ga bounds for the benchmark configurations.

Calls only ``oracle`` (and the ``synth`` input generators); nothing here comes
from the HIP path.  Each case is stored as ``tests/golden/<name>.json``:

    python tests/golden/make_golden.py c1 c2_41 c2_365 c2_1013 c3 c5

Cases (unit cell, inputs from ``synth``):
* c1      -- 2D, N = 41, centred square of side 0.6, phases 1 / 10, tol 1e-10
* c2_<N>  -- 2D, centred disc of volume fraction 0.3, phases 1 / 100, tol 1e-10
* c3      -- 3D, N = 63, centred cube of side 0.5, matrix I, inclusion
             Q diag(lambda) Q^T with seed 3, tol 1e-10
* c5      -- 3D, N = 113, 225^3-voxel Gaussian random field (seed 5,
             correlation length 0.05) thresholded at volume fraction 0.4,
             phases 1 / 100, tol 1e-10 (the benchmark workload)
* serve_mix -- the eight requests of synth.serving_requests(21, 8, ...) with
             N drawn from {21, 41, 123}: random non-overlapping discs, contrast
             log-uniform in [10, 1e4], tol 1e-10 (one list of results)
* stall     -- requests 11, 64 and 469 of synth.serving_requests(4, 512, ...)
             (random discs at contrast ~9.6e3, N = 41, 63, 41), tol 1e-10: the
             FP32-iteration form stalls on them below a relative residual of
             ~1e-7 (one list of results)
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import ga, material  # noqa: E402


def case(name):
    if name == "c1":
        return synth.square_inclusion(2, 0.6, 1.0, 10.0), (41, 41), 1e-10
    if name.startswith("c2_"):
        n = int(name[3:])
        return synth.circle_inclusion_vf(0.3, 1.0, 100.0), (n, n), 1e-10
    if name == "c3":
        return synth.cube_inclusion_aniso(0.5, 3), (63, 63, 63), 1e-10
    if name == "c5":
        micro = synth.grf_voxels(5, (225, 225, 225), d=3, corr_len=0.05, vf=0.4, a_matrix=1.0, a_incl=100.0)
        return micro, (113, 113, 113), 1e-10
    raise ValueError(name)


SERVE_MIX = dict(seed=21, n=8, N_choices=(21, 41, 123))


def serve_mix():
    reqs = synth.serving_requests(SERVE_MIX["seed"], SERVE_MIX["n"], rate_per_s=1e6,
                                  N_choices=SERVE_MIX["N_choices"])
    t0 = time.time()
    rows = []
    for r in reqs:
        N = (int(r["N"]),) * 2
        res = ga.ga_bounds(material.make_material(r["micro"]), N, tol=1e-10, maxit=20000)
        rows.append({"id": r["id"], "N": list(N), "upper": res["upper"].tolist(), "lower": res["lower"].tolist(),
                     "iters_primal": res["iters_primal"], "iters_dual": res["iters_dual"]})
    out = {"case": "serve_mix", "requests": SERVE_MIX["seed"], "n": SERVE_MIX["n"],
           "N_choices": list(SERVE_MIX["N_choices"]), "tol": 1e-10, "results": rows,
           "oracle_seconds": time.time() - t0}
    with open(os.path.join(HERE, "serve_mix.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("serve_mix done in %.1f s" % out["oracle_seconds"], flush=True)


STALL = dict(seed=4, n=512, ids=(11, 64, 469))


def stall():
    reqs = synth.serving_requests(STALL["seed"], STALL["n"], rate_per_s=1.0)
    t0 = time.time()
    rows = []
    for rid in STALL["ids"]:
        r = reqs[rid]
        N = (int(r["N"]),) * 2
        res = ga.ga_bounds(material.make_material(r["micro"]), N, tol=1e-10, maxit=20000)
        rows.append({"id": rid, "N": list(N), "upper": res["upper"].tolist(), "lower": res["lower"].tolist(),
                     "iters_primal": res["iters_primal"], "iters_dual": res["iters_dual"]})
    out = {"case": "stall", "requests": STALL["seed"], "n": STALL["n"], "tol": 1e-10, "results": rows,
           "oracle_seconds": time.time() - t0}
    with open(os.path.join(HERE, "stall.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("stall done in %.1f s" % out["oracle_seconds"], flush=True)


def main(names):
    for name in names:
        if name == "serve_mix":
            serve_mix()
            continue
        if name == "stall":
            stall()
            continue
        micro, N, tol = case(name)
        t0 = time.time()
        res = ga.ga_bounds(material.make_material(micro), N, tol=tol, maxit=20000)
        out = {
            "case": name, "N": list(N), "tol": tol,
            "upper": res["upper"].tolist(), "lower": res["lower"].tolist(),
            "gram_A": res["gram_A"].tolist(), "gram_B": res["gram_B"].tolist(),
            "iters_primal": res["iters_primal"], "iters_dual": res["iters_dual"],
            "oracle_seconds": time.time() - t0,
        }
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(out, f, indent=1)
        print(name, "done in %.1f s" % out["oracle_seconds"], flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
