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


def main(names):
    for name in names:
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
