"""GPU parity of the reduced Ga plans (Lemma reduce_grid, Algorithm 3).

* fftgal_plan_reduced: bounds within 1e-10 of the oracle's reduced Ga (FP64;
  1e-6 for the FP32-iteration form), which the oracle pins to the Ga bounds;
  2D/3D, inclusions and voxels, non-cubic grids, generic and specialised
  transform lengths;
* a homogeneous material needs no iteration and is exact; the monitored
  energy starts at the Voigt entry;
* the reduced plan and the double-grid plan of the same N give the same bounds
  on the device (3D, N = 81: specialised reduced kernels against the generic
  length-175 double grid); the lean layout (shifts in turn) and the default
  one (the shifts of a pass in one launch) agree;
* orders that are not 3,5,7-smooth (the primes 41, 113, 1013 of the
  benchmark configurations) run Bluestein transforms: parity with the oracle
  (converged and after 10 steps, entry by entry), and at N = 113 on the 225^3
  benchmark image equality with the double grid;
* unsupported uses raise: an even N, warm starts, batches.
"""

import numpy as np
import pytest

import synth
from oracle import material, reduced

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1412_2033_amd import fftgal
    fftgal.load_library()
    return fftgal


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


CASES = {
    "circle2d_N9": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0, center=(0.05, -0.1)), (9, 9)),
    "square2d_N15x25": (lambda: synth.square_inclusion(2, 0.6, 1.0, 10.0, center=(0.1, 0.2)), (15, 25)),
    "twophase_iso_N15": (lambda: {"d": 2, "kind": "inclusions", "A0": np.eye(2), "shapes": ["rect", "circ"],
                                  "centers": np.array([[0.1, -0.2], [-0.25, 0.2]]),
                                  "sizes": np.array([[0.35, 0.2], [0.12, 0.0]]),
                                  "A_in": np.array([12 * np.eye(2), 0.2 * np.eye(2)])}, (15, 15)),
    "aniso3d_N5": (lambda: synth.cube_inclusion_aniso(0.5, 3), (5, 5, 5)),
    "voxel2d_P15_N9": (lambda: synth.grf_voxels(11, (15, 15), d=2, corr_len=0.15), (9, 9)),
    "voxel3d_P9_N5x7x3": (lambda: synth.grf_voxels(12, (9, 9, 9), d=3, corr_len=0.15), (5, 7, 3)),
    # specialised transform lengths
    "circle2d_N81": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0), (81, 81)),
    "circle2d_N225x125": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 30.0, center=(0.2, 0.1)), (225, 125)),
    # orders that are not 3,5,7-smooth (Bluestein transforms): the benchmark
    # orders 41 and 113 and 1013 (on the row axis, where the energy Gram pass
    # packs two components per transform), and short non-smooth lengths
    "circle2d_N41": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0), (41, 41)),
    "voxel3d_P225_N113x5x5": (lambda: synth.grf_voxels(14, (225, 9, 9), d=3, corr_len=0.1), (113, 5, 5)),
    "circle2d_N5x1013": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0, center=(0.1, 0.05)), (5, 1013)),
    "square2d_N11x13": (lambda: synth.square_inclusion(2, 0.6, 1.0, 10.0, center=(0.1, 0.2)), (11, 13)),
    "aniso3d_N7x11x13": (lambda: synth.cube_inclusion_aniso(0.45, 4), (7, 11, 13)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_reduced_matches_oracle(fg, name):
    make, N = CASES[name]
    micro = make()
    d = len(N)
    print("reduced %s N=%s" % (name, N), flush=True)
    plan = fg.Plan(d, N, "fp64", P=micro.get("P"), scheme="reduced")
    try:
        res = plan.run(micro, rtol=1e-11)
    finally:
        plan.close()
    ref = reduced.reduced_bounds(material.make_material(micro), N, tol=1e-11)
    assert _rel(res["upper"], ref["upper"]) <= 1e-10
    assert _rel(res["lower"], ref["lower"]) <= 1e-10


def test_reduced_fp32_iterations(fg):
    micro = synth.circle_inclusion_vf(0.3, 1.0, 100.0)
    N = (81, 81)
    print("reduced fp32 N=81", flush=True)
    plan = fg.Plan(2, N, "fp32", scheme="reduced")
    try:
        res = plan.run(micro, rtol=1e-5)
    finally:
        plan.close()
    ref = reduced.reduced_bounds(material.make_material(micro), N, tol=1e-11)
    assert _rel(res["upper"], ref["upper"]) <= 1e-6
    assert _rel(res["lower"], ref["lower"]) <= 1e-6


def test_reduced_fp32_3d_against_double_grid(fg):
    # the FP32-iteration form of the reduced plan (shifts of a pass in one
    # launch, 3D, N = 81) within 1e-6 of the FP64 double-grid bounds
    N = (81, 81, 81)
    micro = synth.cube_inclusion_aniso(0.45, 5)
    print("reduced fp32 3D N=81", flush=True)
    red = fg.Plan(3, N, "fp32", scheme="reduced")
    try:
        r = red.run(micro, rtol=5e-6)
    finally:
        red.close()
    ga = fg.Plan(3, N, "fp64")
    try:
        g = ga.run(micro, rtol=1e-10)
    finally:
        ga.close()
    assert _rel(r["upper"], g["upper"]) <= 1e-6
    assert _rel(r["lower"], g["lower"]) <= 1e-6
    assert np.min(np.linalg.eigvalsh(np.asarray(r["upper"]) - np.asarray(r["lower"]))) > 0


@pytest.mark.parametrize("kind", ["inclusions", "voxels"])
def test_reduced_equals_double_grid_3d(fg, kind):
    N = (81, 81, 81)
    micro = synth.cube_inclusion_aniso(0.45, 5) if kind == "inclusions" else \
        synth.grf_voxels(5, (81, 81, 81), d=3, corr_len=0.05)
    print("reduced vs double grid 3D N=81 %s" % kind, flush=True)
    red = fg.Plan(3, N, "fp64", P=micro.get("P"), scheme="reduced")
    try:
        r = red.run(micro, rtol=1e-11)
    finally:
        red.close()
    ga = fg.Plan(3, N, "fp64", P=micro.get("P"))
    try:
        g = ga.run(micro, rtol=1e-11)
    finally:
        ga.close()
    assert _rel(r["upper"], g["upper"]) <= 1e-10
    assert _rel(r["lower"], g["lower"]) <= 1e-10


@pytest.mark.parametrize("d, N", [(2, (81, 81)), (3, (81, 81, 81))])
def test_reduced_lean_equals_grouped(fg, d, N):
    # the lean layout (shifts in turn, one set of intermediates, q accumulated)
    # and the default one (shifts of a pass in one launch, q summed by the
    # update) give the same bounds; the lean workspace is the smaller
    micro = synth.circle_inclusion_vf(0.3, 1.0, 100.0) if d == 2 else synth.cube_inclusion_aniso(0.45, 5)
    print("reduced lean vs grouped d=%d N=%s" % (d, N), flush=True)
    res = {}
    nbytes = {}
    for lean in (False, True):
        plan = fg.Plan(d, N, "fp64", scheme="reduced", lean=lean)
        try:
            res[lean] = plan.run(micro, rtol=1e-11)
            nbytes[lean] = plan.nbytes
        finally:
            plan.close()
    assert nbytes[True] < nbytes[False]
    assert _rel(res[True]["upper"], res[False]["upper"]) <= 1e-10
    assert _rel(res[True]["lower"], res[False]["lower"]) <= 1e-10


def test_reduced_homogeneous_and_history(fg):
    # a homogeneous material has a zero right-hand side (no iteration, exact
    # A); the first monitored energy of a non-trivial solve is the Voigt entry
    from oracle import ga
    A = synth.random_spd(7, 3)
    micro = synth.cube_inclusion_aniso(0.5, 7)
    micro["A0"] = A
    micro["A_in"] = A.reshape(1, 3, 3).copy()
    plan = fg.Plan(3, (5, 7, 5), "fp64", scheme="reduced")
    try:
        res = plan.run(micro, rtol=1e-12)
    finally:
        plan.close()
    np.testing.assert_allclose(res["upper"], A, rtol=1e-13, atol=1e-13 * np.abs(A).max())
    np.testing.assert_allclose(res["lower"], A, rtol=1e-13, atol=1e-13 * np.abs(A).max())
    assert all(i["iters"] == 0 for i in res["info_primal"] + res["info_dual"])
    micro = synth.circle_inclusion_vf(0.3, 1.0, 100.0)
    plan = fg.Plan(2, (15, 15), "fp64", scheme="reduced")
    try:
        plan.run(micro, rtol=1e-10)
        h0 = [plan.history(0, a)[0] for a in range(2)]
    finally:
        plan.close()
    voigt, _ = ga.voigt_reuss(material.make_material(micro), 2)
    for a in range(2):
        assert abs(h0[a] - voigt[a, a]) <= 1e-12 * voigt[a, a]


@pytest.mark.parametrize("name", ["circle2d_N41", "voxel3d_P225_N113x5x5", "circle2d_N5x1013"])
def test_reduced_truncated_entries_match_oracle(fg, name):
    # first order in the operator (10 CG steps, rtol 0): each bound entry
    # against the oracle's reduced Ga of the same iterates (Bluestein lengths)
    make, N = CASES[name]
    micro = make()
    print("reduced truncated %s N=%s" % (name, N), flush=True)
    plan = fg.Plan(len(N), N, "fp64", P=micro.get("P"), scheme="reduced")
    try:
        res = plan.run(micro, rtol=0.0, maxit=10)
    finally:
        plan.close()
    ref = reduced.reduced_bounds(material.make_material(micro), N, tol=0.0, maxit=10)
    for key in ("upper", "lower"):
        b = np.asarray(ref[key])
        assert np.max(np.abs(np.asarray(res[key]) - b)) / np.linalg.norm(b) < 1e-11, key


def test_reduced_equals_double_grid_benchmark_order(fg):
    # the benchmark workload's order N = 113 (a prime: transforms of length 113
    # by Bluestein's convolution of length 225) on its 225^3 random-field
    # image: the reduced plan gives the double-grid plan's bounds
    import torch
    N = (113, 113, 113)
    micro = synth.grf_voxels(5, (225, 225, 225), d=3, corr_len=0.05, vf=0.4, a_matrix=1.0, a_incl=100.0)
    micro["image"] = torch.from_numpy(np.ascontiguousarray(micro["image"])).to("cuda:0")
    print("reduced vs double grid 3D N=113", flush=True)
    red = fg.Plan(3, N, "fp64", P=micro["P"], scheme="reduced")
    try:
        r = red.run(micro, rtol=1e-11)
    finally:
        red.close()
    ga = fg.Plan(3, N, "fp64", P=micro["P"])
    try:
        g = ga.run(micro, rtol=1e-11)
    finally:
        ga.close()
    assert _rel(r["upper"], g["upper"]) <= 1e-10
    assert _rel(r["lower"], g["lower"]) <= 1e-10


def test_reduced_errors(fg):
    with pytest.raises(fg.FftgalError):
        fg.Plan(2, (10, 11), "fp64", scheme="reduced")  # N must be odd
    micro = synth.square_inclusion(2, 0.6, 1.0, 10.0)
    a = fg.Plan(2, (5, 5), "fp64")
    b = fg.Plan(2, (9, 9), "fp64", scheme="reduced")
    try:
        a.run(micro, rtol=1e-10)
        b.set_material(micro)
        with pytest.raises(fg.FftgalError):
            b.warm_start(a)
        batch = fg.Batch(capacity=2, stream=b.stream)
        try:
            with pytest.raises(fg.FftgalError):
                batch.add(b, 0, 0)
        finally:
            batch.close()
    finally:
        a.close()
        b.close()
