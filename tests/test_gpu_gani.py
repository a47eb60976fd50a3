"""GPU parity of the GaNi plans and the a-posteriori guaranteed bounds.

* A GaNi plan (material sampled at the grid points, transforms of size N)
  returns A~_{H,N} and B~_{H,N}^{-1}: both within 1e-10 of the oracle (FP64;
  1e-6 for the FP32-iteration form) and equal to each other (Remark
  duality_gani, odd N).
* fftgal_bounds_of evaluates the exact energies of the GaNi minimisers on a Ga
  plan of the same N (eq. GaNi_apost): within 1e-10 of the oracle, and
  bracketing the Ga bounds of that N.
"""

import numpy as np
import pytest

import synth
from oracle import ga, gani, material

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
    "circle2d_N15": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0, center=(0.05, -0.1)), (15, 15)),
    "square2d_N9x25": (lambda: synth.square_inclusion(2, 0.6, 1.0, 10.0, center=(0.1, 0.2)), (9, 25)),
    "twophase_iso_N15": (lambda: {"d": 2, "kind": "inclusions", "A0": np.eye(2), "shapes": ["rect", "circ"],
                                  "centers": np.array([[0.1, -0.2], [-0.25, 0.2]]),
                                  "sizes": np.array([[0.35, 0.2], [0.12, 0.0]]),
                                  "A_in": np.array([12 * np.eye(2), 0.2 * np.eye(2)])}, (15, 15)),
    "aniso3d_N5": (lambda: synth.cube_inclusion_aniso(0.5, 3), (5, 5, 5)),
    "voxel3d_N9": (lambda: synth.grf_voxels(12, (9, 9, 9), d=3, corr_len=0.15), (9, 9, 9)),
    "voxel2d_P25_N15": (lambda: synth.grf_voxels(11, (25, 25), d=2, corr_len=0.15), (15, 15)),
    # grid sizes with specialised kernels
    "circle2d_N81": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0), (81, 81)),
    "circle2d_N225x125": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 30.0, center=(0.2, 0.1)), (225, 125)),
    "voxel3d_N25x15x9": (lambda: synth.grf_voxels(13, (25, 15, 9), d=3, corr_len=0.15), (25, 15, 9)),
    # orders that are not 3,5,7-smooth (Bluestein transforms): the paper's
    # order 99 = 9 * 11, and an image whose resolution is not smooth either
    "circle2d_N99": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0), (99, 99)),
    "voxel3d_P99x11x13_N99x11x13": (lambda: synth.grf_voxels(15, (99, 11, 13), d=3, corr_len=0.1,
                                                              a_matrix=0.029, a_incl=0.49), (99, 11, 13)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_gani_matches_oracle(fg, name):
    make, N = CASES[name]
    micro = make()
    d = len(N)
    P = micro.get("P")
    print("gani %s N=%s" % (name, N), flush=True)
    plan = fg.Plan(d, N, "fp64", P=P, scheme="gani")
    ga_plan = fg.Plan(d, N, "fp64", P=P)
    try:
        res = plan.run(micro, rtol=1e-11)
        ga_plan.set_material(micro)
        up_b, lo_b, _ = ga_plan.bounds_of(plan)
        ga_res = ga_plan.run(micro, rtol=1e-11)
    finally:
        plan.close()
        ga_plan.close()
    ref = gani.gani(micro, N, tol=1e-11)
    assert _rel(res["upper"], ref["A_gani"]) <= 1e-10
    assert _rel(res["lower"], np.linalg.inv(ref["B_gani"])) <= 1e-10
    assert _rel(res["lower"], res["upper"]) <= 1e-9  # duality for odd N
    ap = gani.apost_bounds(micro, ref)
    assert _rel(up_b, ap["upper"]) <= 1e-9
    assert _rel(lo_b, ap["lower"]) <= 1e-9
    scale = np.abs(ga_res["upper"]).max()
    assert np.min(np.linalg.eigvalsh(up_b - ga_res["upper"])) >= -1e-9 * scale
    assert np.min(np.linalg.eigvalsh(ga_res["lower"] - lo_b)) >= -1e-9 * scale


def test_gani_fp32_iterations(fg):
    micro = synth.circle_inclusion_vf(0.3, 1.0, 100.0)
    N = (81, 81)
    print("gani fp32 N=81", flush=True)
    plan = fg.Plan(2, N, "fp32", scheme="gani")
    try:
        res = plan.run(micro, rtol=1e-5)
    finally:
        plan.close()
    ref = gani.gani(micro, N, tol=1e-11)
    assert _rel(res["upper"], ref["A_gani"]) <= 1e-6
    assert _rel(res["lower"], np.linalg.inv(ref["B_gani"])) <= 1e-6


def test_gani_rejects_even_grid(fg):
    with pytest.raises(fg.FftgalError):
        fg.Plan(2, (10, 11), "fp64", scheme="gani")
