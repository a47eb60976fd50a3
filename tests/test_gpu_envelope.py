"""GPU parity of the upper-upper / lower-lower bounds (Lemma bounds_bounds,
Remark adjusting_A).

* fftgal_envelope_images: the upper and lower voxel images of an inclusion
  description equal the oracle's (same voxel classification; the phase
  eigenvalues agree to rounding), 2D and 3D, boxes, discs, anisotropic phases,
  non-cubic voxel grids, a P that is not a multiple of anything in sight;
* a voxel material with image / image_dual = upper / lower gives the oracle's
  bounds of that envelope material within 1e-10 (FP64; 1e-6 FP32 iterations),
  and those bracket the Ga bounds of the exact inclusion material.
"""

import numpy as np
import pytest

import synth
from oracle import envelope, ga, material

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


def _twophase():
    return {"d": 2, "kind": "inclusions", "A0": np.eye(2), "shapes": ["rect", "circ"],
            "centers": np.array([[0.1, -0.2], [-0.25, 0.2]]), "sizes": np.array([[0.35, 0.2], [0.12, 0.0]]),
            "A_in": np.array([12 * np.eye(2), 0.2 * np.eye(2)])}


IMAGE_CASES = {
    "circle2d_P45": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0, center=(0.03, -0.07)), (45, 45)),
    "twophase2d_P25x16": (_twophase, (25, 16)),
    "aligned_box2d_P9": (lambda: synth.square_inclusion(2, 1.0 / 3.0, 1.0, 10.0), (9, 9)),
    "aniso3d_P9x7x11": (lambda: synth.cube_inclusion_aniso(0.45, 5), (9, 7, 11)),
    "aniso3d_P64": (lambda: synth.cube_inclusion_aniso(0.5, 6), (64, 64, 64)),
}


@pytest.mark.parametrize("name", sorted(IMAGE_CASES))
def test_images_match_oracle(fg, name):
    make, P = IMAGE_CASES[name]
    micro = make()
    d = len(P)
    print("envelope images %s P=%s" % (name, P), flush=True)
    plan = fg.Plan(d, (3,) * d, "fp64")
    try:
        up, lo = plan.envelope_images(micro, P)
        up, lo = up.cpu().numpy(), lo.cpu().numpy()
    finally:
        plan.close()
    rup, rlo = envelope.images(micro, P)
    np.testing.assert_allclose(up, rup, rtol=1e-14, atol=0)
    np.testing.assert_allclose(lo, rlo, rtol=1e-14, atol=0)


BOUND_CASES = {
    # name: (micro, P, N, precision)
    "circle2d_P45_N15": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0), (45, 45), (15, 15), "fp64"),
    "twophase2d_P75_N25": (_twophase, (75, 75), (25, 25), "fp64"),
    "aniso3d_P15_N7": (lambda: synth.cube_inclusion_aniso(0.45, 5), (15, 15, 15), (7, 7, 7), "fp64"),
    "circle2d_P135_N41_fp32": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 30.0), (135, 135), (41, 41), "fp32"),
}


@pytest.mark.parametrize("name", sorted(BOUND_CASES))
def test_envelope_bounds_match_oracle_and_bracket(fg, name):
    make, P, N, prec = BOUND_CASES[name]
    micro = make()
    d = len(N)
    print("envelope bounds %s P=%s N=%s %s" % (name, P, N, prec), flush=True)
    plan = fg.Plan(d, N, prec, P=P)
    try:
        up, lo = plan.envelope_images(micro, P)
        vox = {"d": d, "kind": "voxels", "P": P, "image": up, "image_dual": lo}
        res = plan.run(vox, rtol=1e-11 if prec == "fp64" else 1e-5)
    finally:
        plan.close()
    env = envelope.envelope_micro(micro, P)
    ref = ga.ga_bounds(material.make_material(env), N, tol=1e-11)
    tol = 1e-10 if prec == "fp64" else 1e-6
    assert _rel(res["upper"], ref["upper"]) <= tol
    assert _rel(res["lower"], ref["lower"]) <= tol
    exact = ga.ga_bounds(material.make_material(micro), N, tol=1e-11)
    scale = np.abs(exact["upper"]).max()
    assert np.min(np.linalg.eigvalsh(res["upper"] - exact["upper"])) >= -tol * scale
    assert np.min(np.linalg.eigvalsh(exact["lower"] - res["lower"])) >= -tol * scale


def test_dual_image_host_arrays(fg):
    # host images take the staging path; image_dual on its own (lower image)
    micro = synth.circle_inclusion_vf(0.3, 1.0, 100.0)
    P, N = (45, 45), (15, 15)
    up, lo = envelope.images(micro, P)
    plan = fg.Plan(2, N, "fp64", P=P)
    try:
        res = plan.run({"d": 2, "kind": "voxels", "P": P, "image": up, "image_dual": lo}, rtol=1e-11)
    finally:
        plan.close()
    ref = ga.ga_bounds(material.make_material(envelope.envelope_micro(micro, P)), N, tol=1e-11)
    assert _rel(res["upper"], ref["upper"]) <= 1e-10
    assert _rel(res["lower"], ref["lower"]) <= 1e-10


def test_envelope_errors(fg):
    plan = fg.Plan(2, (5, 5), "fp64", P=(9, 9))
    try:
        with pytest.raises(fg.FftgalError):
            plan.envelope_images(synth.grf_voxels(1, (9, 9), d=2), (9, 9))  # not inclusions
        bad = synth.circle_inclusion_vf(0.3, 1.0, 100.0)
        bad["A_in"] = np.array([-np.eye(2)])
        with pytest.raises(fg.FftgalError):
            plan.envelope_images(bad, (9, 9))  # not SPD
        with pytest.raises(fg.FftgalError):
            plan.envelope_images(synth.circle_inclusion_vf(0.3, 1.0, 100.0), (0, 9))
        up, lo = plan.envelope_images(synth.circle_inclusion_vf(0.3, 1.0, 100.0), (9, 9))
        with pytest.raises(ValueError):
            plan.set_material({"d": 2, "kind": "voxels", "P": (9, 9), "image": up, "image_dual": lo.cpu().numpy()})
    finally:
        plan.close()
