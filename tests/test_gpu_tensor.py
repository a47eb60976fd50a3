"""GPU parity of matrix-valued materials (plans made with FFTGAL_TENSOR).

Matrix voxel images (eq. gridcomp with a symmetric positive definite C^p per
voxel: seeded Voronoi polycrystals, one rotated anisotropic conductivity per
grain) and inclusion sets with their own anisotropic A_i per inclusion in an
anisotropic matrix (eq. inclcomp): every entry of the bounds against the
oracle's, converged (1e-10 of the norm) and after a fixed number of CG steps
(first order in the operator, 1e-11), including cases whose row pass and
expand/project passes run at specialised lengths (81, 125).
"""

import numpy as np
import pytest

import synth
from oracle import ga, material

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1412_2033_amd import fftgal
    fftgal.load_library()
    return fftgal


CASES = {
    "poly2d_N13": (lambda: synth.polycrystal(1, (25, 25), d=2, n_grains=6), (13, 13)),
    "poly2d_N9x41": (lambda: synth.polycrystal(2, (15, 81), d=2, n_grains=5), (9, 41)),
    "poly2d_N63x9": (lambda: synth.polycrystal(3, (125, 15), d=2, n_grains=5), (63, 9)),
    "poly3d_N7": (lambda: synth.polycrystal(4, (15, 15, 15), d=3, n_grains=6), (7, 7, 7)),
    "poly3d_N5x5x63": (lambda: synth.polycrystal(5, (9, 9, 125), d=3, n_grains=4), (5, 5, 63)),
    "multi2d_N21x15": (lambda: synth.multiphase_aniso(6, d=2, n=3), (21, 15)),
    "multi3d_N9x7x9": (lambda: synth.multiphase_aniso(7, d=3, n=3), (9, 7, 9)),
    "multi3d_N41x5x5": (lambda: synth.multiphase_aniso(8, d=3, n=2), (41, 5, 5)),
    "multi3d_N5x5x41": (lambda: synth.multiphase_aniso(9, d=3, n=3), (5, 5, 41)),
}


def _gpu(fg, micro, N, precision="fp64", rtol=1e-10, maxit=20000, device_image=False):
    import torch
    print("tensor case N=%s %s" % (N, precision), flush=True)
    if device_image:
        micro = dict(micro)
        micro["image"] = torch.from_numpy(np.ascontiguousarray(micro["image"])).to("cuda:0")
    plan = fg.Plan(len(N), N, precision, P=micro.get("P"), tensor=True)
    try:
        return plan.run(micro, rtol=rtol, maxit=maxit)
    finally:
        plan.close()


def _entries(res, ref, tol):
    for key in ("upper", "lower"):
        b = np.asarray(ref[key])
        err = np.max(np.abs(np.asarray(res[key]) - b)) / np.linalg.norm(b)
        assert err < tol, (key, err)


@pytest.mark.parametrize("name", sorted(CASES))
def test_tensor_fp64_matches_oracle(fg, name):
    make, N = CASES[name]
    micro = make()
    res = _gpu(fg, micro, N)
    ref = ga.ga_bounds(material.make_material(micro), N, tol=1e-10)
    _entries(res, ref, 1e-10)
    assert np.min(np.linalg.eigvalsh(np.asarray(res["upper"]) - np.asarray(res["lower"]))) > 0
    # genuinely anisotropic: off-diagonal entries well above rounding
    up = np.asarray(res["upper"])
    assert np.max(np.abs(up - np.diag(np.diag(up)))) > 1e-4 * np.max(np.abs(up))


@pytest.mark.parametrize("name", ["poly2d_N9x41", "poly3d_N5x5x63", "multi3d_N41x5x5", "multi2d_N21x15"])
def test_tensor_truncated_entries_match_oracle(fg, name):
    make, N = CASES[name]
    micro = make()
    res = _gpu(fg, micro, N, rtol=0.0, maxit=10)
    ref = ga.ga_bounds(material.make_material(micro), N, tol=0.0, maxit=10)
    _entries(res, ref, 1e-11)


@pytest.mark.parametrize("name", ["poly2d_N13", "poly3d_N7", "multi3d_N9x7x9", "poly2d_N9x41"])
def test_tensor_fp32_form(fg, name):
    make, N = CASES[name]
    micro = make()
    res = _gpu(fg, micro, N, "fp32", rtol=5e-6)
    ref = ga.ga_bounds(material.make_material(micro), N, tol=1e-10)
    _entries(res, ref, 1e-6)
    assert np.min(np.linalg.eigvalsh(np.asarray(res["upper"]) - np.asarray(res["lower"]))) > 0


def test_tensor_device_image_equals_host_image(fg):
    make, N = CASES["poly3d_N7"]
    micro = make()
    a = _gpu(fg, micro, N)
    b = _gpu(fg, micro, N, device_image=True)
    assert np.array_equal(a["upper"], b["upper"]) and np.array_equal(a["lower"], b["lower"])


def test_isotropic_tensor_image_equals_scalar_image(fg):
    scal = synth.grf_voxels(21, (25, 25), d=2, corr_len=0.1)
    tens = dict(scal)
    tens["image"] = scal["image"][..., None, None] * np.eye(2)
    N = (13, 13)
    a = _gpu(fg, tens, N)
    plan = fg.Plan(2, N, "fp64", P=scal["P"])
    b = plan.run(scal, rtol=1e-10)
    plan.close()
    for key in ("upper", "lower"):
        assert np.max(np.abs(a[key] - b[key])) <= 1e-12 * np.max(np.abs(b[key]))


def test_tensor_errors(fg):
    poly = synth.polycrystal(1, (9, 9), d=2, n_grains=3)
    multi = synth.multiphase_aniso(6, d=2, n=3)
    plan = fg.Plan(2, (5, 5), "fp64", P=(9, 9))
    try:
        for micro in (poly, multi):
            with pytest.raises(fg.FftgalError) as e:
                plan.set_material(micro)  # needs FFTGAL_TENSOR
            assert e.value.code == -1 and "FFTGAL_TENSOR" in str(e.value)
    finally:
        plan.close()
    bad = dict(poly)
    img = poly["image"].copy()
    img[3, 4] = np.array([[1.0, 2.0], [2.0, 1.0]])  # indefinite
    img[0, 0, 0, 1] += 0.5  # not symmetric
    bad["image"] = img
    plan = fg.Plan(2, (5, 5), "fp64", P=(9, 9), tensor=True)
    try:
        with pytest.raises(fg.FftgalError) as e:
            plan.set_material(bad)
        assert e.value.code == -1 and "2 voxels" in str(e.value)
    finally:
        plan.close()
    with pytest.raises(fg.FftgalError):
        fg.Plan(2, (5, 5), "fp64", scheme="gani", tensor=True)
