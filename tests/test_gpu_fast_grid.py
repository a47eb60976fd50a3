"""GPU tests of FFTGAL_FAST_GRID: Ga plans on the double grid with specialised
kernels instead of the smallest 3,5,7-smooth one.

The double-grid quadrature is exact for every M >= 2N - 1 (Lemma
integ_eval_VM), so a plan on the larger grid must give the bounds of the
default grid: converged, to 1e-10 (FP64; the FP32-iteration form to 1e-6), and
after a fixed number of CG steps entry by entry against the oracle (which
integrates on M = 2N - 1) to 1e-11, first order in the operator.  The grids
taken are those the flag documents: 2D N = 21 on 81^2 (the single work-group
solver), 2D N = 201 on 729^2, 3D (35, 3, 151) on 81 x 5 x 729 (the middle
axis keeps its short generic length), 3D N = 81 on 225^3 and 3D N = 21 on 81^3 (a small
grid).
"""

import numpy as np
import pytest

import synth
from oracle import ga, material

pytestmark = pytest.mark.gpu

K = 6


@pytest.fixture(scope="module")
def fg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1412_2033_amd import fftgal
    fftgal.load_library()
    return fftgal


CASES = {
    "disc2d_N21": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0, center=(0.05, -0.1)), (21, 21), (81, 81)),
    "circles2d_N201": (lambda: synth.random_circles(3, contrast=50.0), (201, 201), (729, 729)),
    "aniso3d_N35x3x151": (lambda: synth.cube_inclusion_aniso(0.45, 6), (35, 3, 151), (81, 5, 729)),
    "vox3d_N81": (lambda: synth.grf_voxels(5, (161, 161, 161), d=3, corr_len=0.05, vf=0.4, a_incl=100.0),
                  (81, 81, 81), (225, 225, 225)),
    # 5.8 times the points of 45^3, taken because the grid is small
    "vox3d_N21": (lambda: synth.grf_voxels(7, (41, 41, 41), d=3, corr_len=0.1, vf=0.4, a_incl=30.0),
                  (21, 21, 21), (81, 81, 81)),
}


def _run(fg, micro, N, precision, fast, **kw):
    print("fast grid case N=%s %s fast=%s %s" % (N, precision, fast, kw), flush=True)
    plan = fg.Plan(len(N), N, precision, P=micro.get("P"), fast_grid=fast)
    try:
        res = plan.run(micro, **kw)
        res["M"] = plan.M
    finally:
        plan.close()
    return res


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("name", sorted(CASES))
def test_fast_grid_gives_the_default_bounds(fg, name):
    make, N, Mfast = CASES[name]
    micro = make()
    a = _run(fg, micro, N, "fp64", False, rtol=1e-11)
    b = _run(fg, micro, N, "fp64", True, rtol=1e-11)
    assert tuple(b["M"]) == Mfast and tuple(a["M"]) != Mfast
    for key in ("upper", "lower"):
        assert _rel(b[key], a[key]) < 1e-10, (key, _rel(b[key], a[key]))
    c = _run(fg, micro, N, "fp32", True, rtol=5e-6)
    assert tuple(c["M"]) == Mfast
    for key in ("upper", "lower"):
        assert _rel(c[key], a[key]) < 1e-6, (key, _rel(c[key], a[key]))


@pytest.mark.parametrize("name", ["disc2d_N21", "aniso3d_N35x3x151"])
def test_fast_grid_truncated_matches_oracle(fg, name):
    make, N, Mfast = CASES[name]
    micro = make()
    res = _run(fg, micro, N, "fp64", True, rtol=0.0, maxit=K)
    assert tuple(res["M"]) == Mfast
    ref = ga.ga_bounds(material.make_material(micro), N, tol=0.0, maxit=K)
    for key in ("upper", "lower"):
        err = _rel(res[key], ref[key])
        print("  %s: max entry error %.2e of |ref|" % (key, err))
        assert err < 1e-11, (key, err)


def test_fast_grid_refused_by_other_schemes(fg):
    with pytest.raises(fg.FftgalError):
        fg.Plan(2, (21, 21), "fp64", scheme="gani", fast_grid=True)
