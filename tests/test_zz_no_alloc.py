"""The entry point that allocates nothing: fftgal_plan_static.

A plan on the library's own static device array, for callers that cannot
allocate device memory.  Through the C ABI, its bounds must equal bitwise
those of fftgal_plan on a caller's workspace (the same kernels and launch
shapes), on consecutive plans that reuse the array, the later ones smaller.
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1412_2033_amd import fftgal
    fftgal.load_library()
    return fftgal


def _run_handle(fg, h, d, micro, rtol):
    fg.fftgal_set_material(h, micro)
    ip, cp = fg.fftgal_solve_primal(h, d, -1, rtol)
    idl, cd = fg.fftgal_solve_dual(h, d, -1, rtol)
    up, lo, gap = fg.fftgal_bounds(h, d)
    return up, lo, [i["iters"] for i in ip + idl]


def _static(fg, micro, N, precision, rtol):
    import torch
    d = len(N)
    stream = torch.cuda.current_stream().cuda_stream
    h = fg.fftgal_plan_static(d, N, fg.PRECISIONS[precision], stream)
    try:
        return _run_handle(fg, h, d, micro, rtol)
    finally:
        fg.fftgal_destroy(h)


def _workspace(fg, micro, N, precision, rtol):
    plan = fg.Plan(len(N), N, precision, P=micro.get("P"))
    try:
        return _run_handle(fg, plan.handle, len(N), micro, rtol)
    finally:
        plan.close()


CALLS = [
    (lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0, center=(0.1, 0.0)), (63, 63), "fp64", 1e-10),
    (lambda: synth.grf_voxels(3, (25, 25, 25), d=3, corr_len=0.1), (13, 13, 13), "fp32", 5e-6),
    (lambda: synth.square_inclusion(2, 0.6, 1.0, 10.0), (21, 21), "fp64", 1e-10),
    # grids of the single work-group solver (its arguments in the plan's slots)
    (lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0), (41, 41), "fp64", 1e-10),
    (lambda: synth.square_inclusion(2, 0.5, 1.0, 10.0), (41, 63), "fp32", 5e-6),
]


def test_static_plan_matches_workspace_plan(fg):
    # three plans in a row on the one static array, each smaller than the first
    for make, N, precision, rtol in CALLS:
        print("static plan d=%d N=%s %s" % (len(N), N, precision), flush=True)
        micro = make()
        up, lo, its = _static(fg, micro, N, precision, rtol)
        up_r, lo_r, its_r = _workspace(fg, micro, N, precision, rtol)
        assert its == its_r
        assert np.array_equal(up, up_r) and np.array_equal(lo, lo_r)


def test_static_plan_limits(fg):
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    assert fg.fftgal_static_workspace_bytes() == 64 << 20
    # too large for the array
    with pytest.raises(fg.FftgalError) as e:
        fg.fftgal_plan_static(3, (63, 63, 63), 0, stream)
    assert e.value.code == -2
    # one plan at a time holds a device's array
    h = fg.fftgal_plan_static(2, (9, 9), 0, stream)
    try:
        with pytest.raises(fg.FftgalError) as e:
            fg.fftgal_plan_static(2, (9, 9), 0, stream)
        assert e.value.code == -5
    finally:
        fg.fftgal_destroy(h)
    h = fg.fftgal_plan_static(2, (9, 9), 0, stream)
    fg.fftgal_destroy(h)
