"""CPU checks of the C-ABI library: it loads and exports every declared symbol.

No compute call is made here (there is no GPU); only host-side size logic.
"""

import ctypes
import os
import re

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _declared():
    with open(os.path.join(ROOT, "include", "fftgal.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fftgal_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1412_2033_amd import fftgal
    if not os.path.exists(fftgal.LIB_PATH):
        pytest.fail("libfftgal.so not built: run __graft_entry__.build()")
    return fftgal.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "fftgal_plan" in names and "fftgal_bounds" in names
    for n in names:
        assert hasattr(lib, n), n


def test_workspace_bytes_validation(lib):
    from paper_1412_2033_amd import fftgal
    assert fftgal.fftgal_workspace_bytes(2, (41, 41)) > 0
    assert fftgal.fftgal_workspace_bytes(2, (40, 41)) == 0        # even N
    assert fftgal.fftgal_workspace_bytes(4, (5, 5, 5)) == 0        # d = 4
    assert fftgal.fftgal_workspace_bytes(2, (0, 5)) == 0
    assert fftgal.fftgal_workspace_bytes(2, (5, 5), precision=7) == 0
    assert fftgal.fftgal_workspace_bytes(2, (5, 5), P=(10, 9)) == 0  # P must be odd-smooth
    fp64 = fftgal.fftgal_workspace_bytes(3, (63, 63, 63), 0)
    fp32 = fftgal.fftgal_workspace_bytes(3, (63, 63, 63), 1)
    assert fp32 > fp64  # FP32 form keeps FP64 fields for the bounds plus FP32 copies
    big = fftgal.fftgal_workspace_bytes(3, (113, 113, 113), 0)
    assert 0.5e9 < big < 4e9
    # reduced Ga: the lean layout (one set of intermediates) is the smaller one;
    # the flag is refused by the other plan kinds
    grouped = fftgal.fftgal_workspace_bytes(3, (81, 81, 81), 0, scheme="reduced")
    lean = fftgal.fftgal_workspace_bytes(3, (81, 81, 81), fftgal.REDUCED_LEAN, scheme="reduced")
    assert 0 < lean < grouped
    assert fftgal.fftgal_workspace_bytes(3, (81, 81, 81), fftgal.REDUCED_LEAN) == 0
    assert fftgal.fftgal_workspace_bytes(3, (81, 81, 81), fftgal.REDUCED_LEAN, scheme="gani") == 0


def test_fast_grid_workspace(lib):
    # FFTGAL_FAST_GRID: specialised lengths on the axes whose smallest
    # 3,5,7-smooth length is at least 9, when the grid then holds at most
    # four times its points or at most 2^21 points (3D N = 81: 225^3 against
    # 175^3; 2D N = 21: 81^2 against 45^2; (35, 3, 151): 81 x 5 x 729 against
    # 75 x 5 x 315; 3D N = 21: 81^3 against 45^3, 5.8x but small); unchanged
    # where the smooth grid is already specialised (N = 41, 113), too short
    # (N = 3: 5 points) or the specialised one too large (3D N = 201: 729^3
    # against 405^3, 5.8x); Ga plans only
    from paper_1412_2033_amd import fftgal
    F = fftgal.FAST_GRID
    for d, N in ((3, (81, 81, 81)), (2, (21, 21)), (2, (201, 201)), (3, (35, 3, 151)), (3, (21, 21, 21))):
        assert fftgal.fftgal_workspace_bytes(d, N, F) > fftgal.fftgal_workspace_bytes(d, N, 0), N
    for d, N in ((2, (41, 41)), (3, (113, 113, 113)), (3, (201, 201, 201)), (2, (1013, 1013)), (2, (3, 3))):
        assert fftgal.fftgal_workspace_bytes(d, N, F) == fftgal.fftgal_workspace_bytes(d, N, 0), N
    # the same 225^3 intermediates as N = 113, a smaller CG state on Z_81
    assert fftgal.fftgal_workspace_bytes(3, (81, 81, 81), F) < fftgal.fftgal_workspace_bytes(3, (113, 113, 113), 0)
    assert fftgal.fftgal_workspace_bytes(2, (21, 21), F | 1) > 0
    assert fftgal.fftgal_workspace_bytes(2, (21, 21), F, scheme="gani") == 0
    assert fftgal.fftgal_workspace_bytes(2, (21, 21), F, scheme="reduced") == 0


def test_plan_rejects_bad_arguments_without_device(lib):
    h = ctypes.c_void_p()
    N = (ctypes.c_int32 * 3)(4, 5, 5)
    assert lib.fftgal_plan(ctypes.byref(h), 2, N, 0, None, 0, None) == -1
    assert b"odd" in lib.fftgal_last_error(None)
    N = (ctypes.c_int32 * 3)(5, 5, 5)
    assert lib.fftgal_plan(ctypes.byref(h), 2, N, 9, None, 0, None) == -1
    assert lib.fftgal_plan(None, 2, N, 0, None, 0, None) == -1
