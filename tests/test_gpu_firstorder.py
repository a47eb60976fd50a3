"""First-order GPU parity: truncated conjugate gradients, compared entry by entry.

At a converged minimiser the bounds are second order in any defect of the
operator (Def. Ga: they are minimum energies), so a relative operator error
of 1e-6 changes converged bounds by ~1e-12 and passes a 1e-10 test.  After a
fixed number k of CG steps from e_0 = 0 the iterate is a fixed polynomial of
degree k in the operator applied to the right-hand side (Remark CG: Krylov
spaces), and its exact energy depends on the operator to first order.  So
every primal and dual solve here stops after exactly k iterations (rtol 0,
maxit k: the library reports ENOTCONV and still returns the guaranteed
bounds of those fields, Prop. struct_bounds), and each entry of the upper
and lower bound matrices is compared with the oracle's bounds of the same k
iterates, to 1e-11 of the Frobenius norm of the reference.

The cases put every transform length the library has specialised kernels for
(the double grids 81, 125, 225, 245, 729, 2025) on every role a length has in
the operator: axis 1 (the expand and project passes), axis 2 in 3D (the
strided pencil passes) and the last axis (the row pass with the material
multiply), with isotropic materials (inclusions and voxel images: the
isotropic row kernels) and anisotropic inclusions (the general row kernel).
With k = 10 an operator defect of 1e-5 at a single frequency index moves
these bounds by 3e-10 to 1e-7 (measured by planting it in a copy of the
oracle's transforms), far above the 1e-11 tolerance.

The FP32-iteration form is compared with the FP64 GPU run of the same
iterations, to 1e-7, after k = 2 steps on the same geometries at contrast
10: rounding errors of CG grow with the condition number (a single-precision
emulation of these solves moves a 10-step bound at contrast 1e3 by up to
~1e-3 with no defect at all), while after 2 steps at contrast 10 the same
emulation stays below 4e-9 and the residual is still a sizeable fraction of
the right-hand side, so the bounds respond to an operator defect at first
order.
"""

import numpy as np
import pytest

import synth
from oracle import ga, material

pytestmark = pytest.mark.gpu

K = 10  # CG iterations of every truncated FP64 solve
K32 = 2  # CG iterations of the FP32-against-FP64 comparison


@pytest.fixture(scope="module")
def fg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1412_2033_amd import fftgal
    fftgal.load_library()
    return fftgal


def _on_axis(n, axis, d, other=5):
    N = [other] * d
    N[axis] = n
    return tuple(N)


def _aniso(d, seed):
    return synth.cube_inclusion_aniso(0.45, seed, d=d)


def _disc(seed):
    m = synth.random_circles(seed, k_lo=4, k_hi=8, r_lo=0.05, r_hi=0.12, contrast=300.0)
    return m


def _voxels(d, N, seed):
    P = tuple(2 * n - 1 for n in N)
    return synth.grf_voxels(seed, P, d=d, corr_len=0.1, vf=0.4, a_matrix=1.0, a_incl=50.0)


def _cases():
    out = []
    # 3D: 81, 125, 225 on each axis; isotropic voxels and anisotropic inclusions
    for n in (41, 63, 113):
        for axis in range(3):
            N = _on_axis(n, axis, 3)
            out.append(("vox3d_%d_ax%d" % (n, axis), N, "voxels"))
            if n != 41:
                out.append(("aniso3d_%d_ax%d" % (n, axis), N, "aniso"))
    # 2D: all six lengths on both axes, isotropic discs; anisotropic inclusions
    # on the three longest
    for n in (41, 63, 113, 123, 365, 1013):
        for axis in range(2):
            N = _on_axis(n, axis, 2)
            out.append(("disc2d_%d_ax%d" % (n, axis), N, "disc"))
            if n in (123, 365, 1013):
                out.append(("aniso2d_%d_ax%d" % (n, axis), N, "aniso"))
    # two specialised lengths at once
    out.append(("disc2d_123x41", (123, 41), "disc"))
    out.append(("vox3d_41x63x5", (41, 63, 5), "voxels"))
    return out


CASES = {name: (N, kind) for name, N, kind in _cases()}


def _micro(name):
    N, kind = CASES[name]
    d = len(N)
    seed = sum(ord(c) for c in name)
    if kind == "aniso":
        return _aniso(d, seed % 97 + 3)
    if kind == "disc":
        return _disc(seed)
    return _voxels(d, N, seed)


def _micro32(name):
    # the same geometries at contrast 10: the FP32 comparison needs a problem
    # on which FP32 rounding itself stays far below the tolerance (CG rounding
    # errors grow with the condition number: at contrast 1e3 a truncated FP32
    # bound moves by up to ~1e-3 from FP64 with no defect at all)
    N, kind = CASES[name]
    d = len(N)
    seed = sum(ord(c) for c in name)
    if kind == "aniso":
        m = _aniso(d, seed % 97 + 3)
        m["A_in"] = synth.random_spd(seed % 97 + 3, d, 0.3, 1.0).reshape(1, d, d)
        return m
    if kind == "disc":
        return synth.random_circles(seed, k_lo=4, k_hi=8, r_lo=0.05, r_hi=0.12, contrast=10.0)
    P = tuple(2 * n - 1 for n in N)
    return synth.grf_voxels(seed, P, d=d, corr_len=0.1, vf=0.4, a_matrix=1.0, a_incl=10.0)


def _gpu_truncated(fg, micro, N, precision, k=K):
    print("case N=%s %s k=%d" % (N, precision, k), flush=True)
    plan = fg.Plan(len(N), N, precision, P=micro.get("P"))
    try:
        res = plan.run(micro, rtol=0.0, maxit=k)
    finally:
        plan.close()
    for info in res["info_primal"] + res["info_dual"]:
        # a solve whose right-hand side is at the rounding level stops at 0
        assert info["iters"] in (0, k), info
    return res


def _check_entries(res, ref, tol, what):
    for key in ("upper", "lower"):
        a = np.asarray(res[key])
        b = np.asarray(ref[key])
        scale = np.linalg.norm(b)
        err = np.max(np.abs(a - b)) / scale
        print("%s %s: max entry error %.2e of |ref|" % (what, key, err))
        assert err < tol, "%s %s: max entry error %.3e of |ref| (tol %.0e)\n%s\n%s" % (what, key, err, tol, a, b)


@pytest.mark.parametrize("name", sorted(CASES))
def test_truncated_fp64_entries_match_oracle(fg, name):
    N, _ = CASES[name]
    micro = _micro(name)
    res = _gpu_truncated(fg, micro, N, "fp64")
    ref = ga.ga_bounds(material.make_material(micro), N, tol=0.0, maxit=K)
    assert all(i == K or i == 0 for i in ref["iters_primal"] + ref["iters_dual"])
    assert [i["iters"] for i in res["info_primal"]] == ref["iters_primal"]
    assert [i["iters"] for i in res["info_dual"]] == ref["iters_dual"]
    _check_entries(res, ref, 1e-11, name)
    # the truncated iterates give guaranteed bounds too (every CG iterate is
    # admissible): lower <= upper
    assert np.min(np.linalg.eigvalsh(np.asarray(res["upper"]) - np.asarray(res["lower"]))) > 0


@pytest.mark.parametrize("name", sorted(CASES))
def test_truncated_fp32_entries_match_fp64(fg, name):
    N, _ = CASES[name]
    micro = _micro32(name)
    r64 = _gpu_truncated(fg, micro, N, "fp64", K32)
    r32 = _gpu_truncated(fg, micro, N, "fp32", K32)
    _check_entries(r32, r64, 1e-7, name + " fp32")
