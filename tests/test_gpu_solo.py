"""GPU parity of the single work-group 2D solver (small double grids: 81 x 81
in FP64, 81 or 125 on either axis in the FP32-iteration form).

One work-group runs the whole CG iteration of a solve: the operator of
Algorithm 2 on the complex M_1 x M_2 grid (both gradient components packed as
z = y_0 + i y_1), the projection, the CG update and the stopping test of
Remark CG.  Checked here:

* first order, entry by entry (truncated CG as in test_gpu_firstorder:
  every solve stopped after k = 10 steps, bounds against the oracle's bounds
  of the same iterates to 1e-11 of the reference norm) for isotropic discs,
  an anisotropic inclusion, a voxel image and a matrix-valued polycrystal;
* the FP32-iteration form after 2 steps against the FP64 run (1e-7) on
  every grid the solver takes;
* converged bounds against the oracle, and against the per-pass kernels
  (FFTGAL_SEPARATE_PASSES);
* the solver is the one that runs (no per-pass launch during the CG
  iterations), runs are deterministic, and a batch that mixes its solves
  with per-pass solves gives every solve the bounds it has alone.
"""

import numpy as np
import pytest

import synth
from oracle import ga, material

pytestmark = pytest.mark.gpu

K = 10


@pytest.fixture(scope="module")
def fg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1412_2033_amd import fftgal
    fftgal.load_library()
    return fftgal


def _disc(seed, contrast=300.0):
    return synth.random_circles(seed, k_lo=4, k_hi=8, r_lo=0.05, r_hi=0.12, contrast=contrast)


CASES = {
    "disc_41": (lambda: _disc(3), (41, 41)),
    "aniso_41": (lambda: synth.cube_inclusion_aniso(0.45, 7, d=2), (41, 41)),
    "vox_41": (lambda: synth.grf_voxels(5, (81, 81), d=2, corr_len=0.1, vf=0.4, a_matrix=1.0, a_incl=50.0),
               (41, 41)),
    "poly_41": (lambda: synth.polycrystal(6, (45, 81), d=2, n_grains=7), (41, 41)),
}
TENSOR = {"poly_41"}


def _run(fg, micro, N, precision="fp64", rtol=0.0, maxit=K, **kw):
    print("solo case N=%s %s maxit=%d %s" % (N, precision, maxit, kw), flush=True)
    plan = fg.Plan(2, N, precision, P=micro.get("P"), **kw)
    try:
        return plan.run(micro, rtol=rtol, maxit=maxit)
    finally:
        plan.close()


def _entries(res, ref, tol, what):
    for key in ("upper", "lower"):
        a = np.asarray(res[key])
        b = np.asarray(ref[key])
        err = np.max(np.abs(a - b)) / np.linalg.norm(b)
        print("%s %s: max entry error %.2e of |ref|" % (what, key, err))
        assert err < tol, (what, key, err)


@pytest.mark.parametrize("name", sorted(CASES))
def test_solo_truncated_entries_match_oracle(fg, name):
    make, N = CASES[name]
    micro = make()
    res = _run(fg, micro, N, tensor=name in TENSOR)
    ref = ga.ga_bounds(material.make_material(micro), N, tol=0.0, maxit=K)
    assert [i["iters"] for i in res["info_primal"]] == ref["iters_primal"]
    assert [i["iters"] for i in res["info_dual"]] == ref["iters_dual"]
    _entries(res, ref, 1e-11, name)


@pytest.mark.parametrize("N", [(41, 41), (63, 63), (41, 63), (63, 41)])
def test_solo_fp32_truncated_matches_fp64(fg, N):
    micro = _disc(sum(N), contrast=10.0)
    r64 = _run(fg, micro, N, "fp64", maxit=2, separate_passes=True)
    r32 = _run(fg, micro, N, "fp32", maxit=2)
    _entries(r32, r64, 1e-7, "fp32 N=%s" % (N,))


def test_solo_converged_matches_oracle_and_separate_passes(fg):
    micro = _disc(11)
    N = (41, 41)
    a = _run(fg, micro, N, rtol=1e-10, maxit=20000)
    ref = ga.ga_bounds(material.make_material(micro), N, tol=1e-10)
    _entries(a, ref, 1e-10, "converged vs oracle")
    b = _run(fg, micro, N, rtol=1e-10, maxit=20000, separate_passes=True)
    _entries(a, b, 1e-12, "solo vs separate passes")
    assert [i["iters"] for i in a["info_primal"] + a["info_dual"]] == \
        [i["iters"] for i in b["info_primal"] + b["info_dual"]]
    # FP32-iteration form on the 125-point grids: converged bounds near FP64
    N63 = (63, 63)
    micro63 = _disc(12, contrast=100.0)
    r32 = _run(fg, micro63, N63, "fp32", rtol=5e-6, maxit=20000)
    r64 = _run(fg, micro63, N63, "fp64", rtol=1e-10, maxit=20000)
    _entries(r32, r64, 1e-6, "fp32 converged N=63")
    assert np.min(np.linalg.eigvalsh(np.asarray(r32["upper"]) - np.asarray(r32["lower"]))) > 0


def test_solo_is_the_solver_that_runs_and_is_deterministic(fg):
    micro = _disc(13)
    N = (41, 41)
    plan = fg.Plan(2, N, "fp64")
    try:
        plan.set_material(micro)
        plan.set_timing(True)
        plan.read_timing()
        plan.solve_primal(-1, rtol=1e-10)
        t = plan.read_timing()
        assert t["solo"][1] >= 2 and t["expand"][1] == 0 and t["cg_update"][1] == 0, t
        plan.solve_primal(-1, rtol=1e-10)
        plan.solve_dual(-1, rtol=1e-10)
        a = plan.bounds()
        plan.solve_primal(-1, rtol=1e-10)
        plan.solve_dual(-1, rtol=1e-10)
        b = plan.bounds()
        for x, y in zip(a[:2], b[:2]):
            assert np.array_equal(np.asarray(x), np.asarray(y))
    finally:
        plan.close()
    # plans it does not take keep the per-pass kernels
    for N2, prec in (((63, 63), "fp64"), ((123, 41), "fp32")):
        plan = fg.Plan(2, N2, prec)
        try:
            plan.set_material(micro)
            plan.set_timing(True)
            plan.solve_primal(0, rtol=0.0, maxit=3)
            t = plan.read_timing()
            assert t["solo"][1] == 0 and t["expand"][1] == 3, (N2, prec, t)
        finally:
            plan.close()


def test_solo_in_a_mixed_batch_equals_alone(fg):
    import torch
    specs = [((41, 41), "fp64", _disc(21)), ((63, 63), "fp32", _disc(22, 30.0)),
             ((123, 123), "fp32", _disc(23, 30.0)), ((41, 41), "fp32", _disc(24, 30.0))]
    alone = [_run(fg, m, N, p, rtol=1e-8, maxit=3000) for N, p, m in specs]
    b = fg.Batch(32)
    plans = []
    try:
        for N, p, m in specs:
            pl = fg.Plan(2, N, p, stream=b.stream, concurrent=True)
            pl.set_material(m)
            plans.append(pl)
        ids = {}
        for j, pl in enumerate(plans):
            for kind in (0, 1):
                for alpha in range(2):
                    ids[b.add(pl, kind, alpha, 1e-8, 3000)] = j
        left = len(ids)
        while left:
            b.step(8)
            for sid, info, status in b.poll():
                assert status in (0, -4), status
                left -= 1
        for j, pl in enumerate(plans):
            up, lo, _ = pl.bounds()
            assert np.array_equal(np.asarray(up), np.asarray(alone[j]["upper"])), specs[j][:2]
            assert np.array_equal(np.asarray(lo), np.asarray(alone[j]["lower"])), specs[j][:2]
    finally:
        for pl in plans:
            pl.close()
        b.close()
        torch.cuda.synchronize()


def test_solo_history_and_bound_tolerance_match_separate_passes(fg):
    # the energy history (fftgal_history) and the bound-tolerance stop run
    # inside the solver: the same iterates' energies and stopping iterations
    # as the per-pass kernels, to rounding
    micro = synth.circle_inclusion_vf(0.3, 1.0, 200.0, center=(0.05, -0.1))
    N = (41, 41)
    out = {}
    for sep in (False, True):
        plan = fg.Plan(2, N, "fp64", separate_passes=sep)
        try:
            plan.run(micro, rtol=1e-10)
            hist = [plan.history(k, a) for k in (0, 1) for a in range(2)]
            plan.set_bound_tol(1e-6)
            res = plan.run(micro, rtol=1e-12)
            its = [i["iters"] for i in res["info_primal"] + res["info_dual"]]
            out[sep] = (hist, its, res)
        finally:
            plan.close()
    for h0, h1 in zip(out[False][0], out[True][0]):
        assert len(h0) == len(h1)
        np.testing.assert_allclose(h0, h1, rtol=1e-11)
    assert all(abs(a - b) <= 1 for a, b in zip(out[False][1], out[True][1]))
    ref = ga.ga_bounds(material.make_material(micro), N, tol=1e-12, track_energy=True)
    up = np.asarray(out[False][2]["upper"])
    for a in range(2):
        k = out[False][2]["info_primal"][a]["iters"]
        assert abs(up[a, a] - ref["energies_primal"][a][k]) <= 1e-9 * up[a, a]
