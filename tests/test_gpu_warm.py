"""GPU parity of the bound monitoring and the coarse-to-fine warm start (Sec. 6.4).

* fftgal_history: the energies of the CG iterates, from the CG scalars the
  device records, against the oracle's exact quadrature of every iterate
  (FP64, same iteration path up to rounding; compared on the common prefix);
  energy[0] is the Voigt entry (cold start), and the sequence never increases.
* fftgal_warm_start: the first energy of a warm-started fine solve equals the
  coarse plan's bound entry (the prolonged field is the same trigonometric
  polynomial), and the final bounds equal the oracle's Ga bounds of the fine
  grid -- FP64 to 1e-10, FP32 iterations to 1e-6 -- for 2D and 3D, cubic and
  non-cubic grids, mixed precisions, and a grid that is coarser than the
  coarse one along an axis (truncation, still admissible).
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


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def test_history_matches_oracle_energies(fg):
    micro = synth.circle_inclusion_vf(0.3, 1.0, 200.0, center=(0.05, -0.1))
    N = (15, 15)
    print("history circle2d N=15", flush=True)
    plan = fg.Plan(2, N, "fp64")
    try:
        plan.run(micro, rtol=1e-10)
        hist = {(k, a): plan.history(k, a) for k in (0, 1) for a in range(2)}
    finally:
        plan.close()
    mat = material.make_material(micro)
    ref = ga.ga_bounds(mat, N, tol=1e-10, track_energy=True)
    voigt, reuss = ga.voigt_reuss(mat, 2)
    for k, key in ((0, "primal"), (1, "dual")):
        for a in range(2):
            h = hist[(k, a)]
            e = np.array(ref["energies_" + key][a])
            n = min(len(h), len(e))
            assert n >= 10
            np.testing.assert_allclose(h[:n], e[:n], rtol=1e-9)
            assert np.all(np.diff(h) <= 1e-12 * h[0])
            start = voigt[a, a] if k == 0 else np.linalg.inv(reuss)[a, a]
            assert abs(h[0] - start) <= 1e-12 * start


WARM_CASES = {
    # name: (micro, coarse N, fine N, coarse precision, fine precision)
    "circle2d_9to41_fp64": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0), (9, 9), (41, 41), "fp64", "fp64"),
    "square2d_5x7to15x11": (lambda: synth.square_inclusion(2, 0.6, 1.0, 10.0, center=(0.1, 0.2)), (5, 7), (15, 11),
                            "fp64", "fp64"),
    "aniso3d_3to9_fp64": (lambda: synth.cube_inclusion_aniso(0.5, 3), (3, 3, 3), (9, 9, 9), "fp64", "fp64"),
    "voxel3d_5to7_fp32": (lambda: synth.grf_voxels(12, (9, 9, 9), d=3, corr_len=0.15), (5, 5, 5), (7, 7, 7),
                          "fp64", "fp32"),
    "circle2d_fp32to_fp64": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 30.0), (9, 9), (21, 21), "fp32", "fp64"),
    "truncating_axis": (lambda: synth.square_inclusion(2, 0.6, 1.0, 10.0), (9, 9), (15, 7), "fp64", "fp64"),
}


@pytest.mark.parametrize("name", sorted(WARM_CASES))
def test_warm_start_matches_oracle(fg, name):
    make, Nc, N, pc, pf = WARM_CASES[name]
    micro = make()
    d = len(N)
    P = micro.get("P")
    print("warm %s coarse %s %s -> fine %s %s" % (name, Nc, pc, N, pf), flush=True)
    rt = {"fp64": 1e-10, "fp32": 1e-5}
    coarse = fg.Plan(d, Nc, pc, P=P)
    fine = fg.Plan(d, N, pf, P=P)
    try:
        rc = coarse.run(micro, rtol=rt[pc])
        res = fine.run(micro, rtol=rt[pf], warm_from=coarse)
        first = {(k, a): fine.history(k, a)[0] for k in (0, 1) for a in range(d)}
    finally:
        coarse.close()
        fine.close()
    ref = ga.ga_bounds(material.make_material(micro), N, tol=1e-10)
    tol = 1e-10 if pf == "fp64" else 1e-6
    assert _rel(res["upper"], ref["upper"]) <= tol
    assert _rel(res["lower"], ref["lower"]) <= tol
    assert np.min(np.linalg.eigvalsh(res["upper"] - res["lower"])) >= -1e-12 * np.abs(res["upper"]).max()
    if all(n >= m for n, m in zip(N, Nc)):
        # exact transfer: the warm iterate's energy is the coarse plan's bound
        # entry (primal: upper; dual: the dual Gram entry, inverse of lower);
        # an FP32 fine plan rounds the field and evaluates r_0 in FP32
        cB = np.linalg.inv(rc["lower"])
        etol = 1e-11 if pf == "fp64" else 1e-5
        for a in range(d):
            assert abs(first[(0, a)] - rc["upper"][a, a]) <= etol * rc["upper"][a, a]
            assert abs(first[(1, a)] - cB[a, a]) <= etol * cB[a, a]


def test_warm_start_errors(fg):
    micro = synth.square_inclusion(2, 0.6, 1.0, 10.0)
    a = fg.Plan(2, (5, 5), "fp64")
    b = fg.Plan(2, (9, 9), "fp64")
    c = fg.Plan(3, (3, 3, 3), "fp64")
    try:
        with pytest.raises(fg.FftgalError) as e:
            b.warm_start(a)  # no material on the fine plan
        assert e.value.code == -5
        b.set_material(micro)
        a.set_material(micro)
        with pytest.raises(fg.FftgalError) as e:
            b.warm_start(a)  # nothing solved on the coarse plan
        assert e.value.code == -5
        c.set_material(synth.cube_inclusion_aniso(0.5, 3))
        c.solve_primal(0)
        with pytest.raises(fg.FftgalError) as e:
            b.warm_start(c)  # different d
        assert e.value.code == -1
        with pytest.raises(fg.FftgalError) as e:
            b.history(0, 0)  # nothing solved on b
        assert e.value.code == -5
    finally:
        a.close()
        b.close()
        c.close()


@pytest.mark.parametrize("btol", [1e-4, 1e-7])
def test_bound_tolerance_matches_oracle(fg, btol):
    # the bound test stops CG early on the device; each bound entry must equal
    # the oracle's exact energy of its iterate with the same number of steps,
    # and stay on the guaranteed side of the converged Ga bounds
    micro = synth.circle_inclusion_vf(0.3, 1.0, 200.0, center=(0.05, -0.1))
    N = (41, 41)
    print("bound tolerance %g circle2d N=41" % btol, flush=True)
    plan = fg.Plan(2, N, "fp64")
    try:
        plan.set_bound_tol(btol)
        res = plan.run(micro, rtol=1e-12)
    finally:
        plan.close()
    from bound_rule import first_stop
    mat = material.make_material(micro)
    ref = ga.ga_bounds(mat, N, tol=1e-12, track_energy=True)
    gB = np.linalg.inv(res["lower"])
    for a in range(2):
        kp = res["info_primal"][a]["iters"]
        kd = res["info_dual"][a]["iters"]
        # the stopping iteration is where the documented rule first holds on the
        # oracle's exact energies (the device applies it to the CG recurrence,
        # equal up to rounding, so a decision at the threshold may move by one)
        op = first_stop(ref["energies_primal"][a], btol)
        od = first_stop(ref["energies_dual"][a], btol)
        assert kp < ref["iters_primal"][a] and abs(kp - op) <= 1
        assert kd < ref["iters_dual"][a] and abs(kd - od) <= 1
        assert abs(res["upper"][a, a] - ref["energies_primal"][a][kp]) <= 1e-9 * res["upper"][a, a]
        assert abs(gB[a, a] - ref["energies_dual"][a][kd]) <= 1e-9 * gB[a, a]
        assert res["upper"][a, a] >= ref["upper"][a, a] * (1 - 1e-12)
        assert res["lower"][a, a] <= ref["lower"][a, a] * (1 + 1e-12)
