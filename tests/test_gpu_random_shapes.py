"""First-order GPU parity on seeded random shapes: orders, materials and plan
options drawn at random, compared entry by entry with the oracle.

Each case draws d, an odd order per axis (small enough for the oracle), a
material (isotropic square or disc inclusions, an anisotropic cube, a scalar
voxel image at a voxel resolution P that may differ from the double grid and
need not be 3,5,7-smooth, multi-phase anisotropic inclusions or a matrix
voxel image) and the plan flags (concurrent solves, matrix fields, the
per-pass kernels for small 2D grids, the double grid of specialised lengths).  Every primal and dual solve stops
after K conjugate-gradient steps (rtol 0), so the bounds are first order in
the operator (Remark CG: the iterate is a fixed Krylov polynomial), and each
entry must match the oracle's bounds of the same iterates (Prop.
struct_bounds) to 1e-11 of the reference norm.  The draws cover the generic
transform kernels at many odd lengths, Bluestein lengths of the voxel setup
and ragged batches of every pass.  The FP32-iteration form runs the same
draws at low contrast (at most 10, where FP32 rounding of two CG steps stays
far below the tolerance) and after K32 steps must match the FP64 run of the
same steps to 1e-7.  Draws with scalar materials also run as reduced-Ga plans
(Lemma reduce_grid; first order against the oracle's reduced Ga) and as GaNi
plans (Def. GaNi; converged, against the oracle's GaNi, and lower = upper for
odd N by Remark duality_gani).
"""

import numpy as np
import pytest

import synth
from oracle import ga, gani, material, reduced

K = 6
K32 = 2
N2 = (1, 3, 5, 7, 9, 11, 13, 15, 17, 19, 21, 25, 27, 31)
N3 = (1, 3, 5, 7, 9, 11)
KINDS2 = ("square", "disc", "aniso", "vox", "multi", "poly")
KINDS3 = ("square", "aniso", "vox", "multi", "poly")


def _draw(seed, low_contrast=False):
    rng = np.random.Generator(np.random.PCG64(seed))
    d = 2 if rng.random() < 0.55 else 3
    N = tuple(int(rng.choice(N2 if d == 2 else N3)) for _ in range(d))
    if max(N) < 3:  # at least one axis with a nonzero frequency
        N = (3,) + N[1:]
    kind = str(rng.choice(KINDS2 if d == 2 else KINDS3))
    M = tuple(2 * n - 1 for n in N)
    c = float(10.0 ** rng.uniform(0.5, 2.5))
    if low_contrast:
        c = 1.0 + c % 9.0
    if kind == "square":
        micro = synth.square_inclusion(d, float(rng.uniform(0.2, 0.7)), 1.0, c,
                                       center=rng.uniform(-0.2, 0.2, size=d))
    elif kind == "disc":
        micro = synth.circle_inclusion_vf(float(rng.uniform(0.1, 0.5)), 1.0, c,
                                          center=rng.uniform(-0.2, 0.2, size=2))
    elif kind == "aniso":
        sd = int(rng.integers(1, 1000))
        micro = synth.cube_inclusion_aniso(float(rng.uniform(0.3, 0.6)), sd, d=d)
        if low_contrast:
            micro["A_in"] = synth.random_spd(sd, d, 0.0, 1.0).reshape(1, d, d)
    elif kind == "vox":
        P = tuple(int(m if rng.random() < 0.5 else 2 * rng.integers(2, m + 2) + 1) for m in M)
        micro = synth.grf_voxels(int(rng.integers(1, 1000)), P, d=d, corr_len=0.15,
                                 vf=float(rng.uniform(0.2, 0.6)), a_matrix=1.0, a_incl=c)
    elif kind == "multi":
        hi = 1.0 if low_contrast else 2.0
        micro = synth.multiphase_aniso(int(rng.integers(1, 1000)), d=d, n=int(rng.integers(1, 4)), log10_hi=hi)
    else:
        P = tuple(int(2 * rng.integers(2, m + 2) + 1) for m in M)
        hi = 1.0 if low_contrast else 2.0
        micro = synth.polycrystal(int(rng.integers(1, 1000)), P, d=d, n_grains=int(rng.integers(2, 7)),
                                  log10_hi=hi)
    opts = {"concurrent": bool(rng.random() < 0.4)}
    if kind in ("multi", "poly"):
        opts["tensor"] = True
    if d == 2 and rng.random() < 0.3:
        opts["separate_passes"] = True
    if rng.random() < 0.35:
        opts["fast_grid"] = True  # the specialised double grid (same bounds)
    return N, kind, micro, opts


SEEDS = list(range(101, 131))


@pytest.fixture(scope="module")
def fg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1412_2033_amd import fftgal
    fftgal.load_library()
    return fftgal


@pytest.mark.gpu
@pytest.mark.parametrize("seed", SEEDS)
def test_random_shape_truncated_matches_oracle(fg, seed):
    N, kind, micro, opts = _draw(seed)
    print("random case seed=%d N=%s %s %s" % (seed, N, kind, opts), flush=True)
    plan = fg.Plan(len(N), N, "fp64", P=micro.get("P"), **opts)
    try:
        res = plan.run(micro, rtol=0.0, maxit=K)
    finally:
        plan.close()
    ref = ga.ga_bounds(material.make_material(micro), N, tol=0.0, maxit=K)
    assert [i["iters"] for i in res["info_primal"]] == ref["iters_primal"]
    assert [i["iters"] for i in res["info_dual"]] == ref["iters_dual"]
    for key in ("upper", "lower"):
        a = np.asarray(res[key])
        b = np.asarray(ref[key])
        err = np.max(np.abs(a - b)) / np.linalg.norm(b)
        print("  %s: max entry error %.2e of |ref|" % (key, err))
        assert err < 1e-11, (key, err, a, b)


def _run(fg, micro, N, precision, k, opts):
    plan = fg.Plan(len(N), N, precision, P=micro.get("P"), **opts)
    try:
        return plan.run(micro, rtol=0.0, maxit=k)
    finally:
        plan.close()


@pytest.mark.gpu
@pytest.mark.parametrize("seed", SEEDS)
def test_random_shape_fp32_matches_fp64(fg, seed):
    N, kind, micro, opts = _draw(seed, low_contrast=True)
    print("random fp32 case seed=%d N=%s %s %s" % (seed, N, kind, opts), flush=True)
    r64 = _run(fg, micro, N, "fp64", K32, opts)
    r32 = _run(fg, micro, N, "fp32", K32, opts)
    assert [i["iters"] for i in r32["info_primal"] + r32["info_dual"]] == \
        [i["iters"] for i in r64["info_primal"] + r64["info_dual"]]
    for key in ("upper", "lower"):
        a = np.asarray(r32[key])
        b = np.asarray(r64[key])
        err = np.max(np.abs(a - b)) / np.linalg.norm(b)
        print("  %s: max entry error %.2e of |fp64|" % (key, err))
        assert err < 1e-7, (key, err, a, b)


def _draw_scalar(seed):
    # the reduced Ga and GaNi plans: scalar materials (inclusions with one
    # matrix each are reduced to the two-phase / isotropic classes by the
    # draw), orders >= 3 on every axis, no matrix-field or concurrent flags
    N, kind, micro, opts = _draw(seed)
    N = tuple(max(n, 3) for n in N)
    if kind in ("multi", "poly"):
        M = tuple(2 * n - 1 for n in N)
        micro = synth.grf_voxels(seed, M, d=len(N), corr_len=0.15, vf=0.4, a_matrix=1.0, a_incl=30.0)
        kind = "vox"
    return N, kind, micro


@pytest.mark.gpu
@pytest.mark.parametrize("seed", SEEDS[:15])
def test_random_shape_reduced_truncated_matches_oracle(fg, seed):
    # Lemma reduce_grid: the operator on the N-grid with 2^d shifted
    # transforms (Bluestein at the orders that are not 3,5,7-smooth)
    N, kind, micro = _draw_scalar(seed)
    print("random reduced case seed=%d N=%s %s" % (seed, N, kind), flush=True)
    plan = fg.Plan(len(N), N, "fp64", P=micro.get("P"), scheme="reduced")
    try:
        res = plan.run(micro, rtol=0.0, maxit=K)
    finally:
        plan.close()
    ref = reduced.reduced_bounds(material.make_material(micro), N, tol=0.0, maxit=K)
    for key in ("upper", "lower"):
        b = np.asarray(ref[key])
        err = np.max(np.abs(np.asarray(res[key]) - b)) / np.linalg.norm(b)
        print("  %s: max entry error %.2e of |ref|" % (key, err))
        assert err < 1e-11, (key, err)


@pytest.mark.gpu
@pytest.mark.parametrize("seed", SEEDS[15:])
def test_random_shape_gani_matches_oracle(fg, seed):
    # Def. GaNi (material sampled on the grid of the order N), converged;
    # duality of the two GaNi values for odd N (Remark duality_gani)
    N, kind, micro = _draw_scalar(seed)
    print("random gani case seed=%d N=%s %s" % (seed, N, kind), flush=True)
    plan = fg.Plan(len(N), N, "fp64", P=micro.get("P"), scheme="gani")
    try:
        res = plan.run(micro, rtol=1e-11)
    finally:
        plan.close()
    ref = gani.gani(micro, N, tol=1e-11)
    up = np.asarray(res["upper"])
    lo = np.asarray(res["lower"])
    assert np.linalg.norm(up - ref["A_gani"]) <= 1e-10 * np.linalg.norm(ref["A_gani"])
    Bi = np.linalg.inv(ref["B_gani"])
    assert np.linalg.norm(lo - Bi) <= 1e-10 * np.linalg.norm(Bi)
    assert np.linalg.norm(lo - up) <= 1e-9 * np.linalg.norm(up)


def test_draws_cover_the_options():
    # the seeded draws exercise every material kind, both dimensions and every flag
    draws = [_draw(s) for s in SEEDS]
    kinds = {k for _, k, _, _ in draws}
    assert kinds == set(KINDS2)
    assert {len(N) for N, _, _, _ in draws} == {2, 3}
    assert any(o["concurrent"] for _, _, _, o in draws)
    assert any(o.get("separate_passes") for _, _, _, o in draws)
    assert sum(bool(o.get("fast_grid")) for _, _, _, o in draws) >= 5
    assert any(m.get("P") is not None and tuple(m["P"]) != tuple(2 * n - 1 for n in N)
               for N, _, m, _ in draws)
