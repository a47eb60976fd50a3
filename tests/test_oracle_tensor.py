"""Pins of the oracle's matrix-valued materials.

* Voxel images with a symmetric positive definite matrix per voxel (eq.
  gridcomp with C^p in R^{d x d}; Lemma grid_compos applied entry by entry)
  and inclusion composites with a different anisotropic A_i per inclusion
  (eq. inclcomp, eq. inclcomp_formula).
* An isotropic matrix image C^p = c^p I has exactly the coefficients and
  bounds of the scalar image c^p.
* A matrix image whose voxels resolve axis-aligned boxes exactly equals the
  inclusion composite of those boxes: the voxel route (DFT of the image times
  the sinc window) and the closed-form route (eq. char_func_Four, pinned
  against quadrature elsewhere) are independent computations of the same
  Fourier coefficients.
* Route O1 (dense Lemma FD_matrix_full) equals route O2 (Algorithm 2 + CG)
  for both material classes.
* A homogeneous matrix image gives A_H = A exactly; the bounds of a random
  polycrystal satisfy Reuss <= lower <= upper <= Voigt and tighten with N.
"""

import numpy as np
import pytest

import synth
from oracle import dense, ga, grids, material


def _loewner_ge(a, b, tol=1e-12):
    return np.min(np.linalg.eigvalsh(a - b)) >= -tol * np.max(np.abs(a))


def _coeffs(mat, N):
    k = grids.freq_grid([2 * n - 1 for n in N])
    return mat.coeff_A(k), mat.coeff_B(k)


@pytest.mark.parametrize("d, P", [(2, (15, 9)), (3, (9, 7, 5))])
def test_isotropic_tensor_image_equals_scalar_image(d, P):
    rng = np.random.default_rng(1 + d)
    c = 10.0 ** rng.uniform(0, 2, size=P)
    scal = {"d": d, "kind": "voxels", "P": P, "image": c}
    tens = {"d": d, "kind": "voxels", "P": P, "image": c[..., None, None] * np.eye(d)}
    ms, mt = material.make_material(scal), material.make_material(tens)
    N = tuple(max(3, p // 2 | 1) for p in P)
    for a, b in zip(_coeffs(ms, N), _coeffs(mt, N)):
        assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(a))
    bs = ga.ga_bounds(ms, N, tol=1e-12)
    bt = ga.ga_bounds(mt, N, tol=1e-12)
    for key in ("upper", "lower"):
        assert np.max(np.abs(bs[key] - bt[key])) <= 1e-12 * np.max(np.abs(bs[key]))


def _aligned_boxes(d, P, seed):
    """Matrix phase A0 and two boxes whose faces lie on voxel faces, each with
    its own SPD matrix: the inclusion descriptor and the matching tensor image."""
    A0 = synth.random_spd(seed, d, 0.0, 0.5)
    A1 = synth.random_spd(seed + 1, d, 1.0, 2.0)
    A2 = synth.random_spd(seed + 2, d, -1.0, 0.0)
    # box b covers voxel indices lo_b .. hi_b (inclusive) along each axis
    spans = [[(1, 3)] * d, [(5, 6)] * d]
    spans[1][0] = (4, 7)
    centers, sizes = [], []
    img = np.empty(tuple(P) + (d, d))
    img[...] = A0
    for (span, A) in zip(spans, (A1, A2)):
        c = [0.5 * (lo + hi) / P[a] for a, (lo, hi) in enumerate(span)]
        h = [(hi - lo + 1) / P[a] for a, (lo, hi) in enumerate(span)]
        centers.append(c)
        sizes.append(h)
        idx = tuple(slice(lo, hi + 1) for lo, hi in span)
        img[idx] = A
    # voxel p sits at p / P for p < (P + 1) / 2 and at (p - P) / P otherwise:
    # the spans above lie in the first half, so storage index = p
    incl = {"d": d, "kind": "inclusions", "A0": A0, "shapes": ["rect", "rect"], "centers": np.array(centers),
            "sizes": np.array(sizes), "A_in": np.array([A1, A2])}
    vox = {"d": d, "kind": "voxels", "P": tuple(P), "image": img}
    return incl, vox


@pytest.mark.parametrize("d, P, N", [(2, (17, 19), (7, 9)), (3, (17, 17, 19), (5, 5, 7))])
def test_aligned_tensor_image_equals_inclusions(d, P, N):
    incl, vox = _aligned_boxes(d, P, 5 * d)
    mi, mv = material.make_material(incl), material.make_material(vox)
    for a, b in zip(_coeffs(mi, N), _coeffs(mv, N)):
        assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))
    bi = ga.ga_bounds(mi, N, tol=1e-12)
    bv = ga.ga_bounds(mv, N, tol=1e-12)
    for key in ("upper", "lower"):
        assert np.max(np.abs(bi[key] - bv[key])) <= 1e-11 * np.max(np.abs(bi[key]))


@pytest.mark.parametrize("case", ["poly2d", "poly3d", "multi2d", "multi3d"])
def test_dense_route_equals_fft_route(case):
    if case == "poly2d":
        micro, N = synth.polycrystal(3, (11, 13), d=2, n_grains=4), (5, 5)
    elif case == "poly3d":
        micro, N = synth.polycrystal(4, (7, 7, 9), d=3, n_grains=4), (3, 3, 5)
    elif case == "multi2d":
        micro, N = synth.multiphase_aniso(5, d=2, n=3), (7, 5)
    else:
        micro, N = synth.multiphase_aniso(6, d=3, n=3), (3, 5, 3)
    mat = material.make_material(micro)
    o1 = dense.dense_bounds(mat, N)
    o2 = ga.ga_bounds(mat, N, tol=1e-13)
    for key in ("upper", "lower"):
        assert np.max(np.abs(o1[key] - o2[key])) <= 1e-11 * np.max(np.abs(o1[key]))
    # the off-diagonal entries are not negligible: a genuinely anisotropic case
    assert np.max(np.abs(o2["upper"] - np.diag(np.diag(o2["upper"])))) > 1e-3 * np.max(np.abs(o2["upper"]))


@pytest.mark.parametrize("d", [2, 3])
def test_homogeneous_tensor_image_is_exact(d):
    A = synth.random_spd(9 + d, d)
    P = (5,) * d
    micro = {"d": d, "kind": "voxels", "P": P, "image": np.broadcast_to(A, P + (d, d)).copy()}
    res = ga.ga_bounds(material.make_material(micro), (3,) * d, tol=1e-12)
    assert res["iters_primal"] == [0] * d and res["iters_dual"] == [0] * d
    for key in ("upper", "lower"):
        assert np.max(np.abs(res[key] - A)) <= 1e-13 * np.max(np.abs(A))


def test_polycrystal_bounds_chain_and_refinement():
    micro = synth.polycrystal(8, (15, 15), d=2, n_grains=6, log10_lo=0.0, log10_hi=2.0)
    mat = material.make_material(micro)
    voigt, reuss = ga.voigt_reuss(mat, 2)
    prev = None
    for N in (3, 5, 9):
        res = ga.ga_bounds(mat, (N, N), tol=1e-12)
        up, lo = res["upper"], res["lower"]
        assert _loewner_ge(voigt, up) and _loewner_ge(up, lo) and _loewner_ge(lo, reuss)
        if prev is not None:
            assert _loewner_ge(prev[0], up, 1e-10) and _loewner_ge(lo, prev[1], 1e-10)
        prev = (up, lo)
