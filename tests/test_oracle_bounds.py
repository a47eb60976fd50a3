"""Pins for the oracle's Ga bounds against what the paper and mathematics fix.

* homogeneous material: A_{H,N} = B_{H,N}^{-1} = A exactly (the right-hand side
  of Cor. Ga_linsys vanishes);
* laminates: arithmetic mean along the layers (primal) and harmonic mean across
  them (dual) exactly at every N; for a(x_1) = a0 + a1 cos(2 pi x_1) the dual is
  exact for N >= 3 since its minimiser a/<a> - 1 is a trigonometric polynomial;
* discrete Keller identity in 2D: B_{H,N}[a] = R A_{H,N}[1/a] R^T (J_N = R E_N);
* route O1 (dense Lemma FD_matrix_full) equals route O2 (Algorithm 2 + CG);
* Prop. struct_bounds: Reuss <= lower <= upper <= Voigt (Loewner order);
* eq. subspace_hierarchy: bounds tighten monotonically in N;
* Remark CG / Sec. 6.4: the CG energy is non-increasing and starts at Voigt;
* invariance under translation, scaling, and the choice of M >= 2N-1.
"""

import math

import numpy as np
import pytest

import synth
from oracle import dense, ga, material

TOL = 1e-12


def _psd(m, tol):
    return np.min(np.linalg.eigvalsh(0.5 * (m + m.T))) >= -tol


def test_homogeneous_material_is_exact():
    A = synth.random_spd(7, 3)
    micro = synth.cube_inclusion_aniso(0.5, 7)
    micro["A0"] = A
    micro["A_in"] = A.reshape(1, 3, 3).copy()
    res = ga.ga_bounds(material.make_material(micro), (5, 5, 5), tol=TOL)
    np.testing.assert_allclose(res["upper"], A, rtol=1e-13, atol=1e-13 * np.abs(A).max())
    np.testing.assert_allclose(res["lower"], A, rtol=1e-13, atol=1e-13 * np.abs(A).max())
    assert res["iters_primal"] == [0, 0, 0] and res["iters_dual"] == [0, 0, 0]


@pytest.mark.parametrize("N", [5, 11, 21])
def test_step_laminate_exact_entries(N):
    a0, a1, w = 1.0, 10.0, 0.4
    micro = synth.square_inclusion(2, 1.0, a0, a1)
    micro["sizes"] = np.array([[w, 1.0]])  # layer |x_1| < w/2, all x_2
    res = ga.ga_bounds(material.make_material(micro), (N, N), tol=TOL)
    arith = a0 * (1 - w) + a1 * w
    harm = 1.0 / ((1 - w) / a0 + w / a1)
    up, lo = res["upper"], res["lower"]
    assert abs(up[1, 1] - arith) < 1e-12 * arith
    assert abs(lo[0, 0] - harm) < 1e-12 * harm
    assert abs(up[0, 1]) < 1e-12 and abs(lo[0, 1]) < 1e-12
    assert up[0, 0] > harm and lo[1, 1] < arith


def _cos_laminate(alpha0, alpha1, invert=False):
    """a(x_1) = alpha0 + alpha1 cos(2 pi x_1) (or 1/a of that form), with closed-form 1/a series."""
    s = math.sqrt(alpha0 ** 2 - alpha1 ** 2)
    rho = (s - alpha0) / alpha1

    def trig(k):
        out = np.zeros((2, 2) + k.shape[1:], complex)
        on = k[1] == 0
        v = np.where(on & (k[0] == 0), alpha0, 0.0) + np.where(on & (np.abs(k[0]) == 1), alpha1 / 2, 0.0)
        out[0, 0] = out[1, 1] = v
        return out

    def series(k):
        out = np.zeros((2, 2) + k.shape[1:], complex)
        v = np.where(k[1] == 0, rho ** np.abs(k[0]) / s, 0.0)
        out[0, 0] = out[1, 1] = v
        return out

    fA, fB = (series, trig) if invert else (trig, series)
    return material.FourierSeriesMaterial(2, fA, fB), s


@pytest.mark.parametrize("N", [3, 7, 15])
def test_cos_laminate_closed_form(N):
    a0, a1 = 3.0, 2.0
    mat, s = _cos_laminate(a0, a1)
    res = ga.ga_bounds(mat, (N, N), tol=TOL)
    # A_H = diag(harmonic, arithmetic) = diag(s, a0); dual exact for N >= 3
    np.testing.assert_allclose(res["lower"], np.diag([s, a0]), rtol=1e-11, atol=1e-11)
    assert abs(res["upper"][1, 1] - a0) < 1e-12
    assert res["upper"][0, 0] > s
    # mirror: 1/a = b0 + b1 cos -> primal exact, A_H = diag(1/b0, 1/sqrt(b0^2-b1^2))
    b0, b1 = 0.5, 0.3
    mat2, s2 = _cos_laminate(b0, b1, invert=True)
    res2 = ga.ga_bounds(mat2, (N, N), tol=TOL)
    np.testing.assert_allclose(res2["upper"], np.diag([1 / b0, 1 / s2]), rtol=1e-11, atol=1e-11)


def _two_inclusion_micro(invert=False):
    a0, ar, ac = 1.0, 12.0, 0.2
    if invert:
        a0, ar, ac = 1 / a0, 1 / ar, 1 / ac
    return {"d": 2, "kind": "inclusions", "A0": a0 * np.eye(2),
            "shapes": ["rect", "circ"],
            "centers": np.array([[0.1, -0.2], [-0.25, 0.2]]),
            "sizes": np.array([[0.35, 0.2], [0.12, 0.0]]),
            "A_in": np.array([ar * np.eye(2), ac * np.eye(2)])}


@pytest.mark.parametrize("N", [5, 9])
def test_discrete_keller_identity_2d(N):
    R = np.array([[0.0, -1.0], [1.0, 0.0]])
    res_a = ga.ga_bounds(material.make_material(_two_inclusion_micro()), (N, N), tol=TOL)
    res_inv = ga.ga_bounds(material.make_material(_two_inclusion_micro(True)), (N, N), tol=TOL)
    np.testing.assert_allclose(res_a["B_HN"], R @ res_inv["upper"] @ R.T, rtol=1e-11, atol=1e-12)
    assert abs(res_a["upper"][0, 1]) > 1e-4  # a genuinely full matrix


@pytest.mark.parametrize("case", ["rect5", "circ9", "circ15", "two9", "aniso3d", "voxel7"])
def test_dense_route_equals_fft_route(case):
    if case == "rect5":
        micro, N = synth.square_inclusion(2, 0.6, 1.0, 10.0), (5, 5)
    elif case == "circ9":
        micro, N = synth.circle_inclusion_vf(0.3, 1.0, 100.0), (9, 9)
    elif case == "circ15":
        micro, N = synth.circle_inclusion_vf(0.3, 1.0, 100.0, center=(0.13, -0.07)), (15, 13)
    elif case == "two9":
        micro, N = _two_inclusion_micro(), (9, 9)
    elif case == "aniso3d":
        micro, N = synth.cube_inclusion_aniso(0.5, 3), (5, 5, 5)
    else:
        micro, N = synth.grf_voxels(11, (9, 9), d=2, corr_len=0.15), (7, 7)
    mat = material.make_material(micro)
    o2 = ga.ga_bounds(mat, N, tol=1e-13)
    o1 = dense.dense_bounds(mat, N)
    for key in ("upper", "lower"):
        err = np.linalg.norm(o2[key] - o1[key]) / np.linalg.norm(o1[key])
        assert err < 1e-12, (key, err)


def test_loewner_chain_c1():
    mat = material.make_material(synth.square_inclusion(2, 0.6, 1.0, 10.0))
    res = ga.ga_bounds(mat, (21, 21), tol=TOL)
    voigt, reuss = ga.voigt_reuss(mat, 2)
    up, lo = res["upper"], res["lower"]
    assert _psd(up - lo, 0) and _psd(lo - reuss, 0) and _psd(voigt - up, 0)
    assert np.min(np.linalg.eigvalsh(up - lo)) > 1e-3  # a real gap at this N


def test_monotone_in_N_circle():
    mat = material.make_material(synth.circle_inclusion_vf(0.3, 1.0, 100.0))
    prev = None
    for N in (5, 9, 15, 21):
        res = ga.ga_bounds(mat, (N, N), tol=TOL)
        if prev is not None:
            assert _psd(prev["upper"] - res["upper"], 1e-11)
            assert _psd(res["lower"] - prev["lower"], 1e-11)
        prev = res


def test_cg_energy_monotone_from_voigt():
    mat = material.make_material(synth.square_inclusion(2, 0.8, 1.0, 1e4))
    res = ga.ga_bounds(mat, (9, 9), tol=1e-10, track_energy=True)
    voigt, reuss = ga.voigt_reuss(mat, 2)
    for a, en in enumerate(res["energies_primal"]):
        assert abs(en[0] - voigt[a, a]) < 1e-10 * voigt[a, a]
        assert all(en[i + 1] <= en[i] + 1e-12 * en[0] for i in range(len(en) - 1))
        assert abs(en[-1] - res["gram_A"][a, a]) < 1e-9 * en[-1]
    for a, en in enumerate(res["energies_dual"]):
        assert abs(en[0] - 1.0 / reuss[a, a]) < 1e-10 / reuss[a, a]
        assert all(en[i + 1] <= en[i] + 1e-12 * en[0] for i in range(len(en) - 1))


def test_translation_invariance():
    base = synth.square_inclusion(2, 0.45, 1.0, 20.0)
    moved = synth.square_inclusion(2, 0.45, 1.0, 20.0, center=(0.1234, -0.0567))
    r0 = ga.ga_bounds(material.make_material(base), (9, 9), tol=TOL)
    r1 = ga.ga_bounds(material.make_material(moved), (9, 9), tol=TOL)
    np.testing.assert_allclose(r1["upper"], r0["upper"], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(r1["lower"], r0["lower"], rtol=1e-11, atol=1e-12)


def test_symmetry_and_scaling():
    mat = material.make_material(synth.square_inclusion(2, 0.6, 1.0, 10.0))
    res = ga.ga_bounds(mat, (9, 9), tol=TOL)
    for key in ("upper", "lower"):
        m = res[key]
        assert abs(m[0, 1]) < 1e-12 and abs(m[0, 0] - m[1, 1]) < 1e-12 * m[0, 0]
    lam = 3.7
    res2 = ga.ga_bounds(material.make_material(synth.square_inclusion(2, 0.6, lam, 10.0 * lam)),
                        (9, 9), tol=TOL)
    np.testing.assert_allclose(res2["upper"], lam * res["upper"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(res2["lower"], lam * res["lower"], rtol=1e-12, atol=1e-13)
    assert res2["iters_primal"] == res["iters_primal"]


def test_padded_grid_gives_same_bounds():
    """Lemma integ_eval_VM holds for any M >= 2N-1: padding M changes nothing."""
    mat = material.make_material(synth.circle_inclusion_vf(0.3, 1.0, 100.0))
    r0 = ga.ga_bounds(mat, (9, 9), tol=TOL)
    r1 = ga.ga_bounds(mat, (9, 9), M=(21, 25), tol=TOL)
    np.testing.assert_allclose(r1["upper"], r0["upper"], rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(r1["lower"], r0["lower"], rtol=1e-11, atol=1e-13)
