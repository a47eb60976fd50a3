"""Pins for the oracle's upper-upper / lower-lower bounds (Lemma bounds_bounds,
Remark adjusting_A).

* validity: at random points of every voxel the material's extreme eigenvalues
  lie between the lower and the upper image (point evaluation written out here
  from eq. inclcomp, independently of the voxel classification);
* exactness: for a box whose faces lie on voxel faces both images equal the
  exact voxel image, and the resulting bounds equal the closed-form Ga bounds;
* Lemma bounds_bounds: the envelope bounds bracket the Ga bounds of the exact
  material and tighten as the resolution grows.
"""

import numpy as np
import pytest

import synth
from oracle import envelope, ga, material


def _point_extremes(micro, x):
    """Largest and smallest eigenvalue of A at the points x (d, n)."""
    d = int(micro["d"])
    n = x.shape[1]
    phase = np.full(n, -1)
    for i, shape in enumerate(micro["shapes"]):
        c = np.asarray(micro["centers"][i], float)[:, None]
        h = np.asarray(micro["sizes"][i], float)
        dx = x - c
        dx -= np.round(dx)
        if shape == "rect":
            ins = np.all(np.abs(dx) < 0.5 * h[:, None], axis=0)
        else:
            ins = np.sum(dx * dx, axis=0) < h[0] ** 2
        phase[ins] = i
    hi = np.empty(n)
    lo = np.empty(n)
    for i in range(-1, len(micro["shapes"])):
        A = micro["A0"] if i < 0 else micro["A_in"][i]
        w = np.linalg.eigvalsh(np.asarray(A, float))
        hi[phase == i] = w[-1]
        lo[phase == i] = w[0]
    return hi, lo


@pytest.mark.parametrize("case", ["circle2d", "twophase2d", "aniso3d"])
def test_images_bracket_the_material_pointwise(case):
    rng = np.random.default_rng(7)
    if case == "circle2d":
        micro, P = synth.circle_inclusion_vf(0.3, 1.0, 100.0, center=(0.03, -0.07)), (15, 21)
    elif case == "twophase2d":
        micro = {"d": 2, "kind": "inclusions", "A0": np.eye(2), "shapes": ["rect", "circ"],
                 "centers": np.array([[0.1, -0.2], [-0.25, 0.2]]), "sizes": np.array([[0.35, 0.2], [0.12, 0.0]]),
                 "A_in": np.array([12 * np.eye(2), 0.2 * np.eye(2)])}
        P = (25, 15)
    else:
        micro, P = synth.cube_inclusion_aniso(0.45, 5), (9, 7, 11)
    d = len(P)
    up, lo = envelope.images(micro, P)
    idx = np.array(np.unravel_index(np.arange(int(np.prod(P))), P))
    centre = np.array([np.where(idx[a] < (P[a] + 1) // 2, idx[a], idx[a] - P[a]) / P[a] for a in range(d)])
    for _ in range(12):
        off = (rng.random(centre.shape) - 0.5) / np.array(P, float)[:, None]
        hi, lw = _point_extremes(micro, centre + off)
        assert np.all(hi <= up.reshape(-1)) and np.all(lw >= lo.reshape(-1))
    assert np.all(lo <= up)


def test_voxel_aligned_box_is_exact():
    # box [-3/18, 3/18]^2 on a 9 x 9 voxel grid: no voxel is cut
    micro = synth.square_inclusion(2, 1.0 / 3.0, 1.0, 10.0)
    P = (9, 9)
    up, lo = envelope.images(micro, P)
    np.testing.assert_array_equal(up, lo)
    res = ga.ga_bounds(material.make_material(envelope.envelope_micro(micro, P)), (7, 7), tol=1e-12)
    ref = ga.ga_bounds(material.make_material(micro), (7, 7), tol=1e-12)
    for key in ("upper", "lower"):
        np.testing.assert_allclose(res[key], ref[key], rtol=1e-11, atol=1e-12 * np.abs(ref[key]).max())


def test_envelope_bounds_bracket_and_tighten():
    micro = synth.circle_inclusion_vf(0.3, 1.0, 100.0)
    N = (15, 15)
    ref = ga.ga_bounds(material.make_material(micro), N, tol=1e-11)
    widths = []
    for P in (15, 45, 135):
        r = ga.ga_bounds(material.make_material(envelope.envelope_micro(micro, (P, P))), N, tol=1e-11)
        assert np.min(np.linalg.eigvalsh(r["upper"] - ref["upper"])) >= -1e-10
        assert np.min(np.linalg.eigvalsh(ref["lower"] - r["lower"])) >= -1e-10
        widths.append(np.trace(r["upper"] - r["lower"]))
    assert widths[0] > widths[1] > widths[2] > np.trace(ref["upper"] - ref["lower"])
