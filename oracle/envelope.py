"""Upper and lower voxel approximations of an inclusion composite (Lemma
bounds_bounds, Remark adjusting_A).  TEST INFRASTRUCTURE ONLY: used by tests/
and the bench's CPU leg, never by the product path.

Remark adjusting_A: on a voxel grid of resolution P, the upper approximation
takes in every voxel the largest eigenvalue of A over that voxel (times I), the
lower one the smallest, so that A_lower(x) <= A(x) <= A_upper(x) for almost
every x.  For a composite of a matrix phase A0 and non-overlapping inclusions
A_in,i (eq. inclcomp) the extreme eigenvalues over a voxel are those of the
phases that occupy part of it with positive measure.  Lemma bounds_bounds then
gives guaranteed bounds from the Ga primal with A_upper and the Ga dual with
A_lower.

Readings where the paper is silent: voxel p is the box centred at p/P (centred
index) with sides 1/P; a phase is present in a voxel when the intersection has
positive measure; the matrix phase is counted present unless one inclusion
contains the whole voxel (which can only over-approximate the set of phases,
keeping both inequalities).
"""

from __future__ import annotations

import numpy as np

from . import grids


def _phase_extremes(A):
    w = np.linalg.eigvalsh(np.asarray(A, float))
    return float(w[-1]), float(w[0])


def images(micro, P):
    """(upper, lower) voxel images (scalar, P^d each) for an inclusion descriptor."""
    d = int(micro["d"])
    P = tuple(int(p) for p in P)
    xc = grids.grid_points(P)  # voxel centres p/P, centred indices
    half = np.array([0.5 / p for p in P]).reshape((d,) + (1,) * d)
    hi0, lo0 = _phase_extremes(micro["A0"])
    up = np.full(P, -np.inf)
    lo = np.full(P, np.inf)
    matrix_present = np.ones(P, dtype=bool)
    for i, shape in enumerate(micro["shapes"]):
        c = np.asarray(micro["centers"][i], float).reshape((d,) + (1,) * d)
        h = np.asarray(micro["sizes"][i], float)
        dc = xc - c
        dc = np.abs(dc - np.round(dc))  # |centre offset| under the minimum image
        if shape == "rect":
            hh = 0.5 * h.reshape((d,) + (1,) * d)
            meets = np.all(dc < hh + half, axis=0)
            contains = np.all(dc + half <= hh, axis=0)
        elif shape == "circ":
            r = float(h[0])
            near = np.maximum(dc - half, 0.0)  # nearest point of the voxel box
            far = dc + half  # farthest corner
            meets = np.sum(near * near, axis=0) < r * r
            contains = np.sum(far * far, axis=0) <= r * r
        else:
            raise ValueError(shape)
        hi, lw = _phase_extremes(micro["A_in"][i])
        up = np.where(meets, np.maximum(up, hi), up)
        lo = np.where(meets, np.minimum(lo, lw), lo)
        matrix_present &= ~contains
    up = np.where(matrix_present, np.maximum(up, hi0), up)
    lo = np.where(matrix_present, np.minimum(lo, lo0), lo)
    return up, lo


def envelope_micro(micro, P):
    """A voxel descriptor whose primal side is the upper image and whose dual
    side is the lower image (Lemma bounds_bounds)."""
    up, lo = images(micro, P)
    return {"d": int(micro["d"]), "kind": "voxels", "P": tuple(int(p) for p in P), "image": up,
            "image_dual": lo}
