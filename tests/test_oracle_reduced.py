"""Pins for the oracle's reduced Ga (Lemma reduce_grid, Algorithm 3).

* eq. index_split: k = 2r - s covers the double grid Z_{2N} exactly once;
* the operator is that of Algorithm 2: for random trigonometric polynomials of
  order N, Algorithm 3 on their coefficients equals the Fourier coefficients of
  Algorithm 2 applied on the double grid M = 2N - 1 (a different grid size,
  computed without any shift), and the quadratic forms agree (the identity in
  the proof of Lemma reduce_grid) -- 2D/3D, primal/dual, inclusions and voxels,
  non-cubic N;
* a homogeneous material gives Ahat^full = A;
* the reduced Ga bounds equal the Ga bounds of the double grid.
"""

import numpy as np
import pytest

import synth
from oracle import ga, grids, material, reduced

CASES = {
    "circle2d_N9": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0, center=(0.05, -0.1)), (9, 9)),
    "square2d_N7x11": (lambda: synth.square_inclusion(2, 0.6, 1.0, 10.0, center=(0.1, 0.2)), (7, 11)),
    "aniso3d_N5": (lambda: synth.cube_inclusion_aniso(0.5, 3), (5, 5, 5)),
    "voxel2d_P15_N9": (lambda: synth.grf_voxels(11, (15, 15), d=2, corr_len=0.15), (9, 9)),
    "voxel3d_P9_N5x7x3": (lambda: synth.grf_voxels(12, (9, 9, 9), d=3, corr_len=0.15), (5, 7, 3)),
}


def test_index_split_is_a_bijection():
    for n in (3, 5, 9):
        hits = np.zeros(2 * n, dtype=int)
        for r in range(n):
            for s in (0, 1):
                hits[(2 * r - s) % (2 * n)] += 1
        assert np.all(hits == 1)


def _random_trig(N, d, seed):
    """Values on the N-grid of a random real trigonometric polynomial of order N."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((d,) + tuple(N))


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("kind", ["E", "J"])
def test_operator_equals_double_grid(name, kind):
    make, N = CASES[name]
    mat = material.make_material(make())
    d = len(N)
    which = "A" if kind == "E" else "B"
    M = tuple(2 * n - 1 for n in N)
    AM = material.double_grid_matrix(mat, N, M, which)
    AS = reduced.shifted_matrices(mat, N, which)
    axes = tuple(range(1, d + 1))
    for seed in range(2):
        u = _random_trig(N, d, seed)
        uh = grids.dft(u, axes=axes)
        y3 = reduced.matvec_hat(AS, uh, N, kind)
        uM = ga.prolong(u, N, M)  # the same polynomial on the double grid
        y2h = grids.dft(ga.matvec(AM, uM, N, kind), axes=axes)
        keep = grids.in_Z(grids.freq_grid(M), N)
        kN = grids.freq_grid(N)
        idx = tuple(np.mod(kN[a], M[a]) for a in range(d))
        y2 = y2h[(slice(None),) + idx]
        assert np.abs(y2h[:, ~keep]).max() <= 1e-12 * np.abs(y2).max()
        np.testing.assert_allclose(y3, y2, rtol=0, atol=1e-12 * np.abs(y2).max())
        # quadratic forms: (Ahat^full uhat, uhat) = (A_M u, u)_{R^{d x M}}
        q3 = float(np.real(np.sum(reduced.apply_full_hat(AS, uh, N) * np.conj(uh))))
        q2 = ga.inner(material.apply_pointwise(AM, uM), uM)
        assert abs(q3 - q2) <= 1e-12 * abs(q2)


def test_homogeneous_is_the_material():
    A = synth.random_spd(4, 2, 0.0, 1.0)
    micro = synth.square_inclusion(2, 0.5, 1.0, 1.0)
    micro["A0"] = A
    micro["A_in"] = A.reshape(1, 2, 2).copy()
    N = (5, 7)
    AS = reduced.shifted_matrices(material.make_material(micro), N, "A")
    uh = grids.dft(_random_trig(N, 2, 3), axes=(1, 2))
    y = reduced.apply_full_hat(AS, uh, N)
    np.testing.assert_allclose(y, np.einsum("ab,b...->a...", A, uh), atol=1e-13 * np.abs(uh).max())


@pytest.mark.parametrize("name", ["circle2d_N9", "aniso3d_N5", "voxel2d_P15_N9"])
def test_bounds_equal_ga_bounds(name):
    make, N = CASES[name]
    mat = material.make_material(make())
    r = reduced.reduced_bounds(mat, N, tol=1e-12)
    g = ga.ga_bounds(mat, N, tol=1e-12)
    for key in ("upper", "lower"):
        np.testing.assert_allclose(r[key], g[key], rtol=1e-10, atol=1e-10 * np.abs(g[key]).max())
