"""Pins for the oracle's GaNi scheme and its a-posteriori bounds.

* Remark duality_gani: for odd N the GaNi primal and dual matrices are
  inverse to each other, B~_{H,N}^{-1} = A~_{H,N} (2D/3D, inclusions, voxels,
  non-cubic grids);
* a homogeneous material is reproduced exactly;
* the GaNi minimisers from CG equal a dense brute-force minimisation of the
  rectangle-rule quadratic form over E_N at tiny N (projection assembled as a
  dense matrix from the DFT, no FFT and no CG);
* eq. GaNi_apost and Prop. struct_bounds: the a-posteriori bounds are
  guaranteed, so they bracket the Ga bounds of the same N (the Ga fields
  minimise the exact energies over the same spaces).  (They need not lie
  inside the Voigt-Reuss bounds: a GaNi field minimises the sampled energy,
  and its exact energy can exceed that of the zero field.)
* sampling: at P = N a voxel image is sampled to itself.
"""

import numpy as np
import pytest

import synth
from oracle import ga, gani, grids, material

CASES = {
    "circle2d_N15": (lambda: synth.circle_inclusion_vf(0.3, 1.0, 100.0, center=(0.05, -0.1)), (15, 15)),
    "square2d_N9x11": (lambda: synth.square_inclusion(2, 0.6, 1.0, 10.0, center=(0.1, 0.2)), (9, 11)),
    "aniso3d_N5": (lambda: synth.cube_inclusion_aniso(0.5, 3), (5, 5, 5)),
    "voxel3d_N9": (lambda: synth.grf_voxels(12, (9, 9, 9), d=3, corr_len=0.15), (9, 9, 9)),
    "voxel2d_P15_N9": (lambda: synth.grf_voxels(11, (15, 15), d=2, corr_len=0.15), (9, 9)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_gani_duality_for_odd_grids(name):
    make, N = CASES[name]
    r = gani.gani(make(), N, tol=1e-12)
    np.testing.assert_allclose(np.linalg.inv(r["B_gani"]), r["A_gani"], rtol=1e-10,
                               atol=1e-10 * np.abs(r["A_gani"]).max())


def test_homogeneous_is_exact():
    A = synth.random_spd(5, 2, 0.0, 1.0)
    micro = synth.square_inclusion(2, 0.5, 1.0, 1.0)
    micro["A0"] = A
    micro["A_in"] = A.reshape(1, 2, 2).copy()
    r = gani.gani(micro, (7, 9), tol=1e-12)
    np.testing.assert_allclose(r["A_gani"], A, rtol=1e-13)
    ap = gani.apost_bounds(micro, r)
    np.testing.assert_allclose(ap["upper"], A, rtol=1e-13)
    np.testing.assert_allclose(ap["lower"], A, rtol=1e-13)


def _dense_projection(N):
    """G^E on R^{d x N} as a dense matrix: F^{-1} Ghat F with Ghat(k) = k k^T / k.k."""
    d = len(N)
    n = int(np.prod(N))
    k = grids.freq_grid(N).reshape(d, n).astype(float)
    x = grids.grid_points(N).reshape(d, n) * np.array(N, float)[:, None]  # integer grid indices, centred
    ph = np.exp(-2j * np.pi * sum(np.outer(k[a], x[a]) / N[a] for a in range(d)))  # F (unnormalised)
    k2 = np.sum(k * k, axis=0)
    G = np.zeros((d * n, d * n), dtype=complex)
    for a in range(d):
        for b in range(d):
            ghat = np.where(k2 > 0, k[a] * k[b] / np.where(k2 > 0, k2, 1.0), 0.0)
            G[a * n:(a + 1) * n, b * n:(b + 1) * n] = (ph.conj().T * ghat) @ ph / n
    return G.real


def test_gani_matches_dense_minimisation():
    micro = synth.square_inclusion(2, 0.6, 1.0, 10.0, center=(0.1, 0.2))
    N = (5, 7)
    d, n = 2, 35
    r = gani.gani(micro, N, tol=1e-13)
    AN = gani.sample(micro, N, "A")
    G = _dense_projection(N)
    Adiag = np.zeros((d * n, d * n))
    for a in range(d):
        for b in range(d):
            if AN[(a, b)] is not None:
                Adiag[a * n:(a + 1) * n, b * n:(b + 1) * n] = np.diag(AN[(a, b)].ravel())
    # minimise (A (E + e), E + e) over e = G e: solve G A G e = -G A E on range(G)
    K = G @ Adiag @ G + (np.eye(d * n) - G)
    Ah = np.zeros((d, d))
    for a in range(d):
        E = np.repeat(np.eye(d)[a], n)
        e = np.linalg.solve(K, -G @ Adiag @ E)
        f = E + e
        for b in range(d):
            Eb = np.repeat(np.eye(d)[b], n)
            eb = np.linalg.solve(K, -G @ Adiag @ Eb)
            Ah[a, b] = f @ Adiag @ (Eb + eb) / n
        np.testing.assert_allclose(r["fields_primal"][a].reshape(d * n), e, atol=1e-10)
    np.testing.assert_allclose(r["A_gani"], 0.5 * (Ah + Ah.T), rtol=1e-11, atol=1e-12 * np.abs(Ah).max())


@pytest.mark.parametrize("name", sorted(CASES))
def test_apost_bounds_bracket_ga_bounds(name):
    make, N = CASES[name]
    micro = make()
    d = len(N)
    r = gani.gani(micro, N, tol=1e-12)
    ap = gani.apost_bounds(micro, r)
    mat = material.make_material(micro)
    gb = ga.ga_bounds(mat, N, tol=1e-12)
    scale = np.abs(gb["upper"]).max()
    psd = lambda m: np.min(np.linalg.eigvalsh(0.5 * (m + m.T))) >= -1e-10 * scale
    assert psd(ap["upper"] - gb["upper"]) and psd(gb["lower"] - ap["lower"])
    assert psd(ap["upper"] - ap["lower"])


def test_voxel_sampling_at_P_equal_N():
    micro = synth.grf_voxels(3, (9, 15), d=2, corr_len=0.2)
    AN = gani.sample(micro, (9, 15), "A")
    np.testing.assert_array_equal(AN[(0, 0)], micro["image"])
    assert AN[(0, 1)] is None
