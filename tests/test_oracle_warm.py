"""Pins for the oracle's bound monitoring and coarse-to-fine warm start (Sec. 6.4).

* Prolongation: a coarse Ga field, carried to a finer grid by Fourier zero
  padding, is the same trigonometric polynomial, so its exact double-grid
  energy on the fine grid equals the coarse energy (no approximation is made
  in this step); it is admissible on the fine grid (G e = e).
* Warm start: CG started from the prolonged field reaches the same Ga bounds
  (the minimiser is unique); its first energy is the coarse bound entry, below
  the Voigt entry a cold start begins from.  (It does not, in general, save
  iterations to a tight tolerance: the smooth error components it removes are
  the ones CG removes fastest.)
* Monitoring: the energy of the k-th CG iterate equals the initial energy minus
  sum_j alpha_j (r_{j-1}, r_{j-1}) (CG on the quadratic functional whose
  minimum is the Ga energy), cold and warm, and never increases.
"""

import numpy as np
import pytest

import synth
from oracle import ga, grids, material


def _circle(contrast=50.0):
    return material.make_material(synth.circle_inclusion_vf(0.3, 1.0, contrast))


def _aniso3d():
    return material.make_material(synth.cube_inclusion_aniso(0.5, 3))


@pytest.mark.parametrize("kind,which", [("E", "A"), ("J", "B")])
def test_prolonged_field_keeps_its_exact_energy(kind, which):
    mat = _circle()
    Nc, N = (5, 5), (11, 13)
    Mc = tuple(2 * n - 1 for n in Nc)
    M = tuple(2 * n - 1 for n in N)
    AMc = material.double_grid_matrix(mat, Nc, Mc, which)
    AMf = material.double_grid_matrix(mat, N, M, which)
    for a in range(2):
        E = np.eye(2)[a]
        e_c, _ = ga.solve(AMc, Nc, E, kind, tol=1e-12)
        e_f = ga.prolong(e_c, Nc, M)
        assert e_f.shape == (2,) + M
        np.testing.assert_allclose(ga.project(e_f, N, kind), e_f, atol=1e-13)
        ec = ga.energy(AMc, E, e_c)
        ef = ga.energy(AMf, E, e_f)
        assert abs(ef - ec) <= 1e-12 * abs(ec)
        # the zero field of the coarse grid is not a fixed point: the energy moved
        assert ec < ga.energy(AMc, E, np.zeros_like(e_c)) - 1e-6


def test_prolongation_reproduces_a_trigonometric_polynomial():
    # sampling the same polynomial on two grids: prolong must map one onto the other
    rng = np.random.default_rng(1)
    Nc, Mc, M = (5, 7), (9, 13), (21, 15)
    kc = grids.freq_grid(Mc)
    mask = grids.in_Z(kc, Nc)
    coef = np.zeros((2,) + Mc, dtype=complex)
    vals = rng.standard_normal((2, int(mask.sum()))) + 1j * rng.standard_normal((2, int(mask.sum())))
    coef[:, mask] = vals
    coef = 0.5 * (coef + np.conj(coef[(slice(None),) + tuple(np.mod(-kc[a], Mc[a]) for a in range(2))]))
    x_c = grids.grid_points(Mc)
    x_f = grids.grid_points(M)

    def sample(x):
        out = np.zeros((2,) + x.shape[1:])
        for idx in zip(*np.nonzero(mask)):
            k = np.array([kc[a][idx] for a in range(2)])
            ph = np.exp(2j * np.pi * np.tensordot(k, x, axes=1))
            for c in range(2):
                out[c] += np.real(coef[(c,) + idx] * ph)
        return out

    np.testing.assert_allclose(ga.prolong(sample(x_c), Nc, M), sample(x_f), atol=1e-12)


@pytest.mark.parametrize("case", ["circle2d", "aniso3d"])
def test_warm_start_reaches_the_same_bounds_from_a_better_start(case):
    if case == "circle2d":
        mat, Nc, N, d = _circle(), (5, 5), (15, 15), 2
    else:
        mat, Nc, N, d = _aniso3d(), (3, 3, 3), (7, 7, 7), 3
    tol = 1e-10
    coarse = ga.ga_bounds(mat, Nc, tol=tol, track_energy=True)
    cold = ga.ga_bounds(mat, N, tol=tol)
    warm = ga.ga_bounds(mat, N, tol=tol, warm=coarse, track_energy=True)
    for key in ("upper", "lower"):
        np.testing.assert_allclose(warm[key], cold[key], rtol=1e-9, atol=1e-9 * np.abs(cold[key]).max())
    voigt, reuss = ga.voigt_reuss(mat, d)
    # first energy of each warm solve = the coarse bound entry (exact transfer),
    # strictly better than the cold start's Voigt entry
    for a in range(d):
        assert warm["energies_primal"][a][0] < voigt[a, a] * (1 - 1e-6)
        assert warm["energies_dual"][a][0] < np.linalg.inv(reuss)[a, a] * (1 - 1e-6)
        assert abs(warm["energies_primal"][a][0] - coarse["gram_A"][a, a]) <= 1e-12 * coarse["gram_A"][a, a]
        assert abs(warm["energies_dual"][a][0] - coarse["gram_B"][a, a]) <= 1e-12 * coarse["gram_B"][a, a]


@pytest.mark.parametrize("start", ["cold", "warm"])
def test_energy_recurrence_matches_the_quadrature(start):
    mat = _circle(200.0)
    N = (13, 13)
    coarse = ga.ga_bounds(mat, (5, 5), tol=1e-12) if start == "warm" else None
    res = ga.ga_bounds(mat, N, tol=1e-10, track_energy=True, warm=coarse)
    for key in ("primal", "dual"):
        for a in range(2):
            en = np.array(res["energies_" + key][a])
            cgs = res["cg_" + key][a]
            assert len(en) == len(cgs["alphas"]) + 1 >= 3
            rec = en[0] - np.concatenate([[0.0], np.cumsum(np.array(cgs["alphas"]) * np.array(cgs["rr"][:-1]))])
            np.testing.assert_allclose(rec, en, rtol=1e-10)
            assert np.all(np.diff(en) <= 1e-12 * en[0])


def test_cold_start_energy_is_voigt():
    mat = _circle()
    res = ga.ga_bounds(mat, (9, 9), tol=1e-10, track_energy=True)
    voigt, _ = ga.voigt_reuss(mat, 2)
    for a in range(2):
        assert abs(res["energies_primal"][a][0] - voigt[a, a]) <= 1e-12 * voigt[a, a]


@pytest.mark.parametrize("btol", [1e-4, 1e-6, 1e-8])
def test_bound_tolerance_rule_on_exact_energies(btol):
    # the library's bound-based stopping rule (tests/bound_rule.py) applied to
    # the oracle's exact energies of the CG iterates: it stops before
    # convergence, and the energy where it stops is on the guaranteed side of
    # the converged Ga energy (every iterate is admissible, Sec. 6.4) and
    # within a small multiple of btol of it
    from bound_rule import first_stop
    mat = _circle(200.0)
    N = (21, 21)
    ref = ga.ga_bounds(mat, N, tol=1e-12, track_energy=True)
    for key, gram in (("primal", ref["gram_A"]), ("dual", ref["gram_B"])):
        for a in range(2):
            en = ref["energies_" + key][a]
            k = first_stop(en, btol)
            assert k is not None and k < ref["iters_" + key][a]
            conv = gram[a, a]
            assert en[k] >= conv * (1 - 1e-13)
            assert (en[k] - conv) / conv <= 20 * btol
