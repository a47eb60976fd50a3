"""Pins for the discrete projections (Def. discrete_proj, Lemma Helmholtz_decomp)."""

import math

import numpy as np
import pytest

from oracle import ga, grids


def _field(M, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((len(M),) + tuple(M))


@pytest.mark.parametrize("N,M", [((5, 5), (9, 9)), ((5, 7), (9, 15)), ((3, 5, 3), (5, 9, 7))])
def test_projections_idempotent_selfadjoint_complementary(N, M):
    x, y = _field(M, 1), _field(M, 2)
    for kind in ("E", "J"):
        gx = ga.project(x, N, kind)
        np.testing.assert_allclose(ga.project(gx, N, kind), gx, atol=1e-12)
        assert abs(ga.inner(gx, y) - ga.inner(x, ga.project(y, N, kind))) < 1e-12
    # on T_N fields: G^U + G^E + G^J = I (U = constants)
    xN = ga.project(x, N, "E") + ga.project(x, N, "J")
    mean = np.mean(x, axis=tuple(range(1, x.ndim)), keepdims=True)
    xt = xN + mean
    np.testing.assert_allclose(ga.project(xt, N, "E") + ga.project(xt, N, "J") + mean, xt, atol=1e-12)
    # E and J are orthogonal
    assert abs(ga.inner(ga.project(x, N, "E"), ga.project(y, N, "J"))) < 1e-12


@pytest.mark.parametrize("N,M", [((5, 5), (9, 9)), ((3, 3, 3), (5, 5, 5))])
def test_projection_ranks(N, M):
    # dim E_N = |N| - 1, dim J_N = (d-1)(|N| - 1)  (Remark mem_req, Table tab:memory)
    d = len(N)
    n = d * int(np.prod(M))
    for kind, rank in (("E", np.prod(N) - 1), ("J", (d - 1) * (np.prod(N) - 1))):
        cols = []
        for i in range(n):
            e = np.zeros(n)
            e[i] = 1.0
            cols.append(ga.project(e.reshape((d,) + tuple(M)), N, kind).ravel())
        assert np.linalg.matrix_rank(np.array(cols), tol=1e-9) == rank


def test_analytic_gradient_and_rotated_fields():
    """G^E keeps a gradient field and kills a divergence-free one (analytic fields)."""
    N, M = (7, 7), (13, 13)
    x = grids.grid_points(M)
    arg = 2 * math.pi * (x[0] + 2 * x[1])
    grad = np.array([np.cos(arg), 2 * np.cos(arg)])        # grad of sin(arg)/(2 pi)
    rot = np.array([-2 * np.cos(arg), np.cos(arg)])        # R grad: divergence free
    np.testing.assert_allclose(ga.project(grad, N, "E"), grad, atol=1e-12)
    np.testing.assert_allclose(ga.project(grad, N, "J"), 0.0, atol=1e-12)
    np.testing.assert_allclose(ga.project(rot, N, "J"), rot, atol=1e-12)
    np.testing.assert_allclose(ga.project(rot, N, "E"), 0.0, atol=1e-12)
    # frequency (3, 0) lies outside Z_5: both projections vanish for N = (5, 5)
    high = np.array([np.cos(2 * math.pi * 3 * x[0]), 0 * x[0]])
    np.testing.assert_allclose(ga.project(high, (5, 5), "E"), 0.0, atol=1e-12)
    # constants are removed
    np.testing.assert_allclose(ga.project(np.ones((2,) + M), N, "E"), 0.0, atol=1e-12)
