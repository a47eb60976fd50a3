"""Pins for the double-grid quadrature (Lemma integ_eval_VM) and the material setup.

The exact integral (A u_N, v_N)_{L^2} for trigonometric polynomials u_N, v_N is
computed independently: the matrix phase by Parseval, the inclusion part by
adaptive integration of u_N . v_N over the inclusion itself.
"""

import math

import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import dense, grids, material


def _random_trig(N, d, seed):
    """Coefficients (d, N, N) of a real trigonometric polynomial field in T_N^d."""
    rng = np.random.default_rng(seed)
    vals = rng.standard_normal((d,) + tuple(N))
    return grids.dft(vals, axes=tuple(range(1, len(N) + 1)))


def _on_grid(uh, N, M):
    d = uh.shape[0]
    big = np.zeros((d,) + tuple(M), complex)
    kN = grids.freq_grid(N)
    idx = tuple(np.mod(kN[a], M[a]) for a in range(len(N)))
    for c in range(d):
        big[c][idx] = uh[c]
    return np.real(grids.idft(big, axes=tuple(range(1, len(N) + 1))))


def _eval_point(uh, N, x):
    kN = grids.freq_grid(N)
    ph = np.exp(2j * np.pi * (kN[0] * x[0] + kN[1] * x[1]))
    return np.real(np.sum(uh * ph[None], axis=(1, 2)))


def _quadrature(AM, u, v):
    return float(np.sum(material.apply_pointwise(AM, u) * v)) / np.prod(u.shape[1:])


@pytest.mark.parametrize("shape", ["rect", "circ"])
def test_double_grid_is_exact_integral(shape):
    N = (3, 3)
    a0, a1 = 1.0, 7.0
    if shape == "rect":
        micro = synth.square_inclusion(2, 0.6, a0, a1, center=(0.1, -0.05))
        h = micro["sizes"][0]
        c = micro["centers"][0]
        lims = (c[0] - h[0] / 2, c[0] + h[0] / 2,
                lambda x: c[1] - h[1] / 2, lambda x: c[1] + h[1] / 2)
    else:
        micro = synth.circle_inclusion_vf(0.3, a0, a1, center=(-0.2, 0.1))
        r = micro["sizes"][0][0]
        c = micro["centers"][0]
        lims = (c[0] - r, c[0] + r,
                lambda x: c[1] - math.sqrt(max(r * r - (x - c[0]) ** 2, 0.0)),
                lambda x: c[1] + math.sqrt(max(r * r - (x - c[0]) ** 2, 0.0)))
    uh = _random_trig(N, 2, 3)
    vh = _random_trig(N, 2, 4)
    parseval = float(np.real(np.sum(uh * np.conj(vh))))
    g = lambda y, x: float(np.dot(_eval_point(uh, N, (x, y)), _eval_point(vh, N, (x, y))))
    inside, _ = integrate.dblquad(g, lims[0], lims[1], lims[2], lims[3], epsabs=1e-12, epsrel=1e-12)
    exact = a0 * parseval + (a1 - a0) * inside
    mat = material.make_material(micro)
    for M in [(5, 5), (12, 12)]:  # 2N-1 and 2N+6
        AM = material.double_grid_matrix(mat, N, M, "A")
        q = _quadrature(AM, _on_grid(uh, N, M), _on_grid(vh, N, M))
        assert abs(q - exact) < 1e-9 * max(1.0, abs(exact))


def test_quadrature_independent_of_M_and_equals_toeplitz_sum():
    N = (7, 7)
    micro = synth.circle_inclusion_vf(0.3, 1.0, 100.0, center=(0.05, 0.11))
    mat = material.make_material(micro)
    uh = _random_trig(N, 2, 5)
    vh = _random_trig(N, 2, 6)
    vals = []
    for M in [(13, 13), (20, 20), (27, 25)]:
        AM = material.double_grid_matrix(mat, N, M, "A")
        vals.append(_quadrature(AM, _on_grid(uh, N, M), _on_grid(vh, N, M)))
    # Lemma FD_matrix_full: sum_{l,k} conj(vhat(l)) . Ahat(l-k) uhat(k)
    ks, big, col0, a00 = dense.dense_matrix(mat.coeff_A, N)
    allk = np.vstack([np.zeros((1, 2), int), ks])
    table, L = dense._coeff_table(mat.coeff_A, N)
    U = np.concatenate([uh[(slice(None),) + tuple(np.mod(k, N))] for k in allk])
    V = np.concatenate([vh[(slice(None),) + tuple(np.mod(k, N))] for k in allk])
    diff = allk[:, None, :] - allk[None, :, :]
    blk = table[(slice(None), slice(None)) + tuple(np.mod(diff[..., a], L[a]) for a in range(2))]
    n = len(allk)
    full = np.transpose(blk, (2, 0, 3, 1)).reshape(2 * n, 2 * n)
    toeplitz = float(np.real(np.conj(V) @ full @ U))
    for v in vals:
        assert abs(v - toeplitz) < 1e-12 * abs(toeplitz)


@pytest.mark.parametrize("P,N", [(10, 5), (10, 9), (5, 9), (25, 9)])
def test_voxel_image_equals_aligned_rectangle(P, N):
    """Lemma grid_compos vs eq. inclcomp_formula for an image of an aligned box.

    Voxel p covers [p/P - 1/(2P), p/P + 1/(2P)); voxels |p| <= w form a box of
    side (2w+1)/P.  P < 2N-1 exercises periodic enlargement, P > 2N-1 truncation
    (Remark eval_with_FFT).
    """
    w = 1 if P <= 5 else 2
    img = np.ones((P, P))
    idx = np.mod(np.arange(-w, w + 1), P)
    img[np.ix_(idx, idx)] = 10.0
    vox = material.make_material({"d": 2, "kind": "voxels", "P": (P, P), "image": img})
    box = material.make_material(synth.square_inclusion(2, (2 * w + 1) / P, 1.0, 10.0))
    M = (2 * N - 1, 2 * N - 1)
    for which in ("A", "B"):
        a = material.double_grid_matrix(vox, (N, N), M, which)
        b = material.double_grid_matrix(box, (N, N), M, which)
        for key in [(0, 0), (1, 1)]:
            np.testing.assert_allclose(a[key], b[key], atol=1e-12)
        assert a[(0, 1)] is None and b[(0, 1)] is None


def test_dual_coefficients_are_those_of_inverse():
    """A^{-1} for a two-phase composite: coefficients of 1/a match adaptive quadrature."""
    micro = synth.square_inclusion(2, 0.4, 2.0, 8.0)
    mat = material.make_material(micro)
    k = np.array([[0, 1, 3], [0, 2, -1]])
    bh = mat.coeff_B(k)[0, 0]
    for j in range(3):
        kk = k[:, j]
        g = lambda y, x: (1 / 8.0 if (abs(x) < 0.2 and abs(y) < 0.2) else 1 / 2.0) * \
            math.cos(2 * math.pi * (kk[0] * x + kk[1] * y))
        v = 0.0
        for xs in [(-0.5, -0.2), (-0.2, 0.2), (0.2, 0.5)]:
            for ys in [(-0.5, -0.2), (-0.2, 0.2), (0.2, 0.5)]:
                v += integrate.dblquad(g, xs[0], xs[1], ys[0], ys[1], epsabs=1e-13)[0]
        assert abs(bh[j] - v) < 1e-11
