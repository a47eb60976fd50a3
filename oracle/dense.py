"""Route O1: dense Fourier-Galerkin solve at tiny N (Lemma FD_matrix_full).

No FFT, no double grid, no CG.  The energy of a trigonometric field with
coefficients uhat on Z_N is sum_{l,k in Z_N} conj(uhat(l)) . Ahat(l - k) uhat(k)
(Lemma FD_matrix_full: the fully populated matrix has blocks Ahat(l - k)).

Primal (Def. Ga over E_N): uhat(0) = E, uhat(k) = t(k) c_k with t(k) = k/|k|
for k in Z_N \\ {0}; every element of E_N has this form (Helmholtz_trig).
Dual (over J_N): uhat(k) = sum_a t_a(k) c_{k,a} with {t_a(k)} an orthonormal
basis of the plane orthogonal to k (d - 1 vectors).  Writing
K = T^H Ahat_full T and g = T^H [Ahat(l) E]_l, the energy is
E.Ahat(0)E + 2 Re(c^H g) + c^H K c, minimised by K c = -g, so

    A_{H,N} = Ahat(0) - G^H K^{-1} G,   G[:, b] = T^H [Ahat(l) e_b]_l.

The dual gives B_{H,N} the same way with the coefficients of A^{-1}.
"""

from __future__ import annotations

import itertools

import numpy as np


def _freqs_nonzero(N):
    rng = [range(-(n - 1) // 2, (n - 1) // 2 + 1) for n in N]
    ks = [k for k in itertools.product(*rng) if any(k)]
    return np.array(ks, dtype=int)


def _basis(ks, kind):
    """Columns: orthonormal basis vectors per frequency; returns (T (d*n, m), m)."""
    n, d = ks.shape
    cols = []
    for i, k in enumerate(ks):
        kh = k / np.linalg.norm(k)
        if kind == "E":
            vecs = [kh]
        else:
            # orthonormal complement of kh: last d-1 left singular vectors
            u, _, _ = np.linalg.svd(kh.reshape(d, 1))
            vecs = [u[:, j] for j in range(1, d)]
        for v in vecs:
            col = np.zeros(d * n)
            col[i * d:(i + 1) * d] = v
            cols.append(col)
    return np.array(cols).T


def _coeff_table(coeff_fn, N):
    """Fourier coefficients on Z_{2N-1}, stored at index n mod (2N-1)."""
    L = [2 * n - 1 for n in N]
    axes = [np.where(np.arange(m) < (m + 1) // 2, np.arange(m), np.arange(m) - m) for m in L]
    k = np.array(np.meshgrid(*axes, indexing="ij"))
    return coeff_fn(k), L


def dense_matrix(coeff_fn, N):
    """(Ahat(l - k))_{l,k in Z_N \\ {0}} assembled as a (d n) x (d n) matrix, plus helpers."""
    ks = _freqs_nonzero(N)
    table, L = _coeff_table(coeff_fn, N)
    d = len(N)
    n = len(ks)
    diff = ks[:, None, :] - ks[None, :, :]
    idx = tuple(np.mod(diff[..., a], L[a]) for a in range(d))
    blocks = table[(slice(None), slice(None)) + idx]  # (d, d, n, n)
    big = np.transpose(blocks, (2, 0, 3, 1)).reshape(d * n, d * n)
    idx0 = tuple(np.mod(ks[:, a], L[a]) for a in range(d))
    col0 = np.transpose(table[(slice(None), slice(None)) + idx0], (2, 0, 1)).reshape(d * n, d)
    zero = tuple(0 for _ in range(d))
    a00 = table[(slice(None), slice(None)) + zero]
    return ks, big, col0, a00


def dense_homogenized(coeff_fn, N, kind):
    """A_{H,N} (kind 'E', with Ahat) or B_{H,N} (kind 'J', with Bhat) by route O1."""
    ks, big, col0, a00 = dense_matrix(coeff_fn, N)
    T = _basis(ks, kind)
    K = T.conj().T @ big @ T
    G = T.conj().T @ col0
    sol = np.linalg.solve(K, G)
    H = a00 - G.conj().T @ sol
    return np.real(0.5 * (H + H.conj().T))


def dense_bounds(mat, N):
    """Upper A_{H,N} and lower B_{H,N}^{-1} by the dense route."""
    up = dense_homogenized(mat.coeff_A, N, "E")
    BH = dense_homogenized(mat.coeff_B, N, "J")
    return {"upper": up, "B_HN": BH, "lower": np.linalg.inv(BH)}
