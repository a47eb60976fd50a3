"""The reduced Ga: the double-grid scheme rewritten on the grid of the
approximation order with 2^d shifted DFTs.  TEST INFRASTRUCTURE ONLY: used by
tests/ and the bench's CPU leg, never by the product path.

Follows, in order:
* Lemma reduce_grid -- on a double grid of 2N points per axis every index
  k in Z_{2N} splits uniquely as k = 2r - s with r in Z_N and s in {0,1}^d
  (eq. index_split), and the Ga matrix becomes (eq. Afull_decomp_Fourier)
      Ahat^full = 2^{-d} sum_s S*(s) F_N A_N(s) F_N^{-1} S(s),
  S(s) = diag(omega_{2N}^{-s.m}) on Z_N, A_N(s) the double-grid material
  (eq. MBA_GA with M = 2N) at the points x = (2r - s) / (2N).
* Algorithm 3 -- y = Ghat_{N,N} sum_s 2^{-d} S*(s) F_N A_N(s) F_N^{-1} S(s) x
  on Fourier coefficients x on Z_N; here applied to the values of a
  trigonometric polynomial on the N-grid (one DFT before, one after), so that
  the CG of Remark CG runs in the inner product (u, v)_{R^{d x N}}, which by
  Parseval equals sum_k uhat(k) . conj(vhat(k)).
* eq. Ga_linsys_R -- Ghat Ahat^full ehat = -Ghat Ahat^full Ehat (primal; the
  dual with Bhat and Ghat^J); the bounds are the energy Gram matrices of
  Prop. struct_bounds, with the energy (Ahat^full u, u) evaluated as
  2^{-d} sum_s (A_N(s) u_s, u_s)_{R^{d x N}}, u_s the values of u at the
  shifted points (the quadratic form in the proof of Lemma reduce_grid).

Reading: omega_M = exp(2 pi i / M) and the DFT conventions of `grids`
(values = sum_k omega^{+m k} uhat(k)); grid point j of the N-grid is x = j / N
and index (2 j - s) mod 2N of the double grid is the point (2 j - s) / (2N).
"""

from __future__ import annotations

import itertools

import numpy as np

from . import ga, grids, material


def shifts(d):
    """The 2^d shift vectors s in {0,1}^d."""
    return [np.array(s) for s in itertools.product((0, 1), repeat=d)]


def shifted_matrices(mat, N, which="A"):
    """{tuple(s): A_N(s)}: the double-grid material of eq. MBA_GA on 2N points
    per axis, restricted to the points (2r - s) / (2N), r in Z_N (entry format
    of material.double_grid_matrix)."""
    N = tuple(int(n) for n in N)
    d = len(N)
    A2 = material.double_grid_matrix(mat, N, tuple(2 * n for n in N), which)
    out = {}
    for s in shifts(d):
        idx = np.ix_(*[np.mod(2 * np.arange(N[a]) - s[a], 2 * N[a]) for a in range(d)])
        out[tuple(s)] = {key: (None if v is None else np.ascontiguousarray(v[idx])) for key, v in A2.items()}
    return out


def _phase(N, s):
    """S(s): omega_{2N}^{-s.m} on the Fourier array of shape N."""
    k = grids.freq_grid(N)
    return np.exp(-1j * np.pi * sum(s[a] * k[a] / N[a] for a in range(len(N))))


def apply_full_hat(AS, xh, N):
    """Ahat^full x = 2^{-d} sum_s S*(s) F_N A_N(s) F_N^{-1} S(s) x (eq. Afull_decomp_Fourier)."""
    d = len(N)
    axes = tuple(range(1, d + 1))
    y = np.zeros_like(xh, dtype=complex)
    for s in shifts(d):
        ph = _phase(N, s)
        z = grids.idft(xh * ph[None], axes=axes)
        z = material.apply_pointwise(AS[tuple(s)], z)
        y += np.conj(ph)[None] * grids.dft(z, axes=axes)
    return y / 2.0 ** d


def matvec_hat(AS, xh, N, kind):
    """Algorithm 3: y = Ghat_{N,N} Ahat^full x on Fourier coefficients (d, *N)."""
    return ga.project_hat(apply_full_hat(AS, xh, N), N, kind)


def matvec(AS, u, N, kind):
    """Algorithm 3 on the values of a trigonometric polynomial on the N-grid."""
    axes = tuple(range(1, u.ndim))
    return np.real(grids.idft(matvec_hat(AS, grids.dft(u, axes=axes), N, kind), axes=axes))


def energy(AS, E, e, N):
    """(Ahat^full (E + e), E + e): 2^{-d} sum_s (A_N(s) u_s, u_s) with u_s the
    values of E + e at the shifted points (2r - s) / (2N)."""
    d = len(N)
    axes = tuple(range(1, d + 1))
    f = e + np.asarray(E, float)[(...,) + (None,) * d]
    fh = grids.dft(f, axes=axes)
    tot = 0.0
    for s in shifts(d):
        us = np.real(grids.idft(fh * _phase(N, s)[None], axes=axes))
        tot += ga.inner(material.apply_pointwise(AS[tuple(s)], us), us)
    return tot / 2.0 ** d


def solve(AS, N, E, kind, tol=1e-10, maxit=10_000):
    """Minimiser of eq. Ga_linsys_R for one E (primal 'E' with A) or J (dual 'J'
    with B), as N-grid values, by CG from zero."""
    d = len(N)
    Ef = np.asarray(E, float)[(...,) + (None,) * d] * np.ones((d,) + tuple(N))
    b = -matvec(AS, Ef, N, kind)
    load = np.real(grids.idft(apply_full_hat(AS, grids.dft(Ef, axes=tuple(range(1, d + 1))), N),
                              axes=tuple(range(1, d + 1))))
    floor = ga.RESIDUAL_FLOOR * np.sqrt(ga.inner(load, load))
    e, info = ga.cg(lambda p: matvec(AS, p, N, kind), b, tol, maxit, abs_stop=floor)
    e = np.real(grids.idft(ga.project_hat(grids.dft(e, axes=tuple(range(1, d + 1))), N, kind),
                           axes=tuple(range(1, d + 1))))
    return e, info


def gram(AS, fields, N):
    """Energy Gram matrix (Ahat^full (E_a + e_a), E_b + e_b) for E_a = e_a
    (polarisation of the quadratic form)."""
    d = len(fields)
    out = np.zeros((d, d))
    for a in range(d):
        Ea = np.eye(d)[a]
        out[a, a] = energy(AS, Ea, fields[a], N)
    for a in range(d):
        for b in range(a + 1, d):
            Ea, Eb = np.eye(d)[a], np.eye(d)[b]
            both = energy(AS, Ea + Eb, fields[a] + fields[b], N)
            out[a, b] = out[b, a] = 0.5 * (both - out[a, a] - out[b, b])
    return out


def reduced_bounds(mat, N, tol=1e-10, maxit=10_000):
    """Guaranteed bounds of Prop. struct_bounds from the reduced Ga."""
    N = tuple(int(n) for n in N)
    d = len(N)
    out = {"N": N, "iters_primal": [], "iters_dual": [], "fields_primal": [], "fields_dual": []}
    for kind, which in (("E", "A"), ("J", "B")):
        AS = shifted_matrices(mat, N, which)
        key = "primal" if kind == "E" else "dual"
        fields = []
        for a in range(d):
            e, info = solve(AS, N, np.eye(d)[a], kind, tol, maxit)
            fields.append(e)
            out["iters_" + key].append(info["iters"])
            out["fields_" + key].append(e)
        out["gram_A" if kind == "E" else "gram_B"] = gram(AS, fields, N)
    out["upper"] = out["gram_A"]
    out["lower"] = np.linalg.inv(out["gram_B"])
    return out
