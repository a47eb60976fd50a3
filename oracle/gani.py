"""GaNi -- Galerkin approximation with numerical integration -- and its
a-posteriori guaranteed bounds.  TEST INFRASTRUCTURE ONLY: used by tests/ and
the bench's CPU leg, never by the product path.

Follows, in order:
* eq. approx_bilin and Remark FD_GaNi -- the rectangle rule on the grid of the
  approximation order N: (A u, v) ~ (1/|N|) sum_k A(x_N^k) u(x_N^k) . v(x_N^k),
  with A sampled at the grid points x_N^k = k/N (not a Fourier series);
* Def. GaNi -- A~_{H,N} E.E = min over E_N of that quadratic form (dual: A^{-1}
  over J_N), whose minimisers solve eq. GaNi_linsys, G_N A~_N e = -G_N A~_N E,
  by CG with the operator of Algorithm 1 (transforms of size N);
* Remark duality_gani -- for odd N, B~_{H,N}^{-1} = A~_{H,N};
* eq. GaNi_apost -- A~_{H,N}^bound E.E = (A (E + e~), E + e~)_{L^2}: the exact
  energy of the GaNi minimiser, a guaranteed upper bound (dual: lower bound
  after inversion), here evaluated with the double-grid quadrature of Lemma
  integ_eval_VM on M = 2N - 1 after carrying the field to that grid.

Readings where the paper is silent: grid point k is x = k/N (mod 1, centred);
a point on an inclusion boundary is outside (strict inequality); voxel p
covers [p/P - 1/(2P), p/P + 1/(2P)) (odd N and P never put a grid point on a
voxel face).
"""

from __future__ import annotations

import numpy as np

from . import ga, grids, material


def _periodic(dx):
    """Minimum-image difference in the unit cell."""
    return dx - np.round(dx)


def sample(micro, N, which="A"):
    """A(x_N^k) (which 'A') or A^{-1}(x_N^k) ('B') on the N-grid, in the entry
    format of material.double_grid_matrix ({(a, b): array of shape N or None})."""
    d = int(micro["d"])
    x = grids.grid_points(N)
    if micro["kind"] == "voxels":
        P = tuple(int(p) for p in micro["P"])
        img = np.asarray(micro["image"], float)
        idx = tuple(np.mod(np.rint(x[a] * P[a]).astype(int), P[a]) for a in range(d))
        val = img[idx]
        if which == "B":
            val = 1.0 / val
        out = {}
        for a in range(d):
            for b in range(d):
                out[(a, b)] = val.copy() if a == b else None
        return out
    A0 = np.asarray(micro["A0"], float)
    field = np.zeros((d, d) + tuple(N))
    inside_any = np.zeros(tuple(N), dtype=bool)
    for i, shape in enumerate(micro["shapes"]):
        c = np.asarray(micro["centers"][i], float)
        h = np.asarray(micro["sizes"][i], float)
        dx = np.array([_periodic(x[a] - c[a]) for a in range(d)])
        if shape == "rect":
            ins = np.all(np.abs(dx) < 0.5 * h.reshape((d,) + (1,) * d), axis=0)
        elif shape == "circ":
            ins = np.sum(dx * dx, axis=0) < h[0] ** 2
        else:
            raise ValueError(shape)
        Ain = np.asarray(micro["A_in"][i], float)
        val = Ain if which == "A" else np.linalg.inv(Ain)
        field[:, :, ins] = val[:, :, None]
        inside_any |= ins
    base = A0 if which == "A" else np.linalg.inv(A0)
    field[:, :, ~inside_any] = base[:, :, None]
    out = {}
    for a in range(d):
        for b in range(d):
            v = field[a, b]
            out[(a, b)] = None if not np.any(v) else np.ascontiguousarray(v)
    return out


def solve(AN, N, E, kind, tol=1e-10, maxit=10_000):
    """GaNi minimiser for E (primal, kind 'E', with A~) or J (dual, 'J', with
    the sampled A^{-1}): eq. GaNi_linsys by CG on the N-grid (Algorithm 1)."""
    return ga.solve(AN, N, E, kind, tol, maxit)


def gani(micro, N, tol=1e-10, maxit=10_000):
    """A~_{H,N}, B~_{H,N} (Def. GaNi) and the minimisers of all 2d solves."""
    N = tuple(int(n) for n in N)
    d = len(N)
    out = {"N": N, "fields_primal": [], "fields_dual": [], "iters_primal": [], "iters_dual": []}
    for kind, which in (("E", "A"), ("J", "B")):
        AN = sample(micro, N, which)
        key = "primal" if kind == "E" else "dual"
        for a in range(d):
            E = np.eye(d)[a]
            e, info = solve(AN, N, E, kind, tol, maxit)
            out["fields_" + key].append(e)
            out["iters_" + key].append(info["iters"])
        g = ga.gram(AN, out["fields_" + key])
        out["A_gani" if kind == "E" else "B_gani"] = 0.5 * (g + g.T)
    return out


def apost_bounds(micro, res):
    """eq. GaNi_apost: exact energies of the GaNi minimisers (double grid
    M = 2N - 1, Lemma integ_eval_VM) -> upper A~^bound, lower (B~^bound)^{-1}."""
    N = res["N"]
    M = tuple(2 * n - 1 for n in N)
    mat = material.make_material(micro)
    out = {}
    for kind, which, key in (("E", "A", "primal"), ("J", "B", "dual")):
        AM = material.double_grid_matrix(mat, N, M, which)
        fields = [ga.prolong(e, N, M) for e in res["fields_" + key]]
        g = ga.gram(AM, fields)
        out[which] = 0.5 * (g + g.T)
    return {"upper": out["A"], "lower": np.linalg.inv(out["B"]), "A_bound": out["A"], "B_bound": out["B"]}
