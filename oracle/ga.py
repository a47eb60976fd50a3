"""The Ga scheme on the double grid: projections, Algorithm 2, CG, bounds.

Follows, in order:
* Def. projection and Def. discrete_proj -- Ghat^E(k) = k (x) k / (k.k),
  Ghat^J(k) = I - k (x) k / (k.k) for k in Z_N \\ {0}; zero at k = 0 and on
  Z_M \\ Z_N; G_{N,M} = F_M^{-1} Ghat F_M.  (Algorithm 2 prints |k| in the
  denominator; Def. projection fixes k.k, which is what is used.)
* Cor. Ga_linsys, eq. Ga_linsys_orig -- G A_M e = -G A_M E (primal, with
  Ghat^E and A_M) and G B_M j = -G B_M J (dual, with Ghat^J and B_M), M = 2N-1
  or any M >= 2N-1 (Lemma integ_eval_VM).
* Algorithm 2 -- y = A_M x; y = F_M y; y = Ghat y; y = F_M^{-1} y.
* Remark CG -- conjugate gradients (Saad, Alg. 6.18) from e_0 = 0, in the inner
  product (u, v)_{R^{d x M}} = (1/|M|) sum_k u^k . v^k of Sec. 4.1.
* Sec. 6.4 -- bounds during the CG iterations, and a coarse-grid solution
  carried to a finer grid (Fourier zero padding) as the initial approximation.
* Def. Ga and Prop. struct_bounds -- A_{H,N} E.E is the exact energy
  (A(E + e), E + e)_{L^2}, which Lemma integ_eval_VM evaluates exactly as
  (A_M (E + e), E + e)_{R^{d x M}}; upper bound A_{H,N}, lower bound B_{H,N}^{-1}.

Readings where the paper is silent: stopping on the relative residual
||r_k|| / ||b|| <= tol (b = r_0 from e_0 = 0; the same absolute target when
CG starts from a coarse-grid field), or once ||r_k|| <= floor * ||A_M E|| (floor = 1e-14:
a right-hand side at the rounding level of the load, as for a laminate loaded
along its layers, is treated as zero instead of being iterated on); the d x d matrix is the
energy Gram matrix of the d solutions for E = e_1..e_d, symmetrised; the
converged field is re-projected with G in FP64 before the quadrature.
"""

from __future__ import annotations

import numpy as np

from . import grids, material


def project_hat(yh, N, kind):
    """Apply Ghat^E (kind 'E') or Ghat^J (kind 'J') of Def. discrete_proj to yh (d, *M)."""
    M = yh.shape[1:]
    k = grids.freq_grid(M).astype(float)
    mask = grids.in_Z(k.astype(int), N)
    mask &= np.any(k != 0, axis=0)
    k2 = np.sum(k * k, axis=0)
    k2 = np.where(mask, k2, 1.0)
    kdoty = np.sum(k * yh, axis=0)
    grad_part = k * (kdoty / k2)[None]
    if kind == "E":
        out = grad_part
    elif kind == "J":
        out = yh - grad_part
    else:
        raise ValueError(kind)
    return np.where(mask[None], out, 0.0)


def project(x, N, kind):
    """G_{N,M} x = F_M^{-1} Ghat F_M x for a real field x of shape (d, *M)."""
    axes = tuple(range(1, x.ndim))
    xh = grids.dft(x, axes=axes)
    return np.real(grids.idft(project_hat(xh, N, kind), axes=axes))


def matvec(AM, x, N, kind):
    """Algorithm 2: y = G_{N,M} A_M x."""
    return project(material.apply_pointwise(AM, x), N, kind)


def inner(u, v):
    """(u, v)_{R^{d x M}} = (1/|M|) sum_k u^k . v^k (Sec. 4.1)."""
    return float(np.sum(u * v)) / float(np.prod(u.shape[1:]))


def energy(AM, E, e):
    """(A_M (E + e), E + e)_{R^{d x M}}: the exact energy of Lemma integ_eval_VM."""
    f = e + np.asarray(E, float)[(...,) + (None,) * (e.ndim - 1)]
    return inner(material.apply_pointwise(AM, f), f)


def cg(apply, b, tol, maxit, monitor=None, abs_stop=0.0, x0=None):
    """Conjugate gradients (Remark CG; Saad Alg. 6.18) from x_0 = 0, or from an
    initial approximation x0 in the minimisation space (Sec. 6.4).

    Stops when ||r_k|| <= tol ||b|| (= tol ||r_0|| from x_0 = 0) or ||r_k|| <=
    abs_stop.  Returns (x, info) with info = {"iters", "rel_res",
    "res_history", "alphas", "rr"}: alphas[k] is the step of iteration k + 1 and
    rr[k] = (r_k, r_k); ``monitor`` is called with the iterate after every step
    (and with x_0 before the first).
    """
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = np.array(x0, dtype=float, copy=True)
        r = b - apply(x)
    rr = inner(r, r)
    rr0 = inner(b, b)
    hist = [float(np.sqrt(rr / rr0)) if rr0 > 0 else 0.0]
    alphas, rrs = [], [rr]
    if monitor is not None:
        monitor(x)
    if rr0 == 0.0 or rr == 0.0 or np.sqrt(rr) <= abs_stop or np.sqrt(rr / rr0) <= tol:
        return x, {"iters": 0, "rel_res": hist[0], "res_history": hist, "alphas": alphas, "rr": rrs}
    p = r.copy()
    it = 0
    while it < maxit and np.sqrt(rr / rr0) > tol and np.sqrt(rr) > abs_stop:
        q = apply(p)
        alpha = rr / inner(p, q)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = inner(r, r)
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
        it += 1
        alphas.append(float(alpha))
        rrs.append(float(rr))
        hist.append(float(np.sqrt(rr / rr0)))
        if monitor is not None:
            monitor(x)
    return x, {"iters": it, "rel_res": float(np.sqrt(rr / rr0)), "res_history": hist, "alphas": alphas, "rr": rrs}


def prolong(e, N_coarse, M):
    """Prolongation I_N o I_M^{-1} of Sec. 6.4: the trigonometric polynomial of
    order N_coarse sampled on its own grid (shape (d, *M_coarse)) is sampled on
    the grid M -- the Fourier coefficients of Z_{N_coarse} are carried over (DFT
    on the coarse grid, zero padding, inverse DFT on M).  No approximation is
    made when every M_a > N_coarse_a."""
    Mc = e.shape[1:]
    axes = tuple(range(1, e.ndim))
    eh = grids.dft(e, axes=axes)
    kc = grids.freq_grid(Mc)
    keep = grids.in_Z(kc, N_coarse)
    out = np.zeros((e.shape[0],) + tuple(M), dtype=complex)
    idx = tuple(np.mod(kc[a][keep], M[a]) for a in range(len(M)))
    for c in range(e.shape[0]):
        out[c][idx] = eh[c][keep]
    return np.real(grids.idft(out, axes=axes))


RESIDUAL_FLOOR = 1e-14


def solve(AM, N, E, kind, tol=1e-10, maxit=10_000, track_energy=False, x0=None):
    """Minimiser of Def. Ga for one macroscopic E (primal, kind 'E') or J (dual, 'J').

    Solves G A_M e = -G A_M E by CG (Cor. Ga_linsys) from 0 or from the
    admissible field x0, then re-projects e with G.
    """
    M = next(a for a in AM.values() if a is not None).shape
    d = len(M)
    Ef = np.asarray(E, float)[(...,) + (None,) * d] * np.ones((d,) + M)
    load = material.apply_pointwise(AM, Ef)
    b = -project(load, N, kind)
    floor = RESIDUAL_FLOOR * np.sqrt(inner(load, load))
    energies = []
    mon = (lambda x: energies.append(energy(AM, E, x))) if track_energy else None
    e, info = cg(lambda p: matvec(AM, p, N, kind), b, tol, maxit, mon, abs_stop=floor, x0=x0)
    e = project(e, N, kind)
    info["energies"] = energies
    return e, info


def gram(AM, fields):
    """Energy Gram matrix (A_M (E_a + e_a), E_b + e_b)_{R^{d x M}} for E_a = e_a."""
    d = len(fields)
    out = np.zeros((d, d))
    for a in range(d):
        fa = fields[a].copy()
        fa[a] += 1.0
        ya = material.apply_pointwise(AM, fa)
        for b in range(d):
            fb = fields[b].copy()
            fb[b] += 1.0
            out[a, b] = inner(ya, fb)
    return out


def ga_bounds(mat, N, M=None, tol=1e-10, maxit=10_000, track_energy=False, warm=None):
    """Guaranteed bounds of Prop. struct_bounds from the Ga scheme (Def. Ga).

    Returns a dict with ``upper`` = A_{H,N}, ``lower`` = B_{H,N}^{-1}, the
    unsymmetrised Gram matrices, the CG iteration counts, the fields, the CG
    scalars and (optionally) the per-iteration energies of each primal/dual
    solve.  ``warm`` (the result of a coarser ga_bounds) starts every solve
    from the prolongation of the coarse field (Sec. 6.4).
    """
    N = tuple(int(n) for n in N)
    d = len(N)
    M = tuple(2 * n - 1 for n in N) if M is None else tuple(int(m) for m in M)
    out = {"N": N, "M": M, "iters_primal": [], "iters_dual": [],
           "energies_primal": [], "energies_dual": [], "fields_primal": [], "fields_dual": [],
           "cg_primal": [], "cg_dual": []}
    for kind, which in (("E", "A"), ("J", "B")):
        AM = material.double_grid_matrix(mat, N, M, which)
        fields = []
        key = "primal" if kind == "E" else "dual"
        for a in range(d):
            E = np.zeros(d)
            E[a] = 1.0
            x0 = None
            if warm is not None:
                x0 = prolong(warm["fields_" + key][a], warm["N"], M)
            e, info = solve(AM, N, E, kind, tol, maxit, track_energy, x0=x0)
            fields.append(e)
            out["iters_" + key].append(info["iters"])
            out["energies_" + key].append(info["energies"])
            out["fields_" + key].append(e)
            out["cg_" + key].append({"alphas": info["alphas"], "rr": info["rr"]})
        g = gram(AM, fields)
        if kind == "E":
            out["gram_A"] = g
        else:
            out["gram_B"] = g
    out["upper"] = 0.5 * (out["gram_A"] + out["gram_A"].T)
    out["B_HN"] = 0.5 * (out["gram_B"] + out["gram_B"].T)
    out["lower"] = np.linalg.inv(out["B_HN"])
    out["gap"] = float(np.trace(out["upper"] - out["lower"]) / 2.0)  # eq. error
    return out


def voigt_reuss(mat, d):
    """Voigt bound <A> = Ahat(0) and Reuss bound <A^{-1}>^{-1} = Bhat(0)^{-1}."""
    k0 = np.zeros((d, 1), dtype=int)
    voigt = np.real(mat.coeff_A(k0)[:, :, 0])
    reuss = np.linalg.inv(np.real(mat.coeff_B(k0)[:, :, 0]))
    return voigt, reuss
