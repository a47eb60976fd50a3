"""Seeded microstructure descriptors for the periodic unit cell (-1/2, 1/2)^d.

A microstructure is a plain dict, the common currency of the oracle and of
the GPU binding:

``{"d": d, "kind": "inclusions", "A0": (d,d),
   "shapes": ["rect"|"circ", ...], "centers": (n,d), "sizes": (n,d), "A_in": (n,d,d)}``
    Matrix phase ``A0`` with non-overlapping inclusions.  ``sizes`` holds the
    side lengths ``h`` of a rectangle/box, or ``(r, 0, ...)`` for a circle.
    ``A_in`` is the absolute conductivity inside each inclusion (not an
    increment over ``A0``).

``{"d": d, "kind": "voxels", "P": (P_1..P_d), "image": array of shape P}``
    Piecewise-constant isotropic image: voxel ``p`` (stored at index ``p mod P``)
    is centred at ``p / P`` and has scalar conductivity ``image[p]``; an image of
    shape ``P + (d, d)`` holds a symmetric positive definite matrix per voxel.

All randomness comes from ``numpy.random.Generator(PCG64(seed))``.
"""

from __future__ import annotations

import math

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def square_inclusion(d, side, a_matrix, a_incl, center=None):
    """Centred square (d=2) or cube (d=3) of edge ``side`` with isotropic phases."""
    c = np.zeros(d) if center is None else np.asarray(center, float)
    return {
        "d": d,
        "kind": "inclusions",
        "A0": a_matrix * np.eye(d),
        "shapes": ["rect"],
        "centers": c.reshape(1, d),
        "sizes": np.full((1, d), float(side)),
        "A_in": (a_incl * np.eye(d)).reshape(1, d, d),
    }


def circle_inclusion_vf(vf, a_matrix, a_incl, center=None):
    """Centred disc in 2D with volume fraction ``vf`` (radius sqrt(vf/pi))."""
    r = math.sqrt(vf / math.pi)
    c = np.zeros(2) if center is None else np.asarray(center, float)
    return {
        "d": 2,
        "kind": "inclusions",
        "A0": a_matrix * np.eye(2),
        "shapes": ["circ"],
        "centers": c.reshape(1, 2),
        "sizes": np.array([[r, 0.0]]),
        "A_in": (a_incl * np.eye(2)).reshape(1, 2, 2),
    }


def random_spd(seed, d=3, log10_lo=1.0, log10_hi=3.0):
    """Q diag(lambda) Q^T with lambda = 10**U(lo, hi) and Q Haar-distributed (det +1)."""
    rng = _rng(seed)
    lam = 10.0 ** rng.uniform(log10_lo, log10_hi, size=d)
    g = rng.standard_normal((d, d))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    a = q @ np.diag(lam) @ q.T
    return 0.5 * (a + a.T)


def cube_inclusion_aniso(side, seed, d=3):
    """Centred cube of edge ``side``; isotropic matrix 1, anisotropic SPD inclusion."""
    a_in = random_spd(seed, d)
    return {
        "d": d,
        "kind": "inclusions",
        "A0": np.eye(d),
        "shapes": ["rect"],
        "centers": np.zeros((1, d)),
        "sizes": np.full((1, d), float(side)),
        "A_in": a_in.reshape(1, d, d),
    }


def polycrystal(seed, P, d=3, n_grains=12, log10_lo=0.0, log10_hi=2.0):
    """Voxel image of anisotropic grains: a periodic Voronoi tessellation.

    ``n_grains`` seed points uniform in the cell; voxel p (centre p / P) belongs
    to the seed nearest under the periodic minimum image (ties to the lower
    seed index).  Each grain has its own conductivity Q diag(lambda) Q^T
    (``random_spd`` with sub-seeds: eigenvalues 10**U(lo, hi), Q Haar).
    Returns a voxel descriptor whose image has shape P + (d, d).
    """
    P = tuple(int(p) for p in (P if np.iterable(P) else (P,) * d))
    ss = np.random.SeedSequence(seed)
    subs = ss.spawn(n_grains + 1)
    rng = np.random.Generator(np.random.PCG64(subs[0]))
    seeds = rng.uniform(-0.5, 0.5, size=(n_grains, d))
    mats = np.array([random_spd(int(subs[g + 1].generate_state(1)[0]), d, log10_lo, log10_hi)
                     for g in range(n_grains)])
    axes = [np.where(np.arange(p) < (p + 1) // 2, np.arange(p), np.arange(p) - p) / p for p in P]
    x = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1)  # voxel centres, shape P + (d,)
    best = np.full(P, np.inf)
    grain = np.zeros(P, dtype=int)
    for g in range(n_grains):
        dd = x - seeds[g]
        dd -= np.round(dd)
        dist = np.sum(dd * dd, axis=-1)
        closer = dist < best
        best = np.where(closer, dist, best)
        grain = np.where(closer, g, grain)
    return {"d": d, "kind": "voxels", "P": P, "image": mats[grain]}


def multiphase_aniso(seed, d=3, n=3, log10_lo=0.0, log10_hi=2.0):
    """Non-overlapping boxes (placed on a lattice of cell positions), each with
    its own anisotropic SPD conductivity, in an anisotropic SPD matrix phase:
    eq. inclcomp with a different A_i per inclusion."""
    ss = np.random.SeedSequence(seed)
    subs = ss.spawn(n + 2)
    rng = np.random.Generator(np.random.PCG64(subs[0]))
    # n boxes of side 0.3 in distinct cells of a 3^d lattice of spacing 1/3
    cells = rng.permutation(3 ** d)[:n]
    centers = np.array([[((c // 3 ** a) % 3) / 3.0 - 1.0 / 3.0 for a in range(d)] for c in cells])
    centers += rng.uniform(-0.01, 0.01, size=centers.shape)
    sizes = rng.uniform(0.2, 0.3, size=(n, d))
    A0 = random_spd(int(subs[1].generate_state(1)[0]), d, 0.0, 0.5)
    A_in = np.array([random_spd(int(subs[i + 2].generate_state(1)[0]), d, log10_lo, log10_hi) for i in range(n)])
    return {"d": d, "kind": "inclusions", "A0": A0, "shapes": ["rect"] * n, "centers": centers, "sizes": sizes,
            "A_in": A_in}


def _min_image_dist(a, b):
    dd = a - b
    dd -= np.round(dd)
    return float(np.sqrt(np.sum(dd * dd)))


def random_circles(seed, k_lo=5, k_hi=50, r_lo=0.02, r_hi=0.08, contrast=None,
                   max_tries=10_000):
    """k non-overlapping discs (periodic minimum-image test), placed largest first.

    Radii ~ U[r_lo, r_hi], count ~ U{k_lo..k_hi}, isotropic contrast
    ~ logU[10, 1e4] unless given (matrix 1).  A placement that fails after
    ``max_tries`` draws per disc restarts from the next sub-seed.
    """
    ss = np.random.SeedSequence(seed)
    for sub in ss.spawn(64):
        rng = np.random.Generator(np.random.PCG64(sub))
        k = int(rng.integers(k_lo, k_hi + 1))
        radii = np.sort(rng.uniform(r_lo, r_hi, size=k))[::-1]
        c = contrast if contrast is not None else 10.0 ** rng.uniform(1.0, 4.0)
        centers = []
        ok = True
        for r in radii:
            placed = False
            for _ in range(max_tries):
                x = rng.uniform(-0.5, 0.5, size=2)
                if all(_min_image_dist(x, y) >= r + ry for y, ry in zip(centers, radii)):
                    centers.append(x)
                    placed = True
                    break
            if not placed:
                ok = False
                break
        if ok:
            n = len(radii)
            sizes = np.zeros((n, 2))
            sizes[:, 0] = radii
            return {
                "d": 2,
                "kind": "inclusions",
                "A0": np.eye(2),
                "shapes": ["circ"] * n,
                "centers": np.array(centers),
                "sizes": sizes,
                "A_in": np.repeat((c * np.eye(2))[None], n, axis=0),
            }
    raise RuntimeError("random_circles: no admissible placement")


def grf_voxels(seed, P, d=3, corr_len=0.05, vf=0.4, a_matrix=1.0, a_incl=100.0):
    """Two-phase voxel image from a thresholded Gaussian random field.

    White noise on the P^d grid is filtered in Fourier space by
    exp(-pi^2 l^2 |k|^2) (Gaussian covariance exp(-r^2 / (2 l^2)) on the unit
    cell); the top ``vf`` fraction of voxels (ties broken by linear index) is
    the inclusion phase, so the volume fraction is exact.
    """
    P = tuple(int(p) for p in (P if np.iterable(P) else (P,) * d))
    rng = _rng(seed)
    w = rng.standard_normal(P)
    freqs = np.meshgrid(*[np.fft.fftfreq(p, 1.0 / p) for p in P], indexing="ij")
    k2 = sum(f * f for f in freqs)
    field = np.real(np.fft.ifftn(np.fft.fftn(w) * np.exp(-(math.pi * corr_len) ** 2 * k2)))
    flat = field.ravel()
    n_in = int(round(vf * flat.size))
    order = np.argsort(-flat, kind="stable")
    img = np.full(flat.size, float(a_matrix))
    img[order[:n_in]] = float(a_incl)
    return {"d": d, "kind": "voxels", "P": P, "image": img.reshape(P)}


def grf_request(seed, N, d=3):
    """A 3D random-field request: voxel image on the doubled grid 2N-1."""
    P = 2 * N - 1
    return grf_voxels(seed, (P,) * d, d=d)


def serving_requests(seed, n, rate_per_s, N_choices=(41, 63, 123, 365)):
    """A stream of 2D random-circle requests with Poisson arrivals.

    Returns a list of dicts ``{"id", "arrival_s", "N", "micro"}``; each request
    draws its own sub-seed from SeedSequence(seed).
    """
    ss = np.random.SeedSequence(seed)
    subs = ss.spawn(n + 1)
    rng = np.random.Generator(np.random.PCG64(subs[0]))
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n):
        r = np.random.Generator(np.random.PCG64(subs[i + 1]))
        N = int(N_choices[int(r.integers(0, len(N_choices)))])
        micro_seed = int(r.integers(0, 2**62))
        out.append({"id": i, "arrival_s": float(t[i]), "N": N,
                    "micro": random_circles(micro_seed)})
    return out


def poisson_arrivals(seed, n, rate_per_s):
    """n Poisson arrival times (the first at t = 0) at ``rate_per_s``."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    return np.cumsum(gaps) - gaps[0]


def serving_requests_3d(seed, n, rate_per_s, N_choices=(41, 63, 113), corr_len=0.05, vf=0.4, contrast=100.0):
    """A stream of 3D random-field requests with Poisson arrivals.

    Each request is a two-phase voxel image on the doubled grid (2N - 1)^3 of
    its own order N (drawn from ``N_choices``): a Gaussian random field of
    correlation length ``corr_len`` thresholded at volume fraction ``vf``,
    phases 1 and ``contrast``.  Returns dicts ``{"id", "arrival_s", "N",
    "micro"}`` like :func:`serving_requests`.
    """
    ss = np.random.SeedSequence(seed)
    subs = ss.spawn(n + 1)
    t = poisson_arrivals(int(subs[0].generate_state(1)[0]), n, rate_per_s)
    out = []
    for i in range(n):
        r = np.random.Generator(np.random.PCG64(subs[i + 1]))
        N = int(N_choices[int(r.integers(0, len(N_choices)))])
        micro = grf_voxels(int(r.integers(0, 2**62)), (2 * N - 1,) * 3, d=3, corr_len=corr_len, vf=vf,
                           a_matrix=1.0, a_incl=contrast)
        out.append({"id": i, "arrival_s": float(t[i]), "N": N, "micro": micro})
    return out


def with_arrivals(requests, seed, rate_per_s):
    """The same requests (shared microstructures) with new Poisson arrival times."""
    t = poisson_arrivals(seed, len(requests), rate_per_s)
    return [dict(r, arrival_s=float(t[i])) for i, r in enumerate(requests)]
