"""Index sets, grid points and DFT conventions (Sec. 3.1 and Sec. 4.1).

Storage convention.  A grid function on M points per axis is an array of
shape ``M`` whose entry ``j`` (per axis) is the value at the grid point
x_M^m = m/M with m = j (mod M); the cell is periodic, so this is the same
point set as the centred Z_M of eq. grid_points.  A Fourier array of shape
``M`` stores the coefficient of frequency k at index k mod M.
"""

from __future__ import annotations

import numpy as np
import scipy.fft

# threads of the library FFT (scipy.fft workers); set_workers changes it
_WORKERS = 1


def set_workers(n):
    """Threads the FFT steps may use (the arithmetic is the same for any n)."""
    global _WORKERS
    _WORKERS = max(1, int(n))


def wrapped_freqs(M):
    """Integer frequencies k in Z_M (eq. index_set: -M/2 <= k < M/2), by storage index."""
    M = int(M)
    j = np.arange(M)
    return np.where(j < (M + 1) // 2, j, j - M)


def freq_grid(M):
    """Arrays (k_1, ..., k_d) of integer frequencies on the Fourier array of shape M."""
    axes = [wrapped_freqs(m) for m in M]
    return np.array(np.meshgrid(*axes, indexing="ij"))


def in_Z(k, N):
    """Mask of frequencies belonging to Z_N for odd N (eq. N_odd, eq. index_set)."""
    m = np.ones(k.shape[1:], dtype=bool)
    for a, n in enumerate(N):
        m &= np.abs(k[a]) <= (n - 1) // 2
    return m


def grid_points(M):
    """Coordinates x_M^m = m/M (eq. grid_points) by storage index, shape (d, *M)."""
    axes = [wrapped_freqs(m) / m for m in M]
    return np.array(np.meshgrid(*axes, indexing="ij"))


def dft(u, axes=None):
    """F_M of eq. DFT: (1/|M|) sum_m omega_M^{-mk} u(m), over the given axes."""
    axes = tuple(range(u.ndim)) if axes is None else tuple(axes)
    size = np.prod([u.shape[a] for a in axes])
    return scipy.fft.fftn(u, axes=axes, workers=_WORKERS) / size


def idft(uh, axes=None):
    """F_M^{-1} of eq. DFT: sum_k omega_M^{mk} uh(k), over the given axes."""
    axes = tuple(range(uh.ndim)) if axes is None else tuple(axes)
    size = np.prod([uh.shape[a] for a in axes])
    return scipy.fft.ifftn(uh, axes=axes, workers=_WORKERS) * size


def naive_dft(u, sign):
    """Direct evaluation of sum_m exp(sign * 2 pi i m.k / M) u(m) over all axes.

    Brute force (one dense DFT matrix per axis, no FFT) for small M; used to pin
    the FFT-based ``dft``/``idft`` conventions.
    """
    out = np.asarray(u, dtype=complex)
    for ax in range(out.ndim):
        M = out.shape[ax]
        m = np.arange(M)
        W = np.exp(sign * 2j * np.pi * np.outer(m, m) / M)
        out = np.moveaxis(np.tensordot(W, np.moveaxis(out, ax, 0), axes=(1, 0)), 0, ax)
    return out


def smooth_grid(n_min):
    """Smallest odd 3,5,7-smooth integer >= n_min (Lemma integ_eval_VM allows any M >= 2N-1)."""
    m = max(1, int(n_min))
    while True:
        if m % 2 == 1:
            x = m
            for p in (3, 5, 7):
                while x % p == 0:
                    x //= p
            if x == 1:
                return m
        m += 1
